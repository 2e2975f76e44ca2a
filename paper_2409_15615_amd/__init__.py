"""MI355X-native Faster-PFH and mutual-NN matching (KISS-Matcher hot path).

The compute path is the HIP library libkmg.so (C ABI in include/kmg.h);
``paper_2409_15615_amd.kmg`` is its Python binding.  Build the library with
``python -m paper_2409_15615_amd.build``.
"""
