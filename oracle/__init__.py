"""FP64 CPU oracle for the Faster-PFH + mutual-NN hot path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package.  The product path (``paper_2409_15615_amd``) never imports it, and
this package never imports the product path.
"""

from .oracle import (  # noqa: F401
    build,
    load,
    set_threads,
    voxelize,
    radius_search,
    normals,
    eig3,
    pair_features,
    spfh,
    fpfh,
    nn_rows,
    mutual_match,
    faster_pfh,
    run_pair,
)
