"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/kmg.h declares, sizes workspaces, and rejects invalid
arguments before touching a device."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kmg.h")


@pytest.fixture(scope="module")
def kmg():
    from paper_2409_15615_amd import kmg as k

    try:
        k.load()
    except (ImportError, OSError) as e:
        pytest.skip(f"libkmg.so not loadable here: {e}")
    return k


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kmg_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("kmg_voxelize", "kmg_normals", "kmg_fpfh", "kmg_match", "kmg_workspace_bytes",
               "kmg_status_string", "kmg_version"):
        assert fn in names


def test_every_declared_symbol_is_exported(kmg):
    lib = kmg.load()
    for fn in declared_functions():
        assert hasattr(lib, fn), f"{fn} is declared in kmg.h but not exported"


def test_only_api_symbols_exported(kmg):
    import subprocess

    out = subprocess.run(["nm", "-D", "--defined-only", kmg._LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert exported and all(e.startswith("kmg_") for e in exported), exported
    assert set(exported) <= set(declared_functions())


def test_status_strings(kmg):
    lib = kmg.load()
    assert lib.kmg_status_string(0) == b"ok"
    assert b"capacity" in lib.kmg_status_string(-2)
    assert lib.kmg_status_string(123) == b"unknown status"
    assert lib.kmg_version() >= 10000


def test_workspace_sizes(kmg):
    p = kmg.make_params(0.3, 0.9, 1.5)
    sizes = {op: kmg.workspace_bytes(op, 20000, 20000, p) for op in range(4)}
    assert all(v > 0 for v in sizes.values())
    assert kmg.workspace_bytes(0, 40000) > sizes[0]
    assert kmg.workspace_bytes(3, 40000, 20000, p) > sizes[3]
    assert kmg.workspace_bytes(9, 10, 10, p) == 0
    assert kmg.workspace_bytes(0, -1) == 0


def _p(**kw):
    from paper_2409_15615_amd import kmg as k

    base = dict(voxel=0.3, r_normal=0.9, r_fpfh=1.5)
    base.update(kw)
    return k.make_params(**base)


@pytest.mark.parametrize("bad", [
    dict(voxel=0.0), dict(voxel=-1.0), dict(r_normal=2.0, r_fpfh=1.5), dict(tau_num=0), dict(tau_lin=0.0),
    dict(tau_lin=1.5), dict(n_bins=0), dict(n_bins=40), dict(voxel=float("nan")),
])
def test_invalid_parameters_rejected(kmg, bad):
    """Invalid parameters return KMG_ERR_ARG without any device work (r_normal must not
    exceed r_FPFH because the normal subset is taken from the r_FPFH search)."""
    lib = kmg.load()
    p = _p(**bad)
    nnz = C.c_int64(0)
    dummy = C.c_void_p(256)  # never dereferenced: validation fails first
    st = lib.kmg_normals(dummy, 10, C.byref(p), dummy, dummy, dummy, dummy, 100, C.byref(nnz), None, dummy,
                         1 << 30, None)
    assert st == kmg.KMG_ERR_ARG
    nj = C.c_int64(0)
    st = lib.kmg_fpfh(dummy, dummy, dummy, dummy, dummy, 10, C.byref(p), None, dummy, dummy, C.byref(nj), None,
                      dummy, 1 << 30, None)
    assert st == kmg.KMG_ERR_ARG


def test_null_and_size_arguments_rejected(kmg):
    lib = kmg.load()
    m = C.c_int64(0)
    d = C.c_void_p(256)
    assert lib.kmg_voxelize(d, 10, 0.1, d, d, 10, None, d, 1 << 30, None) == kmg.KMG_ERR_ARG
    assert lib.kmg_voxelize(d, -5, 0.1, d, d, 10, C.byref(m), d, 1 << 30, None) == kmg.KMG_ERR_ARG
    assert lib.kmg_voxelize(d, 10, 0.0, d, d, 10, C.byref(m), d, 1 << 30, None) == kmg.KMG_ERR_ARG
    assert lib.kmg_voxelize(None, 10, 0.1, d, d, 10, C.byref(m), d, 1 << 30, None) == kmg.KMG_ERR_ARG
    # workspace too small is reported before any launch
    assert lib.kmg_voxelize(d, 1000, 0.1, d, d, 1000, C.byref(m), d, 16, None) == kmg.KMG_ERR_WORKSPACE
    n = C.c_int64(0)
    assert lib.kmg_match(d, None, 10, d, None, 10, 0, 0, d, d, d, 10, C.byref(n), None, d, 1 << 30,
                         None) == kmg.KMG_ERR_ARG
    assert lib.kmg_match(d, None, 10, d, None, 10, 33, 7, d, d, d, 10, C.byref(n), None, d, 1 << 30,
                         None) == kmg.KMG_ERR_ARG
    p = _p()
    assert lib.kmg_normals(d, 10, C.byref(p), d, d, None, d, 100, C.byref(n), None, d, 1 << 30,
                           None) == kmg.KMG_ERR_ARG


def test_binding_refuses_host_tensors(kmg):
    import torch

    with pytest.raises(ValueError):
        kmg.voxelize(torch.zeros(3, 10), 0.1)


def test_tuning_set_get_and_validation(kmg):
    """kmg_set_tuning / kmg_get_tuning on the host: defaults, a valid change, and
    unsupported values refused without changing the tuning."""
    kmg.set_tuning(None)
    d = kmg.get_tuning()
    assert d == {"search_waves": 4, "count_queries": 2, "spfh_pair_mean": 24, "fpfh_rows": 2, "band_tile": 0,
                 "fuse_features": 0, "xcd_split": 2, "match_form": 0, "search_form": 1}
    kmg.set_tuning({"search_waves": 8, "band_tile": 20})
    assert kmg.get_tuning()["search_waves"] == 8 and kmg.get_tuning()["band_tile"] == 20
    for bad in ({"search_waves": 3}, {"count_queries": 8}, {"fpfh_rows": 5}, {"band_tile": 65},
                {"spfh_pair_mean": -1}, {"fuse_features": 2}, {"xcd_split": 4}, {"match_form": 2},
                {"search_form": 2}):
        with pytest.raises(kmg.KmgError):
            kmg.set_tuning(bad)
    lib = kmg.load()
    t = kmg.KmgTuning()
    lib.kmg_get_tuning(C.byref(t))
    t.match_form = 7
    assert lib.kmg_set_tuning(C.byref(t)) == kmg.KMG_ERR_ARG
    kmg.set_tuning(None)
    assert kmg.get_tuning() == d
