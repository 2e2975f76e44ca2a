"""kmg_normals_static (no workspace argument, library-owned static scratch) against
kmg_normals on the same inputs: bit-identical neighbour lists, normals, flags and
|P_normal| on two calls in a row, the second with a smaller cloud; the size limit
and the mode restriction are refused before any device work."""

import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def K():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2409_15615_amd import kmg

    kmg.load()
    torch.cuda.set_device(0)
    return kmg


def kept_cloud(K, d, key):
    p = d["params"]
    _, xyz = K.voxelize(torch.from_numpy(d[key]).cuda(), p.voxel)
    vp = d["vp_src" if key == "src" else "vp_tgt"]
    return xyz.contiguous(), K.make_params(p.voxel, p.r_normal, p.r_fpfh, p.tau_num, p.tau_lin, p.n_bins, vp)


def same(a, b):
    for f in ("normals", "flags", "off", "idx", "n_normal"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f


def test_static_equals_workspace_form_twice(K):
    big = kept_cloud(K, synth.c1_pair(0), "tgt")      # ~42.6k kept points
    small = kept_cloud(K, synth.c0_pair(0), "src")    # ~3.3k kept points
    assert big[0].shape[1] > 10 * small[0].shape[1]
    for xyz, prm in (big, small):
        ref = K.normals(xyz, prm)
        got = K.normals_static(xyz, prm)
        torch.cuda.synchronize()
        same(got, ref)
        print(f"m={xyz.shape[1]} nnz={got.idx.numel()}: equal to kmg_normals")


def test_static_capacity_and_limits(K):
    xyz, prm = kept_cloud(K, synth.c0_pair(0), "tgt")
    lib = K.load()
    m = xyz.shape[1]
    nrm = torch.empty(3 * m, dtype=torch.float32, device="cuda")
    flags = torch.empty(m, dtype=torch.uint8, device="cuda")
    off = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    idx = torch.empty(8, dtype=torch.int32, device="cuda")
    nnz = C.c_int64(0)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    args = (C.c_void_p(nrm.data_ptr()), C.c_void_p(flags.data_ptr()), C.c_void_p(off.data_ptr()),
            C.c_void_p(idx.data_ptr()))
    st = lib.kmg_normals_static(C.c_void_p(xyz.data_ptr()), m, C.byref(prm), *args, 8, C.byref(nnz), None, s)
    assert st == K.KMG_ERR_CAPACITY and nnz.value == K.normals(xyz, prm).idx.numel()
    # beyond the static limit: refused before any device work (no pointer is read)
    st = lib.kmg_normals_static(C.c_void_p(xyz.data_ptr()), K.STATIC_MAX_POINTS + 1, C.byref(prm), *args, 8,
                                C.byref(nnz), None, s)
    assert st == K.KMG_ERR_RANGE
    classic = K.make_params(prm.voxel, prm.r_normal, prm.r_fpfh, mode=K.MODE_CLASSIC_FPFH)
    st = lib.kmg_normals_static(C.c_void_p(xyz.data_ptr()), m, C.byref(classic), *args, 8, C.byref(nnz), None, s)
    assert st == K.KMG_ERR_ARG
    # a correct call after the refused ones
    ref = K.normals(xyz, prm)
    same(K.normals_static(xyz, prm), ref)
