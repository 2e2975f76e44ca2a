"""ctypes binding and chaining for the plain-C FP64 oracle (``kmg_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.

Each wrapper follows one step of the paper's method:
  voxelize      -- voxelized input clouds of size v (Section III-A)
  radius_search -- Eq. A1 (strict <, the query included)
  normals       -- Algorithm 1, Step 1 (cardinality and linearity filters, PCA)
  spfh          -- Algorithm 1, Step 2 plus Eq. A2-A4
  fpfh          -- Eq. A5
  mutual_match  -- the reciprocity test of Section III-C on squared L2 distances
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc -O2 -ffp-contract=off -fopenmp."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
             "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = C.CDLL(_LIB)
    lib.orc_set_threads.argtypes = [C.c_int]
    lib.orc_set_threads.restype = C.c_int
    lib.orc_voxelize.argtypes = [_f32p, C.c_int64, C.c_double, _i32p, C.c_void_p]
    lib.orc_voxelize.restype = C.c_int64
    lib.orc_radius_count.argtypes = [_f32p, C.c_int64, C.c_double, _i32p]
    lib.orc_radius_count.restype = C.c_int64
    lib.orc_radius_fill.argtypes = [_f32p, C.c_int64, C.c_double, _i64p, _i32p]
    lib.orc_radius_fill.restype = None
    lib.orc_radius_count_grid.argtypes = [_f32p, C.c_int64, C.c_double, _i32p]
    lib.orc_radius_count_grid.restype = C.c_int64
    lib.orc_radius_fill_grid.argtypes = [_f32p, C.c_int64, C.c_double, _i64p, _i32p]
    lib.orc_radius_fill_grid.restype = None
    lib.orc_normals.argtypes = [_f32p, C.c_int64, _i64p, _i32p, C.c_double, C.c_int32, C.c_double, _f64p,
                                _f64p, _f64p, _f64p, _i32p, _u8p]
    lib.orc_normals.restype = None
    lib.orc_eig3_sorted.argtypes = [_f64p, _f64p, _f64p]
    lib.orc_eig3_sorted.restype = None
    lib.orc_pair_features.argtypes = [_f64p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_pair_features.restype = None
    lib.orc_bin.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int, C.POINTER(C.c_int)]
    lib.orc_bin.restype = C.c_int
    lib.orc_spfh.argtypes = [_f32p, _f64p, C.c_int64, _i64p, _i32p, _u8p, C.c_int32, C.c_int32, _i32p, _f64p,
                             _i32p, _u8p]
    lib.orc_spfh.restype = C.c_int64
    lib.orc_fpfh.argtypes = [_f32p, C.c_int64, _i64p, _i32p, _u8p, _u8p, _f64p, _i32p, C.c_int32, _f64p]
    lib.orc_fpfh.restype = None
    lib.orc_nn_rows.argtypes = [_f32p, _f32p, C.c_int64, C.c_int, _i64p, C.c_int64, _i32p, _f64p, _f64p]
    lib.orc_nn_rows.restype = None
    _lib = lib
    return lib


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (0 keeps the default); returns the count in use."""
    return int(load().orc_set_threads(int(n)))


def _soa(xyz) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float32))
    assert a.ndim == 2 and a.shape[0] == 3, "points are SoA float32 of shape (3, n)"
    return a


def voxelize(xyz, v: float):
    """Lowest-index representative of every occupied voxel (keys floor(x / v) in FP64).
    Returns (kept int32 ascending, keys int64 (3, m))."""
    xyz = _soa(xyz)
    n = xyz.shape[1]
    kept = np.empty(max(n, 1), np.int32)
    keys = np.empty((3, max(n, 1)), np.int64)
    m = load().orc_voxelize(xyz, n, float(v), kept, keys.ctypes.data)
    # keys were written as a 3 x m block at the start of the buffer
    flat = keys.reshape(-1)[: 3 * m].reshape(3, m).copy()
    return kept[:m].copy(), flat


def radius_search(xyz, r: float, grid: bool = False):
    """Eq. A1 for every point: CSR (off int64[m+1], idx int32[nnz]), lists ascending.
    grid=True takes the candidates from a uniform grid of cell size r instead of
    all points (same sets; for clouds too large for the O(m^2) brute force)."""
    xyz = _soa(xyz)
    m = xyz.shape[1]
    lib = load()
    count, fill = (lib.orc_radius_count_grid, lib.orc_radius_fill_grid) if grid else \
        (lib.orc_radius_count, lib.orc_radius_fill)
    cnt = np.empty(max(m, 1), np.int32)
    total = count(xyz, m, float(r), cnt)
    off = np.zeros(m + 1, np.int64)
    off[1:] = np.cumsum(cnt[:m])
    idx = np.empty(max(int(total), 1), np.int32)
    fill(xyz, m, float(r), off, idx)
    return off, idx[: int(total)].copy()


def normals(xyz, off, idx, r_normal: float, tau_num: int, tau_lin: float, vp):
    """Algorithm 1, Step 1.  Returns dict(normals (3, m) f64, plin, gap, n_normal, B)."""
    xyz = _soa(xyz)
    m = xyz.shape[1]
    out = dict(
        normals=np.zeros((3, m), np.float64),
        plin=np.zeros(m, np.float64),
        gap=np.zeros(m, np.float64),
        n_normal=np.zeros(m, np.int32),
        B=np.zeros(m, np.uint8),
    )
    if m == 0:
        return out
    idx = np.ascontiguousarray(idx, np.int32) if len(idx) else np.zeros(1, np.int32)
    load().orc_normals(xyz, m, np.ascontiguousarray(off, np.int64), idx, float(r_normal), int(tau_num),
                       float(tau_lin), np.ascontiguousarray(vp, np.float64), out["normals"], out["plin"],
                       out["gap"], out["n_normal"], out["B"])
    return out


def eig3(Cm):
    """Sorted (descending) eigen-pairs of a symmetric 3x3 matrix via cyclic Jacobi.
    Returns (lam[3], vec[3, 3]) with vec[i] the eigenvector of lam[i]."""
    lam = np.zeros(3)
    vec = np.zeros(9)
    load().orc_eig3_sorted(np.ascontiguousarray(Cm, np.float64).reshape(9), lam, vec)
    return lam, vec.reshape(3, 3)


def pair_features(pq, nq, pk, nk):
    """Eq. A2 features (f1, f2, f3) for the pair (q, k)."""
    f = np.zeros(3)
    load().orc_pair_features(*(np.ascontiguousarray(a, np.float64) for a in (pq, nq, pk, nk)), f)
    return f


def spfh(xyz, normals64, off, idx, B, tau_num: int, H: int = 11):
    """Algorithm 1, Step 2 and Eq. A2-A4.  Returns dict(counts (m, 3H) int32,
    spfh (m, 3H) f64, Pq int32, J uint8, edges)."""
    xyz = _soa(xyz)
    m = xyz.shape[1]
    D = 3 * H
    out = dict(counts=np.zeros((m, D), np.int32), spfh=np.zeros((m, D)), Pq=np.zeros(m, np.int32),
               J=np.zeros(m, np.uint8), edges=0)
    if m == 0:
        return out
    idx = np.ascontiguousarray(idx, np.int32) if len(idx) else np.zeros(1, np.int32)
    out["edges"] = int(load().orc_spfh(xyz, np.ascontiguousarray(normals64, np.float64), m,
                                       np.ascontiguousarray(off, np.int64), idx,
                                       np.ascontiguousarray(B, np.uint8), int(tau_num), int(H), out["counts"],
                                       out["spfh"], out["Pq"], out["J"]))
    return out


def fpfh(xyz, off, idx, B, J, spfh64, Pq, H: int = 11):
    """Eq. A5 for q in J (rows outside J are zero).  Returns (m, 3H) f64."""
    assert H <= 64
    xyz = _soa(xyz)
    m = xyz.shape[1]
    out = np.zeros((m, 3 * H))
    if m == 0:
        return out
    idx = np.ascontiguousarray(idx, np.int32) if len(idx) else np.zeros(1, np.int32)
    load().orc_fpfh(xyz, m, np.ascontiguousarray(off, np.int64), idx, np.ascontiguousarray(B, np.uint8),
                    np.ascontiguousarray(J, np.uint8), np.ascontiguousarray(spfh64, np.float64),
                    np.ascontiguousarray(Pq, np.int32), int(H), out)
    return out


def nn_rows(X, Y, rows=None):
    """Nearest row of Y for each selected row of X under squared L2 in FP64
    (dimension order, ties to the smaller index).  Returns (nn, best, second)."""
    X = np.ascontiguousarray(X, np.float32)
    Y = np.ascontiguousarray(Y, np.float32)
    dim = X.shape[1] if X.ndim == 2 and X.shape[0] else (Y.shape[1] if Y.ndim == 2 else 0)
    rows = np.arange(X.shape[0], dtype=np.int64) if rows is None else np.ascontiguousarray(rows, np.int64)
    nr = rows.size
    nn = np.full(max(nr, 1), -1, np.int32)
    best = np.full(max(nr, 1), np.inf)
    second = np.full(max(nr, 1), np.inf)
    if nr and X.shape[0]:
        Yc = Y if Y.shape[0] else np.zeros((1, dim), np.float32)
        load().orc_nn_rows(X, Yc, Y.shape[0], dim, rows, nr, nn, best, second)
    return nn[:nr], best[:nr], second[:nr]


def mutual_match(X, Y):
    """Reciprocity test: (i, j) is kept iff j = NN_Y(i) and i = NN_X(j).
    Returns dict(pairs (k, 2) int32 sorted by i, d1, d2 (sqrt of best / second
    squared distance of row i), nn_xy, nn_yx)."""
    nn_xy, b_xy, s_xy = nn_rows(X, Y)
    nn_yx, _, _ = nn_rows(Y, X)
    i = np.arange(nn_xy.size)
    ok = nn_xy >= 0
    ok[ok] = nn_yx[nn_xy[ok]] == i[ok]
    pairs = np.stack([i[ok], nn_xy[ok]], axis=1).astype(np.int32)
    return dict(pairs=pairs, d1=np.sqrt(b_xy[ok]), d2=np.sqrt(s_xy[ok]), nn_xy=nn_xy, nn_yx=nn_yx,
                best_xy=b_xy, second_xy=s_xy)


def faster_pfh(xyz_kept, params, vp, boundary_fp32: bool = True, classical: bool = False, grid: bool = False):
    """Algorithm 1 and Eq. A1-A5 on one voxelized cloud.

    With boundary_fp32 the chain rounds the normals to float32 before the
    histogram step, because the library's interface stores normals as a
    float32 array between the two calls.

    classical=True gives the FPFH that Section III-C contrasts with
    Faster-PFH (Fig. 3a): normals from the r_normal neighbourhood of every
    point with at least 3 points there, no linearity filter, SPFH and FPFH
    for every point with a normal.  The r_normal neighbourhood is the strict
    r_normal subset of the r_FPFH list, which is exactly what a separate
    radius search at r_normal returns."""
    H = int(params.n_bins)
    tau_normal, tau_lin, tau_j = (3, 1.0, 1) if classical else (params.tau_num, params.tau_lin, params.tau_num)
    off, idx = radius_search(xyz_kept, params.r_fpfh, grid=grid)
    nr = normals(xyz_kept, off, idx, params.r_normal, tau_normal, tau_lin, vp)
    n64 = nr["normals"].astype(np.float32).astype(np.float64) if boundary_fp32 else nr["normals"]
    sp = spfh(xyz_kept, n64, off, idx, nr["B"], tau_j, H)
    fp = fpfh(xyz_kept, off, idx, nr["B"], sp["J"], sp["spfh"], sp["Pq"], H)
    j_idx = np.nonzero(sp["J"])[0].astype(np.int32)
    return dict(off=off, idx=idx, normals=nr["normals"], normals_used=n64, plin=nr["plin"], gap=nr["gap"],
                n_normal=nr["n_normal"], B=nr["B"], counts=sp["counts"], spfh=sp["spfh"], Pq=sp["Pq"], J=sp["J"],
                edges=sp["edges"], fpfh=fp, j_idx=j_idx)


def run_pair(src_raw, tgt_raw, params, vp_src, vp_tgt, match: bool = True, classical: bool = False,
             grid: bool = False):
    """Whole hot path for one pair: voxelize both clouds, Faster-PFH on both, then
    mutual matching of the float32 descriptors of the J points.  Correspondences
    are returned as kept-cloud indices (i in the source, j in the target)."""
    out = {}
    for tag, raw, vp in (("src", src_raw, vp_src), ("tgt", tgt_raw, vp_tgt)):
        kept, keys = voxelize(raw, params.voxel)
        xyz = np.ascontiguousarray(_soa(raw)[:, kept])
        fp = faster_pfh(xyz, params, vp, classical=classical, grid=grid)
        fp.update(kept=kept, keys=keys, xyz=xyz)
        out[tag] = fp
    if match:
        X = out["src"]["fpfh"][out["src"]["j_idx"]].astype(np.float32)
        Y = out["tgt"]["fpfh"][out["tgt"]["j_idx"]].astype(np.float32)
        mm = mutual_match(X, Y)
        pairs = mm["pairs"]
        out["pairs"] = np.stack([out["src"]["j_idx"][pairs[:, 0]], out["tgt"]["j_idx"][pairs[:, 1]]], 1) \
            if len(pairs) else np.zeros((0, 2), np.int32)
        out["d1"], out["d2"] = mm["d1"], mm["d2"]
    return out
