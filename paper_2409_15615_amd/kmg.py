"""Thin Python binding of libkmg (argument marshalling only).

Every step of the hot path runs in the HIP library; this module only checks
tensor placement and dtypes, allocates outputs and workspace with torch on
the current device, and passes raw pointers and the current HIP stream to the
C ABI declared in include/kmg.h.  There is no fallback: if libkmg.so is
missing, importing the binding raises.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkmg.so")

KMG_OK = 0
KMG_ERR_ARG = -1
KMG_ERR_CAPACITY = -2
KMG_ERR_DEVICE = -3
KMG_ERR_RANGE = -4
KMG_ERR_WORKSPACE = -5

KMG_FP32, KMG_BF16, KMG_FP16 = 0, 1, 2
OP_VOXELIZE, OP_NORMALS, OP_FPFH, OP_MATCH, OP_GRAPH, OP_KCORE = 0, 1, 2, 3, 4, 5
PRECISIONS = {"fp32": KMG_FP32, "bf16": KMG_BF16, "fp16": KMG_FP16}


class KmgParams(C.Structure):
    _fields_ = [
        ("voxel", C.c_double),
        ("r_normal", C.c_double),
        ("r_fpfh", C.c_double),
        ("tau_lin", C.c_double),
        ("tau_num", C.c_int32),
        ("n_bins", C.c_int32),
        ("viewpoint", C.c_double * 3),
        ("mode", C.c_int32),
        ("reserved", C.c_int32),
    ]


MODE_FASTER_PFH, MODE_CLASSIC_FPFH = 0, 1


class KmgTuning(C.Structure):
    _fields_ = [
        ("search_waves", C.c_int32),
        ("count_queries", C.c_int32),
        ("spfh_pair_mean", C.c_int32),
        ("fpfh_rows", C.c_int32),
        ("band_tile", C.c_int32),
        ("fuse_features", C.c_int32),
        ("xcd_split", C.c_int32),
        ("match_form", C.c_int32),
        ("search_form", C.c_int32),
    ]


TUNING_FIELDS = ("search_waves", "count_queries", "spfh_pair_mean", "fpfh_rows", "band_tile", "fuse_features",
                 "xcd_split", "match_form", "search_form")


class KmgCloud(C.Structure):
    _fields_ = [("xyz", C.c_void_p), ("n", C.c_int64), ("params", KmgParams)]


class KmgMatchOut(C.Structure):
    _fields_ = [("pairs", C.c_void_p), ("d1", C.c_void_p), ("d2", C.c_void_p), ("cap", C.c_int64)]


class KmgError(RuntimeError):
    def __init__(self, fn: str, status: int, lib):
        self.status = status
        msg = lib.kmg_status_string(status).decode() if lib is not None else str(status)
        super().__init__(f"{fn} failed: {msg} ({status})")


_lib = None


def load():
    """Loads libkmg.so (built in-tree by paper_2409_15615_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libkmg.so is not built ({_LIB_PATH}); run: python -m paper_2409_15615_amd.build")
    lib = C.CDLL(_LIB_PATH)
    vp, i64, i32, dbl, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_size_t
    pp = C.POINTER(KmgParams)
    i64p = C.POINTER(C.c_int64)
    lib.kmg_version.restype = i32
    lib.kmg_status_string.argtypes = [i32]
    lib.kmg_status_string.restype = C.c_char_p
    lib.kmg_workspace_bytes.argtypes = [i32, i64, i64, pp]
    lib.kmg_workspace_bytes.restype = sz
    lib.kmg_voxelize.argtypes = [vp, i64, dbl, vp, vp, i64, i64p, vp, sz, vp]
    lib.kmg_voxelize.restype = i32
    lib.kmg_normals.argtypes = [vp, i64, pp, vp, vp, vp, vp, i64, i64p, vp, vp, sz, vp]
    lib.kmg_normals.restype = i32
    lib.kmg_normals_static.argtypes = [vp, i64, pp, vp, vp, vp, vp, i64, i64p, vp, vp]
    lib.kmg_normals_static.restype = i32
    lib.kmg_fpfh.argtypes = [vp, vp, vp, vp, vp, i64, pp, vp, vp, vp, i64p, i64p, vp, sz, vp]
    lib.kmg_fpfh.restype = i32
    lib.kmg_match.argtypes = [vp, vp, i64, vp, vp, i64, i32, i32, vp, vp, vp, i64, i64p, i64p, vp, sz, vp]
    lib.kmg_match.restype = i32
    cp, op = C.POINTER(KmgCloud), C.POINTER(KmgMatchOut)
    lib.kmg_batch_workspace_bytes.argtypes = [i32, i64, i64, i32]
    lib.kmg_batch_workspace_bytes.restype = sz
    lib.kmg_batch_upload.argtypes = [cp, op, i32, i64, i64, vp, sz, vp]
    lib.kmg_batch_upload.restype = i32
    lib.kmg_batch_run.argtypes = [i32, i64, i64, i32, i32, vp, vp, sz, vp]
    lib.kmg_batch_run.restype = i32
    lib.kmg_batch_descriptors.argtypes = [i32, i64, i64, i32, i32, vp, i64, vp, i64, vp, sz, vp]
    lib.kmg_batch_descriptors.restype = i32
    lib.kmg_register_batch.argtypes = [cp, op, i32, i64, i64, i32, vp, vp, sz, vp]
    lib.kmg_register_batch.restype = i32
    i32p = C.POINTER(C.c_int32)
    lib.kmg_corr_graph.argtypes = [vp, i64, vp, i64, vp, vp, vp, i64, i32, dbl, vp, vp, vp, i64, i32p, i64p, vp, sz,
                                   vp]
    lib.kmg_corr_graph.restype = i32
    lib.kmg_max_kcore.argtypes = [vp, vp, i32, vp, vp, i32p, i32p, vp, sz, vp]
    lib.kmg_max_kcore.restype = i32
    lib.kmg_set_tuning.argtypes = [C.POINTER(KmgTuning)]
    lib.kmg_set_tuning.restype = i32
    lib.kmg_get_tuning.argtypes = [C.POINTER(KmgTuning)]
    lib.kmg_get_tuning.restype = i32
    lib.kmg_timing_enable.argtypes = [i32]
    lib.kmg_timing_enable.restype = i32
    lib.kmg_timing_read.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int64), i32]
    lib.kmg_timing_read.restype = i32
    lib.kmg_timing_work.argtypes = [C.POINTER(C.c_int64), i32]
    lib.kmg_timing_work.restype = i32
    lib.kmg_stage_name.argtypes = [i32]
    lib.kmg_stage_name.restype = C.c_char_p
    _lib = lib
    return lib


def get_tuning() -> dict:
    """kmg_get_tuning as a dict of the tunable fields."""
    t = KmgTuning()
    _raise("kmg_get_tuning", load().kmg_get_tuning(C.byref(t)))
    return {f: int(getattr(t, f)) for f in TUNING_FIELDS}


def set_tuning(values=None):
    """kmg_set_tuning: fields not given keep their defaults; None restores all defaults."""
    lib = load()
    if values is None:
        _raise("kmg_set_tuning", lib.kmg_set_tuning(None))
        return
    _raise("kmg_set_tuning", lib.kmg_set_tuning(None))
    t = KmgTuning()
    lib.kmg_get_tuning(C.byref(t))
    for f, v in values.items():
        if f not in TUNING_FIELDS:
            raise ValueError(f"unknown tuning field {f}")
        setattr(t, f, int(v))
    _raise("kmg_set_tuning", lib.kmg_set_tuning(C.byref(t)))


def make_params(voxel, r_normal, r_fpfh, tau_num=3, tau_lin=0.99, n_bins=11, viewpoint=(0.0, 0.0, 0.0),
                mode=MODE_FASTER_PFH):
    p = KmgParams()
    p.voxel, p.r_normal, p.r_fpfh, p.tau_lin = float(voxel), float(r_normal), float(r_fpfh), float(tau_lin)
    p.tau_num, p.n_bins = int(tau_num), int(n_bins)
    p.mode, p.reserved = int(mode), 0
    for c in range(3):
        p.viewpoint[c] = float(viewpoint[c])
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _raise(fn, st):
    if st != KMG_OK:
        raise KmgError(fn, st, _lib)


class Workspace:
    """Caller-owned device scratch, grown on demand and reused across calls."""

    def __init__(self, device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.buf = torch.empty(0, dtype=torch.uint8, device=self.device)

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(int(nbytes * 1.25) + 4096, dtype=torch.uint8, device=self.device)
        return self.buf


_default_ws = {}


def _ws(ws):
    if ws is not None:
        return ws
    dev = torch.cuda.current_device()
    if dev not in _default_ws:
        _default_ws[dev] = Workspace()
    return _default_ws[dev]


def workspace_bytes(op, n0, n1=0, params=None):
    lib = load()
    return int(lib.kmg_workspace_bytes(op, int(n0), int(n1), C.byref(params) if params is not None else None))


def voxelize(xyz, voxel, ws=None):
    """kmg_voxelize.  xyz: (3, n) float32 device SoA.  Returns (kept_idx int32 [m],
    kept_xyz float32 (3, m))."""
    lib = load()
    _check_dev(xyz, torch.float32, "xyz")
    n = xyz.shape[1]
    kept_idx = torch.empty(max(n, 1), dtype=torch.int32, device=xyz.device)
    kept_xyz = torch.empty(3 * max(n, 1), dtype=torch.float32, device=xyz.device)
    w = _ws(ws).get(workspace_bytes(OP_VOXELIZE, n))
    m = C.c_int64(0)
    st = lib.kmg_voxelize(_ptr(xyz), n, float(voxel), _ptr(kept_idx), _ptr(kept_xyz), n, C.byref(m), _ptr(w),
                          w.numel(), _stream())
    _raise("kmg_voxelize", st)
    m = m.value
    return kept_idx[:m], kept_xyz[: 3 * m].view(3, m)


@dataclass
class NormalsOut:
    normals: torch.Tensor
    flags: torch.Tensor
    off: torch.Tensor
    idx: torch.Tensor
    n_normal: torch.Tensor


_nbr_cap_hint = {}


def normals(xyz, params, ws=None, want_n_normal=True):
    """kmg_normals (Algorithm 1, Step 1).  xyz: (3, m) float32 device SoA."""
    lib = load()
    _check_dev(xyz, torch.float32, "xyz")
    m = xyz.shape[1]
    dev = xyz.device
    nrm = torch.empty(3 * max(m, 1), dtype=torch.float32, device=dev)
    flags = torch.empty(max(m, 1), dtype=torch.uint8, device=dev)
    off = torch.empty(m + 1, dtype=torch.int32, device=dev)
    n_normal = torch.empty(max(m, 1), dtype=torch.int32, device=dev) if want_n_normal else None
    cap = max(_nbr_cap_hint.get(dev.index, 0), 64 * m, 1)
    for _ in range(3):  # the classic mode may need a larger capacity for each of its two searches
        # the classic mode keeps its r_normal lists in the workspace, sized like nbr_idx
        w = _ws(ws).get(workspace_bytes(OP_NORMALS, m, cap if params.mode == MODE_CLASSIC_FPFH else 0, params))
        idx = torch.empty(cap, dtype=torch.int32, device=dev)
        nnz = C.c_int64(0)
        st = lib.kmg_normals(_ptr(xyz), m, C.byref(params), _ptr(nrm), _ptr(flags), _ptr(off), _ptr(idx), cap,
                             C.byref(nnz), _ptr(n_normal), _ptr(w), w.numel(), _stream())
        if st == KMG_ERR_CAPACITY:
            cap = max(cap, int(nnz.value))
            _nbr_cap_hint[dev.index] = cap
            continue
        _raise("kmg_normals", st)
        break
    nnz = nnz.value
    return NormalsOut(nrm[: 3 * m].view(3, m), flags[:m], off, idx[:nnz],
                      n_normal[:m] if n_normal is not None else None)


STATIC_MAX_POINTS = 262144


def normals_static(xyz, params, want_n_normal=True):
    """kmg_normals_static: kmg_normals with the library's static scratch (no
    workspace; m <= STATIC_MAX_POINTS, Faster-PFH mode).  The outputs are still
    allocated here, by torch."""
    lib = load()
    _check_dev(xyz, torch.float32, "xyz")
    m = xyz.shape[1]
    dev = xyz.device
    nrm = torch.empty(3 * max(m, 1), dtype=torch.float32, device=dev)
    flags = torch.empty(max(m, 1), dtype=torch.uint8, device=dev)
    off = torch.empty(m + 1, dtype=torch.int32, device=dev)
    n_normal = torch.empty(max(m, 1), dtype=torch.int32, device=dev) if want_n_normal else None
    cap = max(_nbr_cap_hint.get(dev.index, 0), 64 * m, 1)
    for _ in range(2):
        idx = torch.empty(cap, dtype=torch.int32, device=dev)
        nnz = C.c_int64(0)
        st = lib.kmg_normals_static(_ptr(xyz), m, C.byref(params), _ptr(nrm), _ptr(flags), _ptr(off), _ptr(idx), cap,
                                    C.byref(nnz), _ptr(n_normal), _stream())
        if st == KMG_ERR_CAPACITY:
            cap = max(cap, int(nnz.value))
            continue
        _raise("kmg_normals_static", st)
        break
    nnz = nnz.value
    return NormalsOut(nrm[: 3 * m].view(3, m), flags[:m], off, idx[:nnz],
                      n_normal[:m] if n_normal is not None else None)


@dataclass
class FpfhOut:
    fpfh: torch.Tensor
    spfh: torch.Tensor
    j_idx: torch.Tensor
    flags: torch.Tensor
    stats: tuple


def fpfh(xyz, nrm, flags, off, idx, params, ws=None, want_spfh=False):
    """kmg_fpfh (Algorithm 1, Step 2; Eq. A2-A5).  `flags` is updated in place
    (bit 1 = J)."""
    lib = load()
    for t, nm, dt in ((xyz, "xyz", torch.float32), (nrm, "normals", torch.float32), (flags, "flags", torch.uint8),
                      (off, "off", torch.int32), (idx, "idx", torch.int32)):
        _check_dev(t, dt, nm)
    m = xyz.shape[1]
    D = 3 * params.n_bins
    dev = xyz.device
    out = torch.empty((max(m, 1), D), dtype=torch.float32, device=dev)
    sp = torch.empty((max(m, 1), D), dtype=torch.float32, device=dev) if want_spfh else None
    j_idx = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    idx_arg = idx if idx.numel() else torch.empty(1, dtype=torch.int32, device=dev)
    # the classic mode runs a third search: its lists need as many entries as idx
    w = _ws(ws).get(workspace_bytes(OP_FPFH, m, idx.numel() if params.mode == MODE_CLASSIC_FPFH else 0, params))
    nj = C.c_int64(0)
    stats = (C.c_int64 * 2)()
    st = lib.kmg_fpfh(_ptr(xyz), _ptr(nrm), _ptr(flags), _ptr(off), _ptr(idx_arg), m, C.byref(params), _ptr(sp),
                      _ptr(out), _ptr(j_idx), C.byref(nj), stats, _ptr(w), w.numel(), _stream())
    _raise("kmg_fpfh", st)
    return FpfhOut(out[:m], sp[:m] if sp is not None else None, j_idx[: nj.value], flags, (stats[0], stats[1]))


@dataclass
class MatchOut:
    pairs: torch.Tensor
    d1: torch.Tensor
    d2: torch.Tensor
    n_fallback: int


def match(desc_p, desc_q, rows_p=None, rows_q=None, prec="fp32", ws=None):
    """kmg_match (mutual NN).  desc_*: (n, dim) float32 device; rows_*: optional
    int32 row lists.  Returns pairs (k, 2) int32 of row ids, d1, d2."""
    lib = load()
    _check_dev(desc_p, torch.float32, "desc_p")
    _check_dev(desc_q, torch.float32, "desc_q")
    dim = desc_p.shape[1]
    if desc_q.shape[1] != dim:
        raise ValueError("descriptor lengths differ")
    for r, nm in ((rows_p, "rows_p"), (rows_q, "rows_q")):
        if r is not None:
            _check_dev(r, torch.int32, nm)
    np_ = rows_p.numel() if rows_p is not None else desc_p.shape[0]
    nq = rows_q.numel() if rows_q is not None else desc_q.shape[0]
    dev = desc_p.device
    cap = max(min(np_, nq), 1)
    pairs = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    d1 = torch.empty(cap, dtype=torch.float32, device=dev)
    d2 = torch.empty(cap, dtype=torch.float32, device=dev)
    w = _ws(ws).get(_match_ws_dim(np_, nq, dim))
    npairs = C.c_int64(0)
    nfb = C.c_int64(0)
    st = lib.kmg_match(_ptr(desc_p), _ptr(rows_p), np_, _ptr(desc_q), _ptr(rows_q), nq, dim, PRECISIONS[prec],
                       _ptr(pairs), _ptr(d1), _ptr(d2), cap, C.byref(npairs), C.byref(nfb), _ptr(w), w.numel(),
                       _stream())
    _raise("kmg_match", st)
    k = npairs.value
    return MatchOut(pairs[:k], d1[:k], d2[:k], nfb.value)


@dataclass
class GraphOut:
    sel: torch.Tensor   # (n,) int32: correspondence of each vertex
    off: torch.Tensor   # (n + 1,) int32
    adj: torch.Tensor   # (nnz,) int32, rows ascending


def corr_graph(src_xyz, tgt_xyz, pairs, d1, d2, n_tau=3000, beta=0.45, ws=None):
    """kmg_corr_graph: ratio filter to n_tau correspondences, Eq. (3) graph in CSR.
    src_xyz/tgt_xyz: (3, m) float32 kept clouds; pairs (k, 2) int32; d1, d2 (k,) float32."""
    lib = load()
    _check_dev(src_xyz, torch.float32, "src_xyz")
    _check_dev(tgt_xyz, torch.float32, "tgt_xyz")
    pairs = pairs.contiguous()
    k = int(pairs.shape[0])
    dev = src_xyz.device
    n_tau = int(n_tau)
    sel = torch.empty(max(n_tau, 1), dtype=torch.int32, device=dev)
    off = torch.empty(n_tau + 1, dtype=torch.int32, device=dev)
    w = _ws(ws).get(int(lib.kmg_workspace_bytes(OP_GRAPH, k, n_tau, None)))
    n_sel = C.c_int32(0)
    nnz = C.c_int64(0)
    cap = max(1, min(k, n_tau) * 64)
    for _ in range(2):
        adj = torch.empty(cap, dtype=torch.int32, device=dev)
        st = lib.kmg_corr_graph(_ptr(src_xyz), src_xyz.shape[1], _ptr(tgt_xyz), tgt_xyz.shape[1], _ptr(pairs),
                                _ptr(d1), _ptr(d2), k, n_tau, float(beta), _ptr(sel), _ptr(off), _ptr(adj), cap,
                                C.byref(n_sel), C.byref(nnz), _ptr(w), w.numel(), _stream())
        if st == KMG_ERR_CAPACITY and nnz.value > cap:
            cap = int(nnz.value)
            continue
        _raise("kmg_corr_graph", st)
        break
    n = n_sel.value
    return GraphOut(sel[:n], off[:n + 1], adj[:nnz.value])


@dataclass
class KcoreOut:
    core: torch.Tensor     # (n,) int32 core numbers
    members: torch.Tensor  # vertices of the maximum k-core, ascending
    max_core: int


def max_kcore(off, adj, n, ws=None):
    """kmg_max_kcore on a CSR graph of n vertices (device int32 tensors)."""
    lib = load()
    dev = off.device
    core = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    members = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    w = _ws(ws).get(int(lib.kmg_workspace_bytes(OP_KCORE, n, 0, None)))
    nm = C.c_int32(0)
    mx = C.c_int32(0)
    _raise("kmg_max_kcore", lib.kmg_max_kcore(_ptr(off), _ptr(adj), int(n), _ptr(core), _ptr(members), C.byref(nm),
                                              C.byref(mx), _ptr(w), w.numel(), _stream()))
    return KcoreOut(core[:n], members[:nm.value], mx.value)


def _match_ws_dim(np_, nq, dim):
    # the match workspace is sized for descriptors of length 3 * n_bins >= dim
    p = make_params(1.0, 1.0, 1.0, n_bins=(dim + 2) // 3)
    return int(load().kmg_workspace_bytes(OP_MATCH, np_, nq, C.byref(p)))


@dataclass
class CloudOut:
    kept_idx: torch.Tensor
    xyz: torch.Tensor
    normals: NormalsOut
    feats: FpfhOut


def faster_pfh(raw_xyz, params, ws=None):
    """voxelize -> normals -> fpfh for one raw cloud (3, n)."""
    kept_idx, xyz = voxelize(raw_xyz, params.voxel, ws)
    xyz = xyz.contiguous()
    nr = normals(xyz, params, ws)
    ft = fpfh(xyz, nr.normals, nr.flags, nr.off, nr.idx, params, ws)
    return CloudOut(kept_idx, xyz, nr, ft)


def register_pair(src_raw, tgt_raw, params_src, params_tgt, prec="fp32", ws=None):
    """The whole hot path for one pair: Faster-PFH on both clouds, then mutual
    matching of the J descriptors.  Pairs are kept-cloud indices."""
    a = faster_pfh(src_raw, params_src, ws)
    b = faster_pfh(tgt_raw, params_tgt, ws)
    mt = match(a.feats.fpfh, b.feats.fpfh, a.feats.j_idx, b.feats.j_idx, prec=prec, ws=ws)
    return a, b, mt


# ---------------------------------------------------------------------------
# Batched registration
# ---------------------------------------------------------------------------

COUNTS_STRIDE = 8


@dataclass
class PairResult:
    pairs: torch.Tensor
    d1: torch.Tensor
    d2: torch.Tensor
    kept: tuple
    n_j: tuple
    n_fallback: int
    status: int


class Batch:
    """A reusable batch of up to `n_pairs` registration pairs with fixed capacities.

    Owns the workspace, the per-pair output buffers and the device counts;
    `upload` writes a new cloud table (any number of pairs up to `n_pairs`;
    the workspace layout of fewer pairs fits inside that of more), `run`
    enqueues kmg_batch_run on the current stream (capturable in a graph),
    `results` reads the counts back."""

    def __init__(self, n_pairs, raw_cap, nnz_cap, n_bins=11, out_cap=None, device=None):
        lib = load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.n_pairs, self.raw_cap, self.nnz_cap, self.n_bins = int(n_pairs), int(raw_cap), int(nnz_cap), int(n_bins)
        nbytes = int(lib.kmg_batch_workspace_bytes(self.n_pairs, self.raw_cap, self.nnz_cap, self.n_bins))
        if nbytes == 0:
            raise ValueError("invalid batch capacities")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.out_cap = int(out_cap) if out_cap is not None else max(1, self.raw_cap // 2)
        self.pairs = torch.empty((self.n_pairs, self.out_cap, 2), dtype=torch.int32, device=self.device)
        self.d1 = torch.empty((self.n_pairs, self.out_cap), dtype=torch.float32, device=self.device)
        self.d2 = torch.empty((self.n_pairs, self.out_cap), dtype=torch.float32, device=self.device)
        self.counts = torch.zeros((self.n_pairs, COUNTS_STRIDE), dtype=torch.int64, device=self.device)
        self.n_active = self.n_pairs
        self._keep = []

    def upload(self, clouds):
        """clouds: list of 2 * n_pairs (xyz (3, n) float32 device tensor, KmgParams)."""
        lib = load()
        if len(clouds) % 2 or not 0 < len(clouds) // 2 <= self.n_pairs:
            raise ValueError(f"need two clouds per pair and 1..{self.n_pairs} pairs")
        n_active = len(clouds) // 2
        ct = (KmgCloud * len(clouds))()
        total = 0
        for k, (xyz, prm) in enumerate(clouds):
            _check_dev(xyz, torch.float32, "xyz")
            ct[k].xyz = xyz.data_ptr()
            ct[k].n = xyz.shape[1]
            ct[k].params = prm
            total += xyz.shape[1]
        if total > self.raw_cap:
            raise ValueError(f"batch has {total} raw points, capacity {self.raw_cap}")
        ot = (KmgMatchOut * n_active)()
        for i in range(n_active):
            ot[i].pairs = self.pairs[i].data_ptr()
            ot[i].d1 = self.d1[i].data_ptr()
            ot[i].d2 = self.d2[i].data_ptr()
            ot[i].cap = self.out_cap
        self._keep = list(clouds)
        _raise("kmg_batch_upload", lib.kmg_batch_upload(ct, ot, n_active, self.raw_cap, self.nnz_cap,
                                                        _ptr(self.ws), self.ws.numel(), _stream()))
        self.n_active = n_active

    def run(self, prec="fp32"):
        lib = load()
        _raise("kmg_batch_run", lib.kmg_batch_run(self.n_active, self.raw_cap, self.nnz_cap, self.n_bins,
                                                  PRECISIONS[prec], _ptr(self.counts), _ptr(self.ws),
                                                  self.ws.numel(), _stream()))

    def results(self):
        """Reads the counts (synchronises the current stream) -> list of PairResult."""
        cnt = self.counts.cpu().numpy()
        out = []
        for i in range(self.n_active):
            k = int(min(cnt[i, 0], self.out_cap))
            out.append(PairResult(self.pairs[i, :k], self.d1[i, :k], self.d2[i, :k],
                                  (int(cnt[i, 1]), int(cnt[i, 2])), (int(cnt[i, 3]), int(cnt[i, 4])),
                                  int(cnt[i, 5]), int(cnt[i, 6])))
        return out

    def nnz(self):
        return int(self.counts[0, 7].item())

    def descriptors(self, cloud, n_kept, n_j):
        """kmg_batch_descriptors: cloud `cloud`'s kept-space FPFH rows (n_kept, 3H) and
        its J list (own kept indices), copied out of the workspace on the current stream."""
        lib = load()
        D = 3 * self.n_bins
        fp = torch.empty((max(n_kept, 1), D), dtype=torch.float32, device=self.device)
        jj = torch.empty(max(n_j, 1), dtype=torch.int32, device=self.device)
        _raise("kmg_batch_descriptors", lib.kmg_batch_descriptors(
            self.n_active, self.raw_cap, self.nnz_cap, self.n_bins, int(cloud), _ptr(fp), int(n_kept), _ptr(jj),
            int(n_j), _ptr(self.ws), self.ws.numel(), _stream()))
        return fp[:n_kept], jj[:n_j]


def register_batch(clouds, prec="fp32", nnz_per_point=48, out_cap=None):
    """Runs the batched hot path once.  clouds: list of (xyz (3, n) device float32,
    KmgParams), two per pair (source, target).  Grows the neighbour capacity and
    retries once if the batch needs more.  Returns (list of PairResult, Batch)."""
    n_pairs = len(clouds) // 2
    raw = sum(int(x.shape[1]) for x, _ in clouds)
    H = clouds[0][1].n_bins
    nnz_cap = max(1024, nnz_per_point * raw)
    for _ in range(2):
        b = Batch(n_pairs, raw, nnz_cap, H, out_cap=out_cap)
        b.upload(clouds)
        b.run(prec)
        res = b.results()
        if all(r.status != KMG_ERR_WORKSPACE for r in res):
            return res, b
        nnz_cap = b.nnz() + 1024
    raise KmgError("kmg_register_batch", KMG_ERR_WORKSPACE, _lib)
