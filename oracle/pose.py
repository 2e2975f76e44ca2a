"""Host-side registration back end used as TEST SUPPORT for the oracle pins.

Implements, in plain numpy, the steps downstream of matching so that an
end-to-end pin (exact recovery of a known transform) can be checked:
  ratio_filter   -- keep the N_tau correspondences with the lowest d1/d2
                    (Section III-D, last paragraph)
  compat_graph   -- pairwise-invariant edges of Eq. (3) with bound beta
  max_kcore      -- vertices of the maximum k-core (Section III-D)
  gnc_tls        -- graduated non-convexity with a truncated least squares
                    loss (Section III-E), weighted closed-form rotation
"""

from __future__ import annotations

import numpy as np


def ratio_filter(d1, d2, n_tau: int = 3000):
    """Indices of the n_tau correspondences with the smallest d1/d2 (stable)."""
    d1 = np.asarray(d1, np.float64)
    d2 = np.asarray(d2, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(d2 > 0, d1 / d2, np.where(d1 > 0, np.inf, 0.0))
    order = np.argsort(ratio, kind="stable")
    return order[:n_tau]


def _pair_norms(p):
    """||p_u - p_v|| for all u, v, summed as (dx dx + dy dy) + dz dz in FP64."""
    d = p[:, None, :] - p[None, :, :]
    return np.sqrt((d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2])


def compat_graph(a, b, beta: float):
    """Adjacency (boolean, no self loops) of Eq. (3):
    | ||b_j - b_j'|| - ||a_i - a_i'|| | <= 2 beta.  a, b are (k, 3)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    adj = np.abs(_pair_norms(b) - _pair_norms(a)) <= 2.0 * beta
    np.fill_diagonal(adj, False)
    return adj


def core_numbers(adj):
    """Core number of every vertex by repeated removal of a minimum-degree vertex."""
    n = adj.shape[0]
    deg = adj.sum(axis=1).astype(np.int64)
    alive = np.ones(n, bool)
    core = np.zeros(n, np.int64)
    k = 0
    for _ in range(n):
        cand = np.where(alive, deg, np.iinfo(np.int64).max)
        v = int(np.argmin(cand))
        k = max(k, int(deg[v]))
        core[v] = k
        alive[v] = False
        nb = np.nonzero(adj[v] & alive)[0]
        deg[nb] -= 1
    return core


def max_kcore(adj):
    """Vertices whose core number equals the maximum."""
    if adj.shape[0] == 0:
        return np.zeros(0, np.int64)
    core = core_numbers(adj)
    return np.nonzero(core == core.max())[0]


def weighted_rigid(a, b, w):
    """argmin_{R, t} sum w_i ||b_i - R a_i - t||^2 (closed form via SVD)."""
    w = np.asarray(w, np.float64)
    sw = w.sum()
    ca = (w[:, None] * a).sum(0) / sw
    cb = (w[:, None] * b).sum(0) / sw
    H = ((a - ca) * w[:, None]).T @ (b - cb)
    U, _, Vt = np.linalg.svd(H)
    S = np.eye(3)
    S[2, 2] = np.sign(np.linalg.det(Vt.T @ U.T))
    R = Vt.T @ S @ U.T
    return R, cb - R @ ca


def gnc_tls(a, b, noise_bound: float, max_iters: int = 100, mu_step: float = 1.4):
    """GNC with the TLS loss: returns (R, t, inlier mask)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    k = a.shape[0]
    w = np.ones(k)
    c2 = noise_bound * noise_bound
    R, t = weighted_rigid(a, b, w)
    r2 = ((b - a @ R.T - t) ** 2).sum(1)
    if r2.max() <= c2:
        return R, t, np.ones(k, bool)
    mu = c2 / max(2.0 * r2.max() - c2, 1e-30)
    for _ in range(max_iters):
        hi = (mu + 1.0) / mu * c2
        lo = mu / (mu + 1.0) * c2
        w = np.where(r2 >= hi, 0.0, np.where(r2 <= lo, 1.0, noise_bound * np.sqrt(mu * (mu + 1.0) / np.maximum(r2, 1e-300)) - mu))
        if w.sum() < 3:
            break
        R, t = weighted_rigid(a, b, w)
        r2 = ((b - a @ R.T - t) ** 2).sum(1)
        if np.all((w == 0.0) | (w == 1.0)) and mu > 1e6:
            break
        mu *= mu_step
    inl = r2 <= c2
    if inl.sum() >= 3:
        R, t = weighted_rigid(a[inl], b[inl], np.ones(int(inl.sum())))
    return R, t, inl


def register(src_xyz, tgt_xyz, pairs, d1, d2, voxel: float, n_tau: int = 3000):
    """Ratio filter -> Eq. (3) graph -> max k-core -> GNC-TLS.  src_xyz/tgt_xyz are
    (3, m) arrays, pairs (k, 2) kept-cloud indices.  Returns (R, t, n_inliers)."""
    beta = 1.5 * voxel
    sel = ratio_filter(d1, d2, n_tau)
    p = np.asarray(pairs)[sel]
    a = np.asarray(src_xyz, np.float64).T[p[:, 0]]
    b = np.asarray(tgt_xyz, np.float64).T[p[:, 1]]
    core = max_kcore(compat_graph(a, b, beta))
    R, t, inl = gnc_tls(a[core], b[core], beta)
    return R, t, int(inl.sum())
