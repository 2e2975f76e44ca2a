"""Ratio filter + Eq. (3) graph (kmg_corr_graph) and maximum k-core
(kmg_max_kcore) on the GPU against the oracle, bit-exact.

The correspondence sets fed to both sides come from the oracle's own
end-to-end run (or from seeded synthetic sets), never from the HIP path.
"""

import itertools

import numpy as np
import pytest

import synth
from oracle import pose

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def csr_of(adj):
    deg = adj.sum(1)
    off = np.zeros(adj.shape[0] + 1, np.int32)
    off[1:] = np.cumsum(deg)
    idx = np.nonzero(adj)[1].astype(np.int32)  # row-major: rows ascending, columns ascending
    return off, idx


def oracle_graph(src_kept, tgt_kept, pairs, d1, d2, n_tau, beta):
    sel = pose.ratio_filter(d1, d2, n_tau)
    p = pairs[sel]
    a = src_kept.T[p[:, 0]].astype(np.float64)
    b = tgt_kept.T[p[:, 1]].astype(np.float64)
    return sel, pose.compat_graph(a, b, beta)


def check_graph(K, src_kept, tgt_kept, pairs, d1, d2, n_tau, beta):
    sel, adj = oracle_graph(src_kept, tgt_kept, pairs, d1, d2, n_tau, beta)
    g = K.corr_graph(dev(src_kept), dev(tgt_kept), dev(pairs.astype(np.int32)), dev(d1), dev(d2), n_tau, beta)
    np.testing.assert_array_equal(g.sel.cpu().numpy(), sel)
    off, idx = csr_of(adj)
    np.testing.assert_array_equal(g.off.cpu().numpy(), off)
    np.testing.assert_array_equal(g.adj.cpu().numpy(), idx)
    return g, adj


@pytest.mark.parametrize("which", ["planes+spheres", "lidar"])
def test_graph_and_kcore_equal_oracle_on_oracle_correspondences(K, orc, which):
    d = synth.c0_pair(0) if which == "planes+spheres" else synth.c1_pair(0)
    p = d["params"]
    ref = orc.run_pair(d["src"], d["tgt"], p, d["vp_src"], d["vp_tgt"])
    src_kept = np.ascontiguousarray(ref["src"]["xyz"], np.float32)
    tgt_kept = np.ascontiguousarray(ref["tgt"]["xyz"], np.float32)
    pairs = np.asarray(ref["pairs"], np.int32)
    d1 = ref["d1"].astype(np.float32)
    d2 = ref["d2"].astype(np.float32)
    beta = 1.5 * p.voxel
    for n_tau in (3000, 500):
        g, adj = check_graph(K, src_kept, tgt_kept, pairs, d1, d2, n_tau, beta)
        n = adj.shape[0]
        kc = K.max_kcore(g.off, g.adj, n)
        core = pose.core_numbers(adj)
        np.testing.assert_array_equal(kc.core.cpu().numpy(), core)
        assert kc.max_core == core.max()
        np.testing.assert_array_equal(kc.members.cpu().numpy(), pose.max_kcore(adj))
        print(f"{which} n_tau={n_tau}: {n} vertices, {int(adj.sum())} edges, max core {kc.max_core} "
              f"({kc.members.numel()} members)")


def test_graph_edge_cases(K):
    rng = np.random.default_rng(5)
    m = 500
    src = rng.uniform(-20, 20, (3, m)).astype(np.float32)
    tgt = rng.uniform(-20, 20, (3, m)).astype(np.float32)
    k = 900
    pairs = np.stack([rng.integers(0, m, k), rng.integers(0, m, k)], 1).astype(np.int32)
    d2 = rng.uniform(0.5, 2.0, k).astype(np.float32)
    d1 = (d2 * rng.uniform(0.1, 1.0, k)).astype(np.float32)
    d1[100:200] = d1[7]  # tied ratios
    d2[100:200] = d2[7]
    d1[300], d2[300] = 0.0, 0.0
    d1[301], d2[301] = 0.4, 0.0
    for n_tau in (1, 64, 899, 900, 4000):
        check_graph(K, src, tgt, pairs, d1, d2, n_tau, 0.6)
    # no correspondences
    g = K.corr_graph(dev(src), dev(tgt), torch.zeros((0, 2), dtype=torch.int32, device="cuda"),
                     torch.zeros(0, device="cuda"), torch.zeros(0, device="cuda"), 3000, 0.6)
    assert g.sel.numel() == 0 and g.adj.numel() == 0 and g.off.cpu().tolist() == [0]


def test_dense_graph_of_a_rigid_copy(K):
    rng = np.random.default_rng(6)
    m = 2000
    src = rng.uniform(-5, 5, (3, m)).astype(np.float32)
    R = synth.random_rotation(rng)
    tgt = (R @ src.astype(np.float64) + 1.0).astype(np.float32)
    perm = rng.permutation(m)
    pairs = np.stack([perm, perm], 1).astype(np.int32)
    d1 = rng.uniform(0.1, 1.0, m).astype(np.float32)
    d2 = np.full(m, 2.0, np.float32)
    g, adj = check_graph(K, src, tgt, pairs, d1, d2, 3000, 0.05)
    assert adj.sum() == m * (m - 1)  # float32 rounding stays far below 2 beta
    kc = K.max_kcore(g.off, g.adj, m)
    assert kc.max_core == m - 1 and kc.members.numel() == m


@pytest.mark.parametrize("name,n,edges", [
    ("K5", 5, list(itertools.combinations(range(5), 2))),
    ("star", 6, [(0, i) for i in range(1, 6)]),
    ("cycle", 7, [(i, (i + 1) % 7) for i in range(7)]),
    ("K4+K3+isolated", 8, list(itertools.combinations(range(4), 2)) + list(itertools.combinations(range(4, 7), 2))),
    ("no edges", 3, []),
])
def test_kcore_closed_cases(K, name, n, edges):
    adj = np.zeros((n, n), bool)
    for u, v in edges:
        adj[u, v] = adj[v, u] = True
    off, idx = csr_of(adj)
    kc = K.max_kcore(dev(off), dev(idx if idx.size else np.zeros(1, np.int32)), n)
    np.testing.assert_array_equal(kc.core.cpu().numpy(), pose.core_numbers(adj))
    np.testing.assert_array_equal(kc.members.cpu().numpy(), pose.max_kcore(adj))


@pytest.mark.parametrize("seed", range(6))
def test_kcore_random_graphs(K, seed):
    rng = np.random.default_rng(20 + seed)
    n = [300, 1000, 3000, 8192, 12000, 16384][seed]
    p = [0.3, 0.05, 0.01, 0.002, 0.004, 0.001][seed]
    upper = np.triu(rng.random((n, n)) < p, 1)
    adj = upper | upper.T
    off, idx = csr_of(adj)
    kc = K.max_kcore(dev(off), dev(idx), n)
    np.testing.assert_array_equal(kc.core.cpu().numpy(), pose.core_numbers(adj))


def test_kcore_slow_convergence_falls_back_to_peel(K):
    """A long path with shuffled labels: the h-index sweeps lower one step of the path per
    sweep, so they do not converge within their budget and the block peel decides."""
    rng = np.random.default_rng(31)
    n = 4000
    order = rng.permutation(n)
    path, clique = order[:-20], order[-20:]
    adj = np.zeros((n, n), bool)
    adj[path[:-1], path[1:]] = True
    # a clique apart from the path, so that the maximum core is not the path
    adj[np.ix_(clique, clique)] = True
    adj[clique, clique] = False
    adj |= adj.T
    off, idx = csr_of(adj)
    kc = K.max_kcore(dev(off), dev(idx), n)
    np.testing.assert_array_equal(kc.core.cpu().numpy(), pose.core_numbers(adj))
    np.testing.assert_array_equal(kc.members.cpu().numpy(), pose.max_kcore(adj))
