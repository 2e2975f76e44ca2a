"""Norm-band pruning of the FP64 matching form on the GPU against the oracle.

The band skips partner rows whose norm differs from the query's by more than
R (R^2 = the second smallest exact distance to the 64 partner rows nearest in
norm), which cannot change the exact mutual nearest neighbours.  These cases
stress the pruning: norms all equal (nothing can be skipped), norms spread
over decades (almost everything is skipped), partners of one row (no seed
bound), exact duplicates (R = 0), clusters of equal norms at chunk edges, and
both orientations of the one-sided form (the smaller set queries first).
Correspondences, d1 and d2 must equal the oracle's bit for bit.
"""

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check(K, orc, X, Y):
    mm = orc.mutual_match(X, Y)
    out = K.match(dev(X), dev(Y))
    np.testing.assert_array_equal(out.pairs.cpu().numpy(), mm["pairs"])
    np.testing.assert_array_equal(out.d1.cpu().numpy(), mm["d1"].astype(np.float32))
    np.testing.assert_array_equal(out.d2.cpu().numpy(), mm["d2"].astype(np.float32))
    return mm


def test_equal_norms(K, orc):
    # every row a permutation of one multiset: one norm for all, no row can be skipped
    rng = np.random.default_rng(1)
    base = rng.gamma(0.8, 5.0, 33).astype(np.float32)
    X = np.stack([base[rng.permutation(33)] for _ in range(900)])
    Y = np.stack([base[rng.permutation(33)] for _ in range(1100)])
    check(K, orc, X, Y)


@pytest.mark.parametrize("shape", [(700, 2000), (2000, 700), (3000, 3000)])
def test_spread_norms(K, orc, shape):
    # rows scaled over four decades: narrow bands, both orientations
    rng = np.random.default_rng(shape[0] + shape[1])
    X = rng.gamma(0.7, 1.0, (shape[0], 33)) * np.exp(rng.uniform(0, 9, (shape[0], 1)))
    Y = X[rng.integers(0, shape[0], shape[1])] * (1 + 0.02 * rng.standard_normal((shape[1], 33)))
    check(K, orc, X.astype(np.float32), np.abs(Y).astype(np.float32))


@pytest.mark.parametrize("shape", [(1, 40), (40, 1), (2, 3), (3, 2), (65, 64), (64, 65)])
def test_tiny_partners(K, orc, shape):
    rng = np.random.default_rng(7 * shape[0] + shape[1])
    X = rng.gamma(0.7, 10.0, (shape[0], 33)).astype(np.float32)
    Y = rng.gamma(0.7, 10.0, (shape[1], 33)).astype(np.float32)
    check(K, orc, X, Y)


def test_duplicates_and_equal_norm_clusters(K, orc):
    rng = np.random.default_rng(5)
    X = rng.gamma(0.7, 10.0, (1500, 33)).astype(np.float32)
    Y = X[rng.integers(0, 1500, 1700)].copy()  # exact copies: R = 0 for many queries
    Y[:200] = Y[0]                               # a 200-row block of one row, across chunk edges
    X[300:340] = X[301]
    check(K, orc, X, Y)


def test_wide_and_narrow_queries_mixed(K, orc):
    # half the queries have near twins (small R), half are isolated (large R)
    rng = np.random.default_rng(8)
    Y = rng.gamma(0.7, 10.0, (4000, 33)).astype(np.float32)
    near = Y[rng.integers(0, 4000, 1500)] * (1 + 1e-3 * rng.standard_normal((1500, 33)))
    far = rng.gamma(0.7, 30.0, (1500, 33))
    X = np.abs(np.concatenate([near, far])).astype(np.float32)[rng.permutation(3000)]
    check(K, orc, X, Y)


def test_lidar_descriptors_with_rows(K, orc):
    # row lists on both sides (the batch form's J lists): the band maps packed positions back to rows
    d = synth.c0_pair(1)
    ref = orc.run_pair(d["src"], d["tgt"], d["params"], d["vp_src"], d["vp_tgt"])
    Fs, Ft = ref["src"]["fpfh"].astype(np.float32), ref["tgt"]["fpfh"].astype(np.float32)
    js, jt = ref["src"]["j_idx"].astype(np.int32), ref["tgt"]["j_idx"].astype(np.int32)
    mm = orc.mutual_match(Fs[js], Ft[jt])
    out = K.match(dev(Fs), dev(Ft), dev(js), dev(jt))
    pairs = out.pairs.cpu().numpy()
    np.testing.assert_array_equal(pairs, np.stack([js[mm["pairs"][:, 0]], jt[mm["pairs"][:, 1]]], 1)
                                  if len(mm["pairs"]) else pairs)
    np.testing.assert_array_equal(out.d1.cpu().numpy(), mm["d1"].astype(np.float32))


@pytest.mark.parametrize("tuning", [None, {"band_tile": 4}, {"match_form": 1, "band_tile": 16}])
def test_disjoint_tile_bands(K, orc, tuning):
    # query norms over six decades, each query with a near twin among the rows (small R): the
    # four 16-query tiles of a wave need disjoint chunk ranges, so no chunk is shared by all
    # four and every tile runs its own range alone
    rng = np.random.default_rng(11)
    n = 1024
    base = rng.gamma(0.7, 1.0, (n, 33))
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    X = base * (10.0 ** np.linspace(0.0, 6.0, n))[:, None]
    twins = X * (1 + 1e-3 * rng.standard_normal((n, 33)))
    filler = rng.gamma(0.7, 1.0, (1000, 33)) * (10.0 ** rng.uniform(0.0, 6.0, (1000, 1)))
    Y = np.abs(np.concatenate([twins, filler]))[rng.permutation(n + 1000)]
    try:
        K.set_tuning(tuning)
        check(K, orc, X.astype(np.float32), Y.astype(np.float32))
        check(K, orc, Y.astype(np.float32), X.astype(np.float32))
    finally:
        K.set_tuning(None)


@pytest.mark.parametrize("shape", [(0, 50), (50, 0), (1, 40), (40, 1), (2, 3), (65, 64), (1100, 700)])
def test_both_directions_small_and_empty(K, orc, shape):
    # both directions in full: a cloud whose partner has no rows keeps its slot order (its
    # rows-only copy is empty), every other query set is ordered from its cloud's sorted copy
    rng = np.random.default_rng(13 * shape[0] + shape[1])
    X = rng.gamma(0.7, 10.0, (shape[0], 33)).astype(np.float32)
    Y = rng.gamma(0.7, 10.0, (shape[1], 33)).astype(np.float32)
    try:
        K.set_tuning({"match_form": 1, "band_tile": 16})
        if min(shape) == 0:
            out = K.match(dev(X), dev(Y))
            assert out.pairs.shape[0] == 0
        else:
            check(K, orc, X, Y)
    finally:
        K.set_tuning(None)
