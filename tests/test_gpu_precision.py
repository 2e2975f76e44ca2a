"""Reduced-precision candidate generation (KMG_FP16 / KMG_BF16) on the GPU.

Candidates come from 16-bit tiles with FP32 accumulation; every decision is
re-scored exactly and certified, so the correspondences, d1 and d2 must be
bit-identical to the oracle's FP64 mutual matching, whatever the precision.
The number of exact re-scans (uncertified queries) is printed.
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRECS = ["fp16", "bf16"]


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


def host(t):
    return t.cpu().numpy()


def check(K, orc, X, Y, prec):
    mm = orc.mutual_match(X, Y)
    out = K.match(dev(X), dev(Y), prec=prec)
    np.testing.assert_array_equal(host(out.pairs), mm["pairs"])
    np.testing.assert_array_equal(host(out.d1), mm["d1"].astype(np.float32))
    np.testing.assert_array_equal(host(out.d2), mm["d2"].astype(np.float32))
    return out, mm


@pytest.fixture(scope="module")
def c1_desc(orc):
    d = synth.c1_pair(0)
    ref = orc.run_pair(d["src"], d["tgt"], d["params"], d["vp_src"], d["vp_tgt"])
    X = ref["src"]["fpfh"][ref["src"]["j_idx"]].astype(np.float32)
    Y = ref["tgt"]["fpfh"][ref["tgt"]["j_idx"]].astype(np.float32)
    return X, Y


@pytest.mark.parametrize("prec", PRECS)
def test_lidar_descriptors(K, orc, c1_desc, prec):
    X, Y = c1_desc
    out, mm = check(K, orc, X, Y, prec)
    q = X.shape[0] + Y.shape[0]
    print(f"{prec}: {X.shape[0]} x {Y.shape[0]} -> {len(mm['pairs'])} pairs; exact re-scans {out.n_fallback} "
          f"({100.0 * out.n_fallback / q:.1f}% of queries)")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [(1, 1), (1, 5), (5, 1), (31, 33), (257, 255), (1000, 777), (4097, 300)])
def test_ragged_sizes(K, orc, prec, shape):
    X, Y, _ = synth.synthetic_descriptors(shape[0], shape[1], item=shape[0] * 7 + shape[1])
    check(K, orc, X, Y, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_ties_and_self_match(K, orc, prec):
    rng = np.random.default_rng(9)
    X = rng.integers(0, 4, (700, 33)).astype(np.float32)
    Y = rng.integers(0, 4, (650, 33)).astype(np.float32)
    check(K, orc, X, Y, prec)
    Z = rng.uniform(0, 50, (500, 33)).astype(np.float32)
    Z[100:120] = Z[7]
    out, _ = check(K, orc, Z, Z, prec)
    assert host(out.pairs)[:, 0].tolist() == [i for i in range(500) if not (100 <= i < 120)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dim", [1, 8, 34, 64])
def test_other_lengths(K, orc, prec, dim):
    rng = np.random.default_rng(dim)
    X = rng.gamma(0.7, 10.0, (600, dim)).astype(np.float32)
    Y = np.abs(np.concatenate([X[:300] * (1 + 0.01 * rng.standard_normal((300, dim))),
                               rng.gamma(0.7, 10.0, (200, dim))])).astype(np.float32)
    check(K, orc, X, Y, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_extreme_ranges(K, orc, prec):
    # tiny and huge magnitudes in one set: the per-pair scale and the FP16 subnormal floor
    rng = np.random.default_rng(11)
    X = rng.gamma(0.7, 1.0, (800, 33)).astype(np.float32)
    X[:200] *= 1e-4
    X[200:400] *= 3e3
    Y = np.abs(X[rng.permutation(800)] * (1 + 1e-3 * rng.standard_normal((800, 33)))).astype(np.float32)
    check(K, orc, X, Y, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_batch_pairs_equal_fp32_form(K, prec):
    pairs = [synth.c0_pair(0), synth.indoor_pair(2, 101, 3000)]
    clouds = []
    for d in pairs:
        p = d["params"]
        for xyz, vp in ((d["src"], d["vp_src"]), (d["tgt"], d["vp_tgt"])):
            clouds.append((dev(xyz), K.make_params(p.voxel, p.r_normal, p.r_fpfh, p.tau_num, p.tau_lin, p.n_bins,
                                                   vp)))
    ref, _ = K.register_batch(clouds, prec="fp32")
    got, _ = K.register_batch(clouds, prec=prec)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(host(a.pairs), host(b.pairs))
        np.testing.assert_array_equal(host(a.d1), host(b.d1))
        np.testing.assert_array_equal(host(a.d2), host(b.d2))


@pytest.mark.parametrize("prec", PRECS)
def test_full_size_sampled(K, orc, prec):
    """100k x 100k FPFH-shaped rows: FP32 and reduced forms agree exactly, and
    sampled rows agree with the oracle's one-by-one NN."""
    X, Y, _ = synth.synthetic_descriptors(100000, 100000, item=77)
    a = K.match(dev(X), dev(Y), prec="fp32")
    b = K.match(dev(X), dev(Y), prec=prec)
    np.testing.assert_array_equal(host(a.pairs), host(b.pairs))
    np.testing.assert_array_equal(host(a.d1), host(b.d1))
    np.testing.assert_array_equal(host(a.d2), host(b.d2))
    pairs = host(b.pairs)
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(X.shape[0], 300, replace=False))
    nn, best, second = orc.nn_rows(X, Y, rows)
    back, _, _ = orc.nn_rows(Y, X, nn)
    mutual = back == rows
    index = {int(i): k for k, i in enumerate(pairs[:, 0])}
    for r, n, bst, sec, mu in zip(rows, nn, best, second, mutual):
        assert (int(r) in index) == bool(mu)
        if mu:
            k = index[int(r)]
            assert pairs[k, 1] == n
            assert host(b.d1)[k] == np.float32(np.sqrt(bst)) and host(b.d2)[k] == np.float32(np.sqrt(sec))
    print(f"{prec}: {len(pairs)} pairs; exact re-scans fp32 {a.n_fallback}, {prec} {b.n_fallback} "
          f"({100.0 * b.n_fallback / 2e5:.2f}% of queries); {int(mutual.sum())} of 300 sampled rows mutual")


@pytest.fixture(scope="module")
def c3_rows(orc):
    """Exactly 100,000 J rows per side of the 100k x 100k matching workload (two submaps of
    four ray-cast scans at voxel 0.15 m), computed by the oracle (grid radius search), then
    a seeded subset as the benchmark takes it."""
    d = synth.c3_pair(0)
    p = d["params"]
    rows = []
    for key, vp in (("src", d["vp_src"]), ("tgt", d["vp_tgt"])):
        kept, _ = orc.voxelize(d[key], p.voxel)
        xyz = np.ascontiguousarray(d[key][:, kept])
        fp = orc.faster_pfh(xyz, p, vp, grid=True)
        j = fp["j_idx"]
        assert j.size >= 100000
        pick = np.sort(np.random.default_rng(2409).permutation(j.size)[:100000])
        rows.append(np.ascontiguousarray(fp["fpfh"][j[pick]].astype(np.float32)))
    return rows


_c3_fp32 = {}


@pytest.mark.parametrize("prec", ["fp32"] + PRECS)
def test_c3_rows_sampled(K, orc, c3_rows, prec):
    """The real FPFH rows of the 100k x 100k workload (tightly clustered, unlike the
    synthetic rows): every precision gives the FP32 form's correspondences, d1 and d2,
    and 300 sampled rows agree with the oracle's one-by-one NN and mutual test."""
    X, Y = c3_rows
    b = K.match(dev(X), dev(Y), prec=prec)
    got = (host(b.pairs), host(b.d1), host(b.d2))
    if prec == "fp32":
        _c3_fp32["ref"] = got
    elif "ref" in _c3_fp32:
        for u, v in zip(got, _c3_fp32["ref"]):
            np.testing.assert_array_equal(u, v)
    pairs = got[0]
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(X.shape[0], 300, replace=False))
    nn, best, second = orc.nn_rows(X, Y, rows)
    back, _, _ = orc.nn_rows(Y, X, nn)
    mutual = back == rows
    index = {int(i): k for k, i in enumerate(pairs[:, 0])}
    for r, n, bst, sec, mu in zip(rows, nn, best, second, mutual):
        assert (int(r) in index) == bool(mu), r
        if mu:
            k = index[int(r)]
            assert pairs[k, 1] == n
            assert got[1][k] == np.float32(np.sqrt(bst)) and got[2][k] == np.float32(np.sqrt(sec))
    print(f"c3 rows {prec}: {len(pairs)} pairs; exact re-scans {b.n_fallback} "
          f"({100.0 * b.n_fallback / 2e5:.2f}% of queries); {int(mutual.sum())} of 300 sampled rows mutual")
