"""Batched registration (kmg_register_batch / kmg_batch_run) on the GPU.

Every pair of a batch must give exactly the result it gives alone (bit-equal
correspondences, d1 and d2), the alone result must equal the oracle's, and a
captured graph of kmg_batch_run must reproduce the eager results on every
replay and after a new upload.
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


def kp(K, p, vp):
    return K.make_params(p.voxel, p.r_normal, p.r_fpfh, p.tau_num, p.tau_lin, p.n_bins, vp)


def clouds_of(K, d):
    p = d["params"]
    return [(dev(d["src"]), kp(K, p, d["vp_src"])), (dev(d["tgt"]), kp(K, p, d["vp_tgt"]))]


def small_pairs():
    """An uneven mix: planes+spheres, two indoor rooms, a small-voxel LiDAR pair."""
    out = [synth.c0_pair(0), synth.c0_pair(1)]
    out.append(synth.indoor_pair(2, 101, 3000))
    out.append(synth.indoor_pair(2, 102, 9000))
    out.append(synth.lidar_pair(2, 103, 0.6, n_az=900))
    return out


def as_host(r):
    return (r.pairs.cpu().numpy().copy(), r.d1.cpu().numpy().copy(), r.d2.cpu().numpy().copy(), r.kept, r.n_j)


def test_batch_of_one_equals_oracle(K, orc):
    for d in (synth.c0_pair(0), synth.c1_pair(0)):
        res, _ = K.register_batch(clouds_of(K, d))
        r = res[0]
        assert r.status == 0
        ref = orc.run_pair(d["src"], d["tgt"], d["params"], d["vp_src"], d["vp_tgt"])
        assert r.kept == (len(ref["src"]["kept"]), len(ref["tgt"]["kept"]))
        assert r.n_j == (len(ref["src"]["j_idx"]), len(ref["tgt"]["j_idx"]))
        np.testing.assert_array_equal(r.pairs.cpu().numpy(), ref["pairs"])
        np.testing.assert_array_equal(r.d1.cpu().numpy(), ref["d1"].astype(np.float32))
        np.testing.assert_array_equal(r.d2.cpu().numpy(), ref["d2"].astype(np.float32))
        print(f"{d['name']}: {len(ref['pairs'])} correspondences, oracle-equal")


def test_each_pair_same_alone_and_in_the_mix(K):
    pairs = small_pairs()
    alone = []
    for d in pairs:
        res, _ = K.register_batch(clouds_of(K, d))
        assert res[0].status == 0
        alone.append(as_host(res[0]))
    mixed_clouds = [c for d in pairs for c in clouds_of(K, d)]
    res, _ = K.register_batch(mixed_clouds)
    for i, r in enumerate(res):
        assert r.status == 0
        a = alone[i]
        got = as_host(r)
        np.testing.assert_array_equal(got[0], a[0])
        np.testing.assert_array_equal(got[1], a[1])
        np.testing.assert_array_equal(got[2], a[2])
        assert got[3] == a[3] and got[4] == a[4]
    # the same batch in another order: results follow their pairs
    rev = [c for d in reversed(pairs) for c in clouds_of(K, d)]
    res2, _ = K.register_batch(rev)
    for i, r in enumerate(res2):
        np.testing.assert_array_equal(as_host(r)[0], alone[len(pairs) - 1 - i][0])


def test_batch_pairs_equal_oracle(K, orc):
    pairs = small_pairs()[2:4]
    res, _ = K.register_batch([c for d in pairs for c in clouds_of(K, d)])
    for d, r in zip(pairs, res):
        ref = orc.run_pair(d["src"], d["tgt"], d["params"], d["vp_src"], d["vp_tgt"])
        np.testing.assert_array_equal(r.pairs.cpu().numpy(), ref["pairs"])


def test_empty_and_degenerate_clouds(K):
    p = synth.params_c0()
    empty = torch.zeros((3, 0), dtype=torch.float32, device="cuda")
    line = np.zeros((3, 300), np.float32)
    line[0] = np.linspace(0, 3, 300)
    d = synth.c0_pair(0)
    clouds = [(empty, kp(K, p, np.zeros(3))), (dev(d["tgt"]), kp(K, p, d["vp_tgt"])),
              (dev(line), kp(K, p, np.zeros(3))), (dev(line), kp(K, p, np.zeros(3))),
              (dev(d["src"]), kp(K, p, d["vp_src"])), (dev(d["tgt"]), kp(K, p, d["vp_tgt"]))]
    res, _ = K.register_batch(clouds)
    assert res[0].pairs.shape[0] == 0 and res[0].kept[0] == 0
    assert res[1].pairs.shape[0] == 0 and res[1].n_j == (0, 0)  # collinear: no reliable normals
    alone, _ = K.register_batch(clouds[4:])
    np.testing.assert_array_equal(res[2].pairs.cpu().numpy(), alone[0].pairs.cpu().numpy())


def test_graph_capture_replays(K):
    pairs = small_pairs()
    clouds = [c for d in pairs for c in clouds_of(K, d)]
    eager, b0 = K.register_batch(clouds)
    expect = [as_host(r) for r in eager]
    raw = sum(int(x.shape[1]) for x, _ in clouds)
    b = K.Batch(len(pairs), raw, b0.nnz_cap, 11)
    b.upload(clouds)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        b.counts.zero_()
        b.pairs.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work between replays
        got = [as_host(r) for r in b.results()]
        for gi, ei in zip(got, expect):
            np.testing.assert_array_equal(gi[0], ei[0])
            np.testing.assert_array_equal(gi[1], ei[1])
    # a new batch (pairs in reverse order, same capacities) through the same graph
    rev = [c for d in reversed(pairs) for c in clouds_of(K, d)]
    b.upload(rev)
    g.replay()
    torch.cuda.synchronize()
    got = [as_host(r) for r in b.results()]
    for i, gi in enumerate(got):
        np.testing.assert_array_equal(gi[0], expect[len(pairs) - 1 - i][0])


def test_exact_fallbacks_from_several_pairs(K, orc):
    # lattice planes give many equal descriptors, so the certificate fails for
    # many queries of several pairs at once and one list of exact scans mixes
    # their query sets (in whatever order the re-score appends them)
    pairs = [synth.lattice_pair(0), synth.c0_pair(0), synth.lattice_pair(1, spacing=0.06), synth.c0_pair(1)]
    res, _ = K.register_batch([c for d in pairs for c in clouds_of(K, d)])
    for d, r in zip(pairs, res):
        assert r.status == 0
        ref = orc.run_pair(d["src"], d["tgt"], d["params"], d["vp_src"], d["vp_tgt"])
        np.testing.assert_array_equal(r.pairs.cpu().numpy(), ref["pairs"])
        np.testing.assert_array_equal(r.d1.cpu().numpy(), ref["d1"].astype(np.float32))
        np.testing.assert_array_equal(r.d2.cpu().numpy(), ref["d2"].astype(np.float32))
        print(f"{d['name']}: {len(ref['pairs'])} correspondences, {int(r.n_fallback)} exact scans")
