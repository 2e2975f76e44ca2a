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


# ----------------------------------------------------- kmg_register_batch --

def register_batch_direct(K, clouds, prec, nnz_per_point=64):
    """kmg_register_batch itself (upload + run in one call) through the C ABI; a batch
    whose neighbour lists overflow the reserve (status KMG_ERR_WORKSPACE, with the
    needed count in the counts table) is run once more with that reserve."""
    import ctypes as C

    lib = K.load()
    n_pairs = len(clouds) // 2
    raw = sum(int(x.shape[1]) for x, _ in clouds)
    nnz_cap = max(1024, nnz_per_point * raw)
    out_cap = max(1, raw // 2)
    pairs = torch.empty((n_pairs, out_cap, 2), dtype=torch.int32, device="cuda")
    d1 = torch.empty((n_pairs, out_cap), dtype=torch.float32, device="cuda")
    d2 = torch.empty((n_pairs, out_cap), dtype=torch.float32, device="cuda")
    counts = torch.zeros((n_pairs, K.COUNTS_STRIDE), dtype=torch.int64, device="cuda")
    ct = (K.KmgCloud * len(clouds))()
    for k, (xyz, prm) in enumerate(clouds):
        ct[k].xyz, ct[k].n, ct[k].params = xyz.data_ptr(), xyz.shape[1], prm
    ot = (K.KmgMatchOut * n_pairs)()
    for i in range(n_pairs):
        ot[i].pairs, ot[i].d1, ot[i].d2, ot[i].cap = pairs[i].data_ptr(), d1[i].data_ptr(), d2[i].data_ptr(), out_cap
    for attempt in range(2):
        ws = torch.empty(int(lib.kmg_batch_workspace_bytes(n_pairs, raw, nnz_cap, 11)), dtype=torch.uint8,
                         device="cuda")
        st = lib.kmg_register_batch(ct, ot, n_pairs, raw, nnz_cap, K.PRECISIONS[prec],
                                    C.c_void_p(counts.data_ptr()), C.c_void_p(ws.data_ptr()), ws.numel(),
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == K.KMG_OK, st
        cnt = counts.cpu().numpy()
        if attempt == 0 and np.any(cnt[:, 6] == K.KMG_ERR_WORKSPACE):
            nnz_cap = int(cnt[0, 7]) + 1024
            continue
        break
    out = []
    for i in range(n_pairs):
        assert cnt[i, 6] == K.KMG_OK, (i, cnt[i])
        k = int(cnt[i, 0])
        out.append((pairs[i, :k].cpu().numpy(), d1[i, :k].cpu().numpy(), d2[i, :k].cpu().numpy(),
                    (int(cnt[i, 1]), int(cnt[i, 2])), (int(cnt[i, 3]), int(cnt[i, 4]))))
    return out


def subset_pairs(n_pairs, seed=5):
    """Seeded random subsets (500-2,000 raw points per cloud) of the planes+spheres pair."""
    d = synth.c0_pair(0)
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_pairs):
        e = dict(d)
        for key in ("src", "tgt"):
            n = int(rng.integers(500, 2001))
            e[key] = np.ascontiguousarray(d[key][:, np.sort(rng.choice(d[key].shape[1], n, replace=False))])
        out.append(e)
    return out


def check_against_oracle(orc, pairs, got, grid=False):
    for i, (d, g) in enumerate(zip(pairs, got)):
        ref = orc.run_pair(d["src"], d["tgt"], d["params"], d["vp_src"], d["vp_tgt"], grid=grid)
        assert g[3] == (len(ref["src"]["kept"]), len(ref["tgt"]["kept"])), i
        assert g[4] == (len(ref["src"]["j_idx"]), len(ref["tgt"]["j_idx"])), i
        np.testing.assert_array_equal(g[0], ref["pairs"], err_msg=f"pair {i}")
        np.testing.assert_array_equal(g[1], ref["d1"].astype(np.float32), err_msg=f"pair {i}")
        np.testing.assert_array_equal(g[2], ref["d2"].astype(np.float32), err_msg=f"pair {i}")


def test_register_batch_entry_point(K, orc):
    """kmg_register_batch (one call) gives the upload + run results and the oracle's."""
    pairs = small_pairs()[:3]
    clouds = [c for d in pairs for c in clouds_of(K, d)]
    got = register_batch_direct(K, clouds, "fp32")
    res, _ = K.register_batch(clouds)
    for g, r in zip(got, res):
        np.testing.assert_array_equal(g[0], r.pairs.cpu().numpy())
        np.testing.assert_array_equal(g[1], r.d1.cpu().numpy())
    check_against_oracle(orc, pairs, got)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_more_than_256_pairs(K, orc, prec):
    """257 pairs: above the 256 pairs whose matching is planned one-sided, both
    directions are matched in full; every pair must still equal the oracle."""
    pairs = subset_pairs(257)
    clouds = [c for d in pairs for c in clouds_of(K, d)]
    got = register_batch_direct(K, clouds, prec)
    check_against_oracle(orc, pairs, got)
    print(f"{prec}: 257 pairs, {sum(len(g[0]) for g in got)} correspondences, oracle-equal")


def test_uneven_batch_sizes_against_oracle(K, orc):
    """Eight pairs of the 64-pair uneven batch recipe in one launch, the largest (~57k
    kept-size target) included, each equal to the oracle (pairs, d1, d2, kept and |J|)."""
    sizes = synth.c2_sizes()
    indoor = [int(i) for i in np.argsort(sizes[:32])]
    lidar = [32 + int(i) for i in np.argsort(sizes[32:])]
    items = sorted({indoor[0], indoor[15], indoor[-1], lidar[0], lidar[10], lidar[20], lidar[-2], lidar[-1]})
    assert int(np.argmax(sizes)) in items and len(items) == 8
    pairs = synth.c2_batch(items=items)
    got = register_batch_direct(K, [c for d in pairs for c in clouds_of(K, d)], "fp32")
    check_against_oracle(orc, pairs, got, grid=True)
    print("uneven batch items", items, "kept", [g[3] for g in got], "correspondences", [len(g[0]) for g in got])


def test_list_beyond_supported_length_is_a_range_error(K):
    """A point with more than 8,192 neighbours within r_FPFH (every point of a
    dense 25^3 lattice, all kept, lies within r_FPFH of the centre) is outside
    the supported range: the batch reports KMG_ERR_RANGE for its pairs in
    either search form, and the per-stage normal estimation raises it."""
    g = np.arange(25, dtype=np.float64) * 0.1
    cube = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    rng = np.random.default_rng(7)
    src = (cube + rng.uniform(-0.01, 0.01, cube.shape)).astype(np.float32)
    tgt = (cube + rng.uniform(-0.01, 0.01, cube.shape)).astype(np.float32)
    prm = K.make_params(0.05, 0.3, 2.0, 3, 0.99, 11, (5.0, 5.0, 5.0))
    clouds = [(dev(src), prm), (dev(tgt), prm)]
    for form in (0, 1):
        K.set_tuning({"search_form": form})
        res, _ = K.register_batch(clouds)
        assert res[0].status == K.KMG_ERR_RANGE, form
    K.set_tuning(None)
    kept, xyz = K.voxelize(dev(src), 0.05)
    assert kept.numel() == cube.shape[1]
    with pytest.raises(K.KmgError) as e:
        K.normals(xyz.contiguous(), prm)
    assert e.value.status == K.KMG_ERR_RANGE
