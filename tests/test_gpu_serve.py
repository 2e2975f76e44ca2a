"""Serving loop (paper_2409_15615_amd.serve) on the GPU.

Requests served in continuous batches (FP32 and BF16 candidate forms) must give
exactly the correspondences they give alone; the plain one-at-a-time form must
give the same sets; every request completes after it arrives; batches overlap
on the device when requests keep arriving; a request too large for a batch slot
is rejected on its own while the others are served; a batch whose neighbour
lists overflow is split; requests whose clouds are resident are served from the
resident descriptors with the same results.
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


def make_requests(K, rate, n, small_pool, keys=False):
    from paper_2409_15615_amd.serve import Request

    out = []
    for i, r in enumerate(synth.c4_requests(rate, n, 0, pool=small_pool)):
        p = r["params"]
        out.append(Request(
            r["arrival"], torch.from_numpy(r["src"]).cuda(), torch.from_numpy(r["tgt"]).cuda(),
            K.make_params(p.voxel, p.r_normal, p.r_fpfh, p.tau_num, p.tau_lin, p.n_bins, r["vp_src"]),
            K.make_params(p.voxel, p.r_normal, p.r_fpfh, p.tau_num, p.tau_lin, p.n_bins, r["vp_tgt"]),
            src_key=("s", i) if keys else None, tgt_key=("t", i) if keys else None))
    return out


@pytest.fixture(scope="module")
def pool():
    return synth.c4_pool(n_each=2)


def alone(K, r, prec):
    res, _ = K.register_batch([(r.src, r.params_src), (r.tgt, r.params_tgt)], prec=prec)
    return res[0]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_served_batches_equal_alone_and_plain(K, pool, prec):
    from paper_2409_15615_amd.serve import Server

    reqs = make_requests(K, 5000.0, 24, pool)  # arrivals 0.2 ms apart: requests queue up and batch
    srv = Server(budget_bytes=48 << 30, max_pairs=16, raw_cap=2 << 20, out_cap=130000, prec=prec, max_wait_ms=1.0)
    st = srv.serve(reqs, "batched")
    assert max(st.batch_sizes) > 1, "nothing was batched"
    assert st.max_in_flight >= 2 and st.overlapped_batches >= 1, "no two batches were in flight together"
    assert all(r.done >= r.arrival and r.status == 0 for r in reqs)
    plain = make_requests(K, 5000.0, 24, pool)
    ws = K.Workspace(torch.device("cuda", 0))
    srv.serve(plain, "plain", ws=ws)
    for r, q in zip(reqs, plain):
        a = alone(K, r, prec)
        np.testing.assert_array_equal(r.result.pairs.cpu().numpy(), a.pairs.cpu().numpy())
        np.testing.assert_array_equal(r.result.d1.cpu().numpy(), a.d1.cpu().numpy())
        np.testing.assert_array_equal(r.result.d2.cpu().numpy(), a.d2.cpu().numpy())
        np.testing.assert_array_equal(q.result.pairs.cpu().numpy(), a.pairs.cpu().numpy())
    print(f"{prec}: batch sizes {st.batch_sizes}, max in flight {st.max_in_flight}, "
          f"overlapped {st.overlapped_batches}")


def test_oversized_request_rejected_alone(K, pool):
    from paper_2409_15615_amd.serve import Server

    reqs = make_requests(K, 5000.0, 10, pool)
    srv = Server(budget_bytes=48 << 30, max_pairs=8, raw_cap=2 << 20, out_cap=130000)
    big = reqs[4]
    k = int(srv.raw_cap // big.src.shape[1]) + 1
    big.src = big.src.repeat(1, k).contiguous()  # more raw points than one slot holds
    assert not srv.admits(big)
    st = srv.serve(reqs, "batched")
    assert st.rejected == 1 and big.status == K.KMG_ERR_RANGE and big.served == "rejected"
    for r in reqs:
        if r is big:
            continue
        assert r.status == 0
        np.testing.assert_array_equal(r.result.pairs.cpu().numpy(), alone(K, r, "fp32").pairs.cpu().numpy())


def test_overflowing_batch_is_split(K, pool):
    from paper_2409_15615_amd.serve import Server

    reqs = make_requests(K, 5000.0, 8, pool)
    # a neighbour reserve that holds the largest pair alone but not the whole batch
    nnz = []
    for r in reqs:
        _, b = K.register_batch([(r.src, r.params_src), (r.tgt, r.params_tgt)])
        nnz.append(b.nnz())
    assert sum(nnz) > max(nnz)
    srv = Server(budget_bytes=48 << 30, max_pairs=8, raw_cap=2 << 20, out_cap=130000, nnz_cap=max(nnz), slots=1)
    for r in reqs:
        r.arrival = 0.0  # all requests arrive together: one batch of 8, which must split
    st = srv.serve(reqs, "batched")
    assert st.splits >= 1
    for r in reqs:
        assert r.status == 0
        np.testing.assert_array_equal(r.result.pairs.cpu().numpy(), alone(K, r, "fp32").pairs.cpu().numpy())
    print(f"splits {st.splits}, batch sizes {st.batch_sizes}")


def test_resident_descriptors(K, pool):
    """Named clouds: the first pass computes and keeps their descriptors; a second pass of
    the same requests is served from the resident set with the same results; a small
    resident budget evicts the least recently used."""
    from paper_2409_15615_amd.serve import Server

    reqs = make_requests(K, 2000.0, 12, pool, keys=True)
    srv = Server(budget_bytes=48 << 30, max_pairs=8, raw_cap=2 << 20, out_cap=130000)
    st1 = srv.serve(reqs, "batched")
    assert st1.resident_hits == 0
    first = [r.result for r in reqs]
    again = make_requests(K, 2000.0, 12, pool, keys=True)
    st2 = srv.serve(again, "batched")
    assert st2.resident_hits == len(again)
    for r, f in zip(again, first):
        assert r.served == "resident"
        np.testing.assert_array_equal(r.result.pairs.cpu().numpy(), f.pairs.cpu().numpy())
        np.testing.assert_array_equal(r.result.d1.cpu().numpy(), f.d1.cpu().numpy())
        np.testing.assert_array_equal(r.result.d2.cpu().numpy(), f.d2.cpu().numpy())
    # eviction: a budget of about two clouds keeps the most recent ones only
    from paper_2409_15615_amd.serve import DescriptorCache

    c = DescriptorCache(3 * 1000 * 33 * 4)
    for i in range(4):
        c.put(i, torch.zeros((1000, 33), device="cuda"), torch.zeros(10, dtype=torch.int32, device="cuda"))
    assert list(c.items) == [2, 3] and c.bytes <= c.budget
