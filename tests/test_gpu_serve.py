"""Serving loop (paper_2409_15615_amd.serve) on the GPU.

Requests served in continuous batches must give exactly the correspondences
they give alone; the plain one-at-a-time form must give the same sets; every
request completes after it arrives.
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


def make_requests(K, rate, n, small_pool):
    from paper_2409_15615_amd.serve import Request

    out = []
    for r in synth.c4_requests(rate, n, 0, pool=small_pool):
        p = r["params"]
        out.append(Request(
            r["arrival"], torch.from_numpy(r["src"]).cuda(), torch.from_numpy(r["tgt"]).cuda(),
            K.make_params(p.voxel, p.r_normal, p.r_fpfh, p.tau_num, p.tau_lin, p.n_bins, r["vp_src"]),
            K.make_params(p.voxel, p.r_normal, p.r_fpfh, p.tau_num, p.tau_lin, p.n_bins, r["vp_tgt"])))
    return out


@pytest.fixture(scope="module")
def pool():
    return synth.c4_pool(n_each=2)


def test_served_batches_equal_alone_and_plain(K, pool):
    from paper_2409_15615_amd.serve import Server

    reqs = make_requests(K, 5000.0, 24, pool)  # arrivals 0.2 ms apart: requests queue up and batch
    srv = Server(budget_bytes=24 << 30, max_pairs=16, raw_cap=2 << 20, out_cap=130000)
    st = srv.serve(reqs, "batched")
    assert max(st.batch_sizes) > 1, "nothing was batched"
    assert all(r.done >= r.arrival for r in reqs)
    plain = make_requests(K, 5000.0, 24, pool)
    ws = K.Workspace(torch.device("cuda", 0))
    srv.serve(plain, "plain", ws=ws)
    for r, q in zip(reqs, plain):
        assert r.result.status == 0
        alone, _ = K.register_batch([(r.src, r.params_src), (r.tgt, r.params_tgt)])
        np.testing.assert_array_equal(r.result.pairs.cpu().numpy(), alone[0].pairs.cpu().numpy())
        np.testing.assert_array_equal(r.result.d1.cpu().numpy(), alone[0].d1.cpu().numpy())
        np.testing.assert_array_equal(q.result.pairs.cpu().numpy(), alone[0].pairs.cpu().numpy())
    print(f"batch sizes {st.batch_sizes}")


def test_overflowing_batch_is_split(K, pool):
    from paper_2409_15615_amd.serve import Server

    reqs = make_requests(K, 5000.0, 8, pool)
    # a neighbour capacity that holds the largest pair alone but not the whole batch
    nnz = []
    for r in reqs:
        _, b = K.register_batch([(r.src, r.params_src), (r.tgt, r.params_tgt)])
        nnz.append(b.nnz())
    assert sum(nnz) > max(nnz)
    srv = Server(budget_bytes=24 << 30, max_pairs=8, raw_cap=2 << 20, out_cap=130000, nnz_cap=max(nnz))
    reqs[-1].arrival = 0.0  # all requests arrive together: one batch of 8, which must split
    for r in reqs:
        r.arrival = 0.0
    st = srv.serve(reqs, "batched")
    assert st.splits >= 1
    for r in reqs:
        assert r.result.status == 0
        alone, _ = K.register_batch([(r.src, r.params_src), (r.tgt, r.params_tgt)])
        np.testing.assert_array_equal(r.result.pairs.cpu().numpy(), alone[0].pairs.cpu().numpy())
    print(f"splits {st.splits}, batch sizes {st.batch_sizes}")
