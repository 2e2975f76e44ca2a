"""Serving loop for registration requests: open-loop arrivals, continuous
batching through kmg_batch_run, admission under a device-memory budget.

A request is one pair of raw clouds already resident in device memory.  The
loop admits every request that has arrived, in arrival order, into the next
batch while the batch stays within the workspace's raw-point and pair
capacities, runs the batch (one kmg_batch_run on one stream), waits for it,
and stamps every request of the batch with the completion time.  Latency is
completion minus arrival on the host monotonic clock.  The plain form serves
the same queue one request at a time with the per-stage calls.

A batch whose neighbour lists overflow the workspace (KMG_ERR_WORKSPACE) is
split in halves and each half is run again; a pair that overflows alone is
reported with that status.  Host work here is bookkeeping only: every step of
the registration runs in libkmg's kernels.
"""

from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import torch

from . import kmg


@dataclass
class Request:
    arrival: float            # seconds from the start of the trace
    src: torch.Tensor         # (3, n) float32, device
    tgt: torch.Tensor
    params_src: kmg.KmgParams
    params_tgt: kmg.KmgParams
    warmup: bool = False
    done: float = -1.0        # completion time, seconds from the start
    result: object = None     # kmg.PairResult (batched) or kmg.MatchOut (plain)
    batch_size: int = 0

    @property
    def raw(self) -> int:
        return int(self.src.shape[1]) + int(self.tgt.shape[1])


@dataclass
class ServeStats:
    latencies_ms: list = field(default_factory=list)
    batch_sizes: list = field(default_factory=list)
    wall_s: float = 0.0
    splits: int = 0


def workspace_plan(budget_bytes: int, max_pairs: int, raw_cap: int, nnz_per_point: int, n_bins: int = 11,
                   out_cap: int = 0) -> tuple:
    """Largest raw-point capacity (halving from raw_cap) whose workspace and
    output buffers fit in budget_bytes -> (raw_cap, nnz_cap, bytes)."""
    lib = kmg.load()
    while raw_cap >= 1024:
        nnz_cap = nnz_per_point * raw_cap
        ws = int(lib.kmg_batch_workspace_bytes(max_pairs, raw_cap, nnz_cap, n_bins))
        outs = max_pairs * max(1, out_cap) * 16 + max_pairs * 64
        if ws and ws + outs <= budget_bytes:
            return raw_cap, nnz_cap, ws + outs
        raw_cap //= 2
    raise ValueError("the memory budget does not hold a minimal batch")


class Server:
    """Continuous-batching server over one preallocated kmg batch workspace."""

    def __init__(self, budget_bytes: int = 200 << 30, max_pairs: int = 128, raw_cap: int = 8 << 20,
                 nnz_per_point: int = 48, out_cap: int = 240000, n_bins: int = 11, prec: str = "fp32",
                 device=None, nnz_cap: int = 0):
        self.raw_cap, self.nnz_cap, self.bytes = workspace_plan(budget_bytes, max_pairs, raw_cap, nnz_per_point,
                                                                n_bins, out_cap)
        if nnz_cap > 0:  # an explicit neighbour capacity (tests of the overflow split)
            self.nnz_cap = int(nnz_cap)
        self.max_pairs = max_pairs
        self.prec = prec
        self.batch = kmg.Batch(max_pairs, self.raw_cap, self.nnz_cap, n_bins, out_cap=out_cap, device=device)
        self.splits = 0

    def admits(self, req: Request) -> bool:
        return req.raw <= self.raw_cap

    def run_batch(self, reqs: list) -> list:
        """Runs reqs (which fit the capacities) -> PairResult per request."""
        clouds = []
        for r in reqs:
            clouds += [(r.src, r.params_src), (r.tgt, r.params_tgt)]
        self.batch.upload(clouds)
        self.batch.run(self.prec)
        res = self.batch.results()  # waits for the stream
        if len(reqs) > 1 and any(x.status == kmg.KMG_ERR_WORKSPACE for x in res):
            self.splits += 1
            h = len(reqs) // 2
            return self.run_batch(reqs[:h]) + self.run_batch(reqs[h:])
        # results are views into the reusable output buffers: keep copies
        return [kmg.PairResult(x.pairs.clone(), x.d1.clone(), x.d2.clone(), x.kept, x.n_j, x.n_fallback, x.status)
                for x in res]

    def serve(self, requests: list, form: str = "batched", ws=None) -> ServeStats:
        """Serves requests (sorted by arrival) open-loop; fills done/result."""
        if form not in ("batched", "plain"):
            raise ValueError(form)
        for r in requests:
            if not self.admits(r):
                raise ValueError(f"request of {r.raw} raw points exceeds the batch capacity {self.raw_cap}")
        stats = ServeStats()
        pending = deque()
        nxt = 0
        n = len(requests)
        finished = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while finished < n:
            now = time.perf_counter() - t0
            while nxt < n and requests[nxt].arrival <= now:
                pending.append(requests[nxt])
                nxt += 1
            if not pending:
                wait = requests[nxt].arrival - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
                continue
            take = [pending.popleft()]
            if form == "batched":
                raw = take[0].raw
                while pending and len(take) < self.max_pairs and raw + pending[0].raw <= self.raw_cap:
                    raw += pending[0].raw
                    take.append(pending.popleft())
                results = self.run_batch(take)
            else:
                a, b, mt = kmg.register_pair(take[0].src, take[0].tgt, take[0].params_src, take[0].params_tgt,
                                             prec=self.prec, ws=ws)
                torch.cuda.synchronize()
                results = [mt]
            t_done = time.perf_counter() - t0
            for r, res in zip(take, results):
                r.done = t_done
                r.result = res
                r.batch_size = len(take)
            stats.batch_sizes.append(len(take))
            finished += len(take)
        stats.wall_s = time.perf_counter() - t0
        stats.latencies_ms = [1e3 * (r.done - r.arrival) for r in requests if not r.warmup]
        stats.splits = self.splits
        return stats
