"""Serving loop for registration requests: open-loop arrivals, continuous
batching over several workspace slots, admission under a device-memory
budget, resident descriptors with LRU eviction.

A request is one pair of raw clouds already resident in device memory.  The
device budget is split once into a share for resident descriptors and
`slots` batch slots; each slot owns a kmg batch workspace, its output
buffers and a HIP stream (default priority).  The loop is event driven:

  * arrivals are admitted as they come.  A request whose device-memory
    estimate (the library's batch workspace size for its raw points and
    neighbour entries) exceeds one slot is rejected on its own
    (status KMG_ERR_RANGE, stats.rejected); the others are queued;
  * a free slot takes the queued requests in arrival order while their
    summed estimates fit the slot, once the oldest has waited
    `max_wait_ms` (or the slot would be full, or no more arrivals are
    due), uploads them and enqueues kmg_batch_run on its stream without
    waiting: requests that arrive meanwhile go to the next free slot, so
    batches overlap on the device;
  * finished slots are found by polling their completion events; every
    request of a finished batch is stamped with the completion time.  A
    batch that reports KMG_ERR_WORKSPACE (neighbour lists beyond the
    slot's reserve) or KMG_ERR_RANGE for some pair is split in halves that
    go back to the front of the queue; a request that fails alone keeps
    that status;
  * requests may name their clouds (src_key, tgt_key).  After a batch, the
    descriptors of named clouds are copied out of the workspace
    (kmg_batch_descriptors) into the resident set, least recently used
    first out when its share of the budget is full; a request whose two
    clouds are both resident is served by kmg_match on those descriptors
    alone (the same correspondences, d1 and d2 as the full path).

Latency is completion minus arrival on the host monotonic clock.  The plain
form serves the same queue one request at a time with the per-stage calls.
Host work here is bookkeeping only: every step of the registration runs in
libkmg's kernels.
"""

from __future__ import annotations

import time
from collections import OrderedDict, deque
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
    src_key: object = None    # names of the clouds, for resident descriptors
    tgt_key: object = None
    done: float = -1.0        # completion time, seconds from the start
    result: object = None     # kmg.PairResult (batched), kmg.MatchOut (plain / resident)
    status: int = 0           # kmg status of the request (KMG_ERR_RANGE when rejected)
    batch_size: int = 0
    served: str = ""          # "batch", "resident", "plain" or "rejected"

    @property
    def raw(self) -> int:
        return int(self.src.shape[1]) + int(self.tgt.shape[1])


@dataclass
class ServeStats:
    latencies_ms: list = field(default_factory=list)
    batch_sizes: list = field(default_factory=list)
    wall_s: float = 0.0
    splits: int = 0
    rejected: int = 0
    resident_hits: int = 0
    max_in_flight: int = 0       # largest number of batches on the device at once
    overlapped_batches: int = 0  # batches launched while another was in flight


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


class DescriptorCache:
    """Resident descriptors (kept-space FPFH rows and J list per named cloud),
    least recently used first out under a byte budget."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.bytes = 0
        self.items = OrderedDict()

    def get(self, key):
        if key is None or key not in self.items:
            return None
        self.items.move_to_end(key)
        return self.items[key]

    def put(self, key, fpfh, j_idx):
        nbytes = fpfh.numel() * 4 + j_idx.numel() * 4
        if key is None or nbytes > self.budget:
            return
        if key in self.items:
            self.bytes -= self.items.pop(key)[2]
        while self.items and self.bytes + nbytes > self.budget:
            self.bytes -= self.items.popitem(last=False)[1][2]
        self.items[key] = (fpfh, j_idx, nbytes)
        self.bytes += nbytes


class _Slot:
    def __init__(self, max_pairs, raw_cap, nnz_cap, n_bins, out_cap, device):
        self.batch = kmg.Batch(max_pairs, raw_cap, nnz_cap, n_bins, out_cap=out_cap, device=device)
        self.stream = torch.cuda.Stream(device=self.batch.device)  # default priority
        self.event = None
        self.reqs = None

    @property
    def busy(self):
        return self.event is not None


class Server:
    """Continuous batching over `slots` batch workspaces sized to the device budget."""

    def __init__(self, budget_bytes: int = 200 << 30, max_pairs: int = 128, raw_cap: int = 8 << 20,
                 nnz_per_point: int = 48, out_cap: int = 240000, n_bins: int = 11, prec: str = "fp32",
                 device=None, nnz_cap: int = 0, slots: int = 2, max_wait_ms: float = 2.0,
                 resident_fraction: float = 0.05):
        self.resident = DescriptorCache(int(budget_bytes * resident_fraction))
        per_slot = (budget_bytes - self.resident.budget) // max(1, slots)
        self.raw_cap, self.nnz_cap, self.slot_bytes = workspace_plan(per_slot, max_pairs, raw_cap, nnz_per_point,
                                                                     n_bins, out_cap)
        if nnz_cap > 0:  # an explicit neighbour reserve (tests of the overflow split)
            self.nnz_cap = int(nnz_cap)
        self.bytes = self.slot_bytes * slots + self.resident.budget
        self.max_pairs = max_pairs
        self.nnz_per_point = nnz_per_point
        self.n_bins = n_bins
        self.prec = prec
        self.max_wait = max_wait_ms * 1e-3
        self.slots = [_Slot(max_pairs, self.raw_cap, self.nnz_cap, n_bins, out_cap, device) for _ in range(slots)]
        self.device = self.slots[0].batch.device
        self.match_stream = torch.cuda.Stream(device=self.device)
        self.match_ws = kmg.Workspace(self.device)
        lib = kmg.load()
        base = int(lib.kmg_batch_workspace_bytes(1, 0, 0, n_bins))
        self._per_raw = (int(lib.kmg_batch_workspace_bytes(1, 1 << 20, nnz_per_point << 20, n_bins)) - base) / (1 << 20)
        self._base = base
        self.splits = 0

    # -- admission -----------------------------------------------------------

    def estimate_bytes(self, req: Request) -> float:
        """Device memory the request takes in a batch: its share of the workspace for
        its raw points and their neighbour entries (nnz_per_point per raw point)."""
        return self._per_raw * req.raw

    def slot_budget(self) -> float:
        return self._per_raw * self.raw_cap

    def admits(self, req: Request) -> bool:
        return self.estimate_bytes(req) <= self.slot_budget()

    # -- one batch -------------------------------------------------------------

    def _launch(self, slot: _Slot, reqs: list):
        clouds = []
        for r in reqs:
            clouds += [(r.src, r.params_src), (r.tgt, r.params_tgt)]
        with torch.cuda.stream(slot.stream):
            slot.batch.upload(clouds)
            slot.batch.run(self.prec)
            slot.event = torch.cuda.Event()
            slot.event.record(slot.stream)
        slot.reqs = reqs

    def _finish(self, slot: _Slot, t_done: float, pending: deque, stats: ServeStats) -> list:
        """Consumes a finished slot: returns the requests completed by it; failed
        batches go back to the queue in halves."""
        reqs = slot.reqs
        with torch.cuda.stream(slot.stream):
            res = slot.batch.results()
            bad = [x.status for x in res if x.status in (kmg.KMG_ERR_WORKSPACE, kmg.KMG_ERR_RANGE)]
            out = []
            if bad and len(reqs) > 1:
                self.splits += 1
                stats.splits += 1
                h = len(reqs) // 2
                pending.extendleft(reversed([reqs[:h], reqs[h:]]))  # halves first, in order
            else:
                for i, (r, x) in enumerate(zip(reqs, res)):
                    # results are views into the slot's output buffers: keep copies (stream-ordered)
                    r.result = kmg.PairResult(x.pairs.clone(), x.d1.clone(), x.d2.clone(), x.kept, x.n_j,
                                              x.n_fallback, x.status)
                    r.status = x.status
                    r.done = t_done
                    r.batch_size = len(reqs)
                    r.served = "batch"
                    if x.status == kmg.KMG_OK:
                        for k, key in ((2 * i, r.src_key), (2 * i + 1, r.tgt_key)):
                            if key is not None and self.resident.get(key) is None:
                                fp, jj = slot.batch.descriptors(k, x.kept[k % 2], x.n_j[k % 2])
                                self.resident.put(key, fp, jj)
                    out.append(r)
                stats.batch_sizes.append(len(reqs))
        slot.event = None
        slot.reqs = None
        return out

    def _serve_resident(self, r: Request, t0: float) -> bool:
        a = self.resident.get(r.src_key)
        b = self.resident.get(r.tgt_key)
        if a is None or b is None:
            return False
        with torch.cuda.stream(self.match_stream):
            r.result = kmg.match(a[0], b[0], a[1], b[1], prec=self.prec, ws=self.match_ws)
        r.done = time.perf_counter() - t0
        r.status = kmg.KMG_OK
        r.batch_size = 1
        r.served = "resident"
        return True

    # -- the loop --------------------------------------------------------------

    def serve(self, requests: list, form: str = "batched", ws=None) -> ServeStats:
        """Serves requests (sorted by arrival) open-loop; fills done / result / status."""
        if form not in ("batched", "plain"):
            raise ValueError(form)
        stats = ServeStats()
        pending = deque()  # entries: a request, or a list of requests split from a failed batch
        nxt = 0
        n = len(requests)
        finished = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while finished < n:
            now = time.perf_counter() - t0
            while nxt < n and requests[nxt].arrival <= now:
                r = requests[nxt]
                nxt += 1
                if form == "batched" and self._serve_resident(r, t0):
                    stats.resident_hits += 1
                    finished += 1
                elif not self.admits(r):
                    r.status, r.done, r.served = kmg.KMG_ERR_RANGE, now, "rejected"
                    stats.rejected += 1
                    finished += 1
                else:
                    pending.append(r)
            if form == "plain":
                if not pending:
                    self._idle(requests, nxt, t0)
                    continue
                r = pending.popleft()
                a, b, mt = kmg.register_pair(r.src, r.tgt, r.params_src, r.params_tgt, prec=self.prec, ws=ws)
                torch.cuda.synchronize()
                r.done, r.result, r.batch_size, r.served = time.perf_counter() - t0, mt, 1, "plain"
                stats.batch_sizes.append(1)
                finished += 1
                continue
            progressed = False
            for slot in self.slots:
                if slot.busy and slot.event.query():
                    done = self._finish(slot, time.perf_counter() - t0, pending, stats)
                    finished += len(done)
                    for r in done:
                        if r.status != kmg.KMG_OK:
                            r.served = "failed"
                    progressed = True
            for slot in self.slots:
                if slot.busy or not pending:
                    continue
                head = pending[0]
                if isinstance(head, list):  # a half of a failed batch: run it as it is
                    take = pending.popleft()
                else:
                    now = time.perf_counter() - t0
                    full = self._fits_count(pending) >= self.max_pairs
                    if not (full or now - head.arrival >= self.max_wait or nxt >= n):
                        continue
                    take = self._take(pending)
                in_flight = sum(s.busy for s in self.slots)
                if in_flight:
                    stats.overlapped_batches += 1
                self._launch(slot, take)
                stats.max_in_flight = max(stats.max_in_flight, in_flight + 1)
                progressed = True
            if not progressed:
                self._idle(requests, nxt, t0, busy=any(s.busy for s in self.slots), pending=bool(pending))
        stats.wall_s = time.perf_counter() - t0
        stats.latencies_ms = [1e3 * (r.done - r.arrival) for r in requests if not r.warmup and r.status == 0]
        return stats

    def _fits_count(self, pending) -> int:
        budget = self.slot_budget()
        used, k = 0.0, 0
        for r in pending:
            if isinstance(r, list) or k >= self.max_pairs:
                break
            used += self.estimate_bytes(r)
            if used > budget:
                break
            k += 1
        return k

    def _take(self, pending) -> list:
        budget = self.slot_budget()
        take = [pending.popleft()]
        used = self.estimate_bytes(take[0])
        while pending and not isinstance(pending[0], list) and len(take) < self.max_pairs:
            e = self.estimate_bytes(pending[0])
            if used + e > budget:
                break
            used += e
            take.append(pending.popleft())
        return take

    def _idle(self, requests, nxt, t0, busy=False, pending=False):
        """Nothing to do now: sleep until the next arrival, or briefly while batches run
        or the oldest queued request waits out the batching window."""
        if busy or pending or nxt >= len(requests):
            time.sleep(2e-5)
            return
        wait = requests[nxt].arrival - (time.perf_counter() - t0)
        if wait > 2e-4:
            time.sleep(wait - 1e-4)
