"""Autotuner of the kernel launch shapes (kmg_set_tuning).

The tunable fields change how the hot-path kernels schedule their work, never
what they compute or the order of any floating-point sum, so every setting
gives bit-identical results.  The tuner checks that as it goes: each setting's
outputs are fingerprinted and must equal the defaults' fingerprint.

The search is coordinate descent from the defaults over the candidate values
of each field, a field at a time, for `rounds` passes; a setting is timed as
the median of `reps` runs after one warm-up run, with HIP events on the
current stream.  Host work only: the timed runs are the library's kernels.
With graph=True each setting's run is captured in a HIP graph and its replays
are timed (`inner` replays per timed run): a small workload launched eagerly
is bound by the host's launch rate, which would hide the device time being
tuned.  A setting replaces the best one only when it is faster by more than
`min_gain` (a fraction), so that timing noise does not pick settings.
"""

from __future__ import annotations

import statistics

import torch

from . import kmg

SPACE = {
    "search_waves": (2, 4, 8),
    "count_queries": (1, 2, 4),
    "spfh_pair_mean": (0, 16, 24, 32, 8192),
    "fpfh_rows": (1, 2, 4, 8, 16),
    "band_tile": (0, 8, 12, 16, 20, 24, 32, 48, 64),
    "fuse_features": (0, 1),
    "xcd_split": (0, 1, 2, 3),
    "match_form": (0, 1),
    "search_form": (0, 1),
}


class InvarianceError(RuntimeError):
    """A launch shape changed the results (must never happen)."""


def capture(run):
    """run() captured in a HIP graph (after one run on a side stream, as capture needs)."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    return g


def time_setting(run, setting, reps=3, graph=False, inner=1):
    """Median device time (ms) of one `run()` under `setting`, after one warm-up run
    (with graph, of one replay of the captured run)."""
    kmg.set_tuning(setting)
    g = capture(run) if graph else None
    fn = g.replay if graph else run
    fn()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(inner):
            fn()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b) / inner)
    del g
    return statistics.median(times)


def autotune(run, fingerprint, space=None, reps=3, rounds=2, start=None, graph=False, inner=1, min_gain=0.0):
    """Coordinate descent over `space` (default SPACE).  run() enqueues the workload on
    the current stream; fingerprint() returns a comparable digest of its outputs
    (called after a run completes).  Returns (best setting, best ms, default ms, log);
    the best setting is left in force."""
    space = SPACE if space is None else space
    kmg.set_tuning(None)
    best = dict(kmg.get_tuning()) if start is None else dict(start)
    t_default = time_setting(run, best, reps, graph, inner)
    ref = fingerprint()
    t_best = t_default
    log = [(dict(best), t_default)]
    tried = {tuple(sorted(best.items())): t_default}
    for _ in range(rounds):
        improved = False
        for field, values in space.items():
            for v in values:
                cand = dict(best, **{field: v})
                key = tuple(sorted(cand.items()))
                if key in tried:
                    continue
                t = time_setting(run, cand, reps, graph, inner)
                tried[key] = t
                log.append((cand, t))
                fp = fingerprint()
                if fp != ref:
                    kmg.set_tuning(None)
                    raise InvarianceError(f"tuning {cand} changed the results: {fp} against {ref}")
                if t < t_best * (1.0 - min_gain):
                    best, t_best, improved = cand, t, True
        if not improved:
            break
    kmg.set_tuning(best)
    return best, t_best, t_default, log
