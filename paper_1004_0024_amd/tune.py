"""Choices the launch-shape autotuner cannot make alone.

Swap cadence, chosen by effective samples per second.

A swap round after every k-th sweep (ising_sweep's swap_every) changes the
chain, so unlike a launch shape it cannot be tuned by time alone: k = 1 costs
the most swap kernels and mixes the ladder fastest.  This tuner runs the chain
from copies of one state at each candidate cadence, records the energy of the
walker at every slot after each sweep, and scores a cadence by the effective
sample size of those energies (Sokal's windowed autocorrelation time, first 20%
dropped) at the coldest slot, summed over systems, per second of GPU time.

Launch shapes of a batch of several buckets.  The library's autotuner times each
bucket alone, but the buckets of one sweep run side by side on the GPU; the
refinement here moves one bucket at a time to the shape that makes the whole sweep
fastest.

Every step runs in the library's kernels; this module only sequences calls and
does the host-side series analysis.
"""
from __future__ import annotations

import numpy as np

from . import learn


def swap_cadence(state, candidates=(1, 2, 4, 8), steps=2000, burn=0.2):
    """Score each cadence from a copy of `state` (which is left unchanged).  Returns
    {"best": k, "trials": [{"swap_every", "ms_per_step", "ess_coldest",
    "ess_median_slot", "ess_per_s"}...]}; the caller passes `best` to later
    ising_sweep calls (and to the oracle, since it changes the chain)."""
    from .binding import State
    g = state.graph
    trials = []
    for every in candidates:
        s2 = State(g).copy_from(state)
        r = learn.run(s2, steps, None, swap_every=int(every))
        e = learn.ess_summary(g, r["e"], burn)
        trials.append({"swap_every": int(every), "ms_per_step": r["ms"] / steps,
                       "ess_coldest": e["coldest_total"], "ess_median_slot": e["median_slot"],
                       "ess_per_s": e["coldest_total"] / (r["ms"] / 1e3)})
        del s2
    best = trials[int(np.argmax([t["ess_per_s"] for t in trials]))]["swap_every"]
    return {"best": best, "trials": trials,
            "objective": "ESS of the coldest slot's energy, summed over systems, per GPU second"}


def _shape_candidates(b):
    """Threads per walker to try for a bucket of S spins: its current count, the
    powers of two at and below S, and above 64 also S, ceil(S/2) and their
    multiples of 64 (the library refuses the ones it cannot run)."""
    import math
    S = b["S"]
    p2 = 1 << math.ceil(math.log2(S))
    cands = {b["tpw"], p2, max(8, p2 // 2)}
    for t in (S, (S + 1) // 2):
        if t > 64:
            cands.update((t, 64 * ((t + 63) // 64)))
    return sorted(c for c in cands if 8 <= c <= 1024)


def _sweep_timer(state, n_sweeps, reps):
    """Microseconds per sweep of the whole batch, every bucket side by side as
    ising_sweep runs them: a captured loop of n_sweeps sweeps, each with its swap
    round, replayed reps times after one untimed replay."""
    import torch

    def timed():
        rep = state.capture(n_sweeps, swap_every=1)
        rep.launch()
        rep.stream.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(rep.stream)
        for _ in range(reps):
            rep.launch()
        e1.record(rep.stream)
        rep.stream.synchronize()
        return e0.elapsed_time(e1) / (reps * n_sweeps) * 1e3
    return timed


def bucket_shapes_side_by_side(state, n_sweeps=100, reps=3):
    """The autotuner times each bucket's launch shapes alone.  This study times the
    whole sweep instead, with one bucket at a time moved to each of its other
    shapes and the rest as they are; each bucket gets its shape back afterwards.
    The chain of `state` advances; pass a scratch state.  Returns {"base_us",
    "trials": [{"bucket", "S", "tpw", "tuned", "us_per_sweep" or "refused"}],
    "base_again_us"}, in microseconds per sweep."""
    from .binding import IsingError
    g = state.graph
    timed = _sweep_timer(state, n_sweeps, reps)
    out = {"base_us": timed(), "trials": []}
    for bi, b in enumerate(g.buckets()):
        for tpw in _shape_candidates(b):
            row = {"bucket": bi, "S": b["S"], "tpw": tpw, "tuned": tpw == b["tpw"]}
            try:
                g.set_launch(bi, tpw, 1 if tpw != b["tpw"] else b["G"])
            except IsingError as e:
                row["refused"] = str(e)[:80]
            else:
                row["us_per_sweep"] = timed()
            out["trials"].append(row)
        g.set_launch(bi, b["tpw"], b["G"])
    out["base_again_us"] = timed()
    return out


def refine_shapes_side_by_side(state, n_sweeps=100, reps=3, min_gain=0.005):
    """After the autotuner: for a batch of several buckets, which run side by side
    on the GPU, move each bucket in turn (most work first) to the candidate shape
    that makes the whole sweep fastest, keeping a change only when it gains more
    than `min_gain`.  The launch shape does not change the chain.  The chain of
    `state` advances; pass a scratch state.  Returns the steps taken: [{"bucket",
    "S", "from", "to", "us_before", "us_after"}] (empty for one bucket)."""
    from .binding import IsingError
    g = state.graph
    bk = g.buckets()
    if len(bk) < 2:
        return []
    timed = _sweep_timer(state, n_sweeps, reps)
    cur = timed()
    steps = []
    for bi in sorted(range(len(bk)), key=lambda i: -bk[i]["work"]):
        b = g.buckets()[bi]
        best = (cur, b["tpw"], b["G"])
        for tpw in _shape_candidates(b):
            if tpw == b["tpw"]:
                continue
            try:
                g.set_launch(bi, tpw, 1)
            except IsingError:
                continue
            t = timed()
            if t < best[0] * (1.0 - min_gain):
                best = (t, tpw, 1)
        g.set_launch(bi, best[1], best[2])
        if best[1] != b["tpw"]:
            steps.append({"bucket": bi, "S": b["S"], "from": b["tpw"], "to": best[1],
                          "us_before": cur, "us_after": best[0]})
            cur = best[0]
    return steps
