"""Swap cadence chosen by effective samples per second.

A swap round after every k-th sweep (ising_sweep's swap_every) changes the
chain, so unlike a launch shape it cannot be tuned by time alone: k = 1 costs
the most swap kernels and mixes the ladder fastest.  This tuner runs the chain
from copies of one state at each candidate cadence, records the energy of the
walker at every slot after each sweep, and scores a cadence by the effective
sample size of those energies (Sokal's windowed autocorrelation time, first 20%
dropped) at the coldest slot, summed over systems, per second of GPU time.
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
