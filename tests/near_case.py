"""Constructed swap decisions that land within 1e-12 of their threshold.

A replica-exchange decision compares u 2^-32 with exp(Delta), Delta =
(beta_k - beta_k+1)(E_a - E_b) (the swap rule of the oracle and the library).
On random inputs |u 2^-32 - exp(Delta)| < 1e-12 essentially never happens, so
a count of such decisions is only tested by building one: pick the ladder so
that the first decision of round 0, pair (0, 1), has exp(Delta) = u 2^-32 +
offset for the known first output u of the system's swap stream.

The energies that enter Delta come from the oracle (the initial spins, or the
spins after one sweep without swaps); beta_1 is solved for and, when the sweep
comes first, re-solved until the energy it produces no longer moves.  Only the
oracle is called here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from decimal import Decimal, getcontext

import numpy as np

import oracle
from gen import Workload, make_random_system


@dataclass
class NearCase:
    workload: Workload      # one system, K = 3 walkers
    u: int                  # first output of the swap stream
    delta: float            # Delta of the decision, as IEEE double computes it
    gap: float              # exp(Delta) - u 2^-32, exactly (50 digits)
    accept: bool            # the exact decision u 2^-32 < exp(Delta)
    after_sweep: bool       # the decision follows one sweep (else it is taken on the initial spins)


def exact_gap(u: int, delta: float) -> Decimal:
    getcontext().prec = 50
    return Decimal(delta).exp() - Decimal(u) / Decimal(2 ** 32)


def build(offset: float, after_sweep: bool, first_seed: int = 1, tries: int = 200) -> NearCase:
    """A one-system workload whose first swap decision has exp(Delta) - u 2^-32 ~= offset."""
    for t in range(first_seed, first_seed + tries):
        base = make_random_system(12, 20, seed=t, K=3, beta_min=0.5, beta_max=1.5)
        wseeds = (5489 + 3 * t + np.arange(3)).astype(np.uint32)
        sseed = 90_000 + t
        u = int(oracle.mt_stream(sseed, 1)[0])
        x = u / 2.0 ** 32
        if not 0.2 < x < 0.9:
            continue
        b0 = float(base.beta[0])
        b1 = float(base.beta[1])
        N, eu, ev, J, h = base.expand()
        ok = False
        for _ in range(30):
            beta = np.array([b0, b1, b1 + 0.5])
            ch = oracle.Chain(N, eu, ev, J, h, beta, wseeds, sseed)
            if after_sweep:
                ch.sweeps(1, swap_every=0)
            E = ch.energy()
            D = int(E[0] - E[1])
            if D <= 0:
                break
            nb1 = b0 - math.log(x + offset) / D
            if nb1 == b1:
                ok = True
                break
            b1 = nb1
        if not ok or not (b0 < b1 < 10.0):
            continue
        delta = (b0 - b1) * float(D)
        gap = exact_gap(u, delta)
        if abs(float(gap) - offset) > 0.05 * abs(offset):
            continue
        sysm = make_random_system(12, 20, seed=t, K=3, beta_min=0.5, beta_max=1.5)
        sysm.beta = np.array([b0, b1, b1 + 0.5])
        wl = Workload(f"near-threshold swap, offset {offset:g}, {'after a sweep' if after_sweep else 'initial'}",
                      [sysm], 1, 1, walker_seeds=wseeds, swap_seeds=np.array([sseed], np.uint32))
        return NearCase(wl, u, delta, float(gap), gap > 0, after_sweep)
    raise RuntimeError("no near-threshold case found")
