"""Pins of the oracle's layer-pair order (the paper's GPU layout, Sec. 3.2 and
Fig. 12c): pairs of slices (2t, 2t+1) with their own generator, even slices
swept before odd ones.

  - With two slices (one pair) the order is the canonical one and the single
    pair generator is the walker's generator: the chain must equal the
    one-generator chain draw for draw.
  - Generator use: after init every pair generator has delivered 2S outputs,
    and the initial spins of slice 2t+j are the top bits of outputs
    j*S .. j*S+S-1 of generator t (checked against the pinned MT19937 stream);
    each sweep takes 2S more outputs from every pair generator.
  - The chain samples the Boltzmann law: a 16-spin layered system (S = 4,
    M = 4 ring) against enumeration, under parallel tempering.
Run by ``test_oracle_pairs.py`` and by its mutation audit.
"""
from __future__ import annotations

import numpy as np

import oracle
from gen import LayeredSystem, make_chimera_system

from . import exact


def _pair_seeds(K, M, base=9000):
    return (base + np.arange(K * (M // 2))).astype(np.uint32)


def _pairs_chain(sysm, pair_seeds, swap_seed=777):
    K = sysm.K
    ch = oracle.Chain.from_system(sysm, 5489 + np.arange(K), swap_seed)
    return ch.set_pairs(sysm.S, sysm.M, pair_seeds)


def pin_pairs_two_slices_is_canonical():
    """M = 2: one pair per walker, even slice then odd slice = ascending index order."""
    for L in (1, 2):
        sysm = make_chimera_system(L, 2, seed=60 + L, K=5, ring=False)
        seeds = _pair_seeds(sysm.K, 2)
        one = oracle.Chain.from_system(sysm, seeds, 777)
        two = _pairs_chain(sysm, seeds)
        assert np.array_equal(one.spins(), two.spins())
        for n in (1, 4, 25):
            one.sweeps(n, swap_every=1)
            two.sweeps(n, swap_every=1)
            assert np.array_equal(one.spins(), two.spins()), (L, n)
            assert np.array_equal(one.energy(), two.energy()), (L, n)
            assert np.array_equal(one.mt()[0], two.pair_mt()[0]), (L, n)
            assert np.array_equal(one.labels()[0], two.labels()[0]), (L, n)
            c1, c2 = one.counters(), two.counters()
            for key in ("flips", "swap_att", "swap_acc"):
                assert np.array_equal(c1[key], c2[key]), (L, n, key)
        assert two.check_fields() == 0


def pin_pairs_generator_use():
    sysm = make_chimera_system(2, 6, seed=64, K=3)
    S, M, K, P = sysm.S, sysm.M, sysm.K, sysm.M // 2
    seeds = _pair_seeds(K, M, 12345)
    ch = _pairs_chain(sysm, seeds)
    spins = ch.spins()
    win, used = ch.pair_mt()
    assert np.all(used == 2 * S)
    for w in range(K):
        for t in range(P):
            top = oracle.mt_stream(int(seeds[w * P + t]), 2 * S) >> 31
            for j in range(2):
                m = 2 * t + j
                want = np.where(top[j * S:(j + 1) * S] == 1, 1, -1)
                assert np.array_equal(spins[w, m * S:(m + 1) * S], want), (w, t, j)
    ch.sweeps(3, swap_every=1)
    win, used = ch.pair_mt()
    assert np.all(used == 2 * S * 4)
    assert ch.check_fields() == 0


def pin_pairs_enumeration():
    """A 4-spin template (a square with a diagonal) in 4 slices on a ring: 16 spins."""
    eu = np.array([0, 1, 2, 0, 0], np.int32)
    ev = np.array([1, 2, 3, 3, 2], np.int32)
    sysm = LayeredSystem(S=4, M=4, ring=True, eu=eu, ev=ev, eJ=np.array([2, -1, 3, -2, 1], np.int8),
                         h=np.array([1, -2, 1, 3], np.int8), J_tau=np.array([1, 2, -1, 1], np.int8),
                         beta=np.array([0.15, 0.35, 0.7, 1.2]))
    N, u, v, J, h = sysm.expand()
    E = exact.energies(N, u, v, J, h)
    S = exact.all_states(N)
    ch = _pairs_chain(sysm, _pair_seeds(4, 4, 31337))
    n = 150_000
    rec = ch.sweeps(n, swap_every=1, record_energy=True, record_bits=True)
    es, bits = rec["energy"][n // 10:], rec["bits"][n // 10:].astype(np.int64)
    for k in range(sysm.K):
        beta = float(sysm.beta[k])
        assert np.array_equal(E[bits[:, k]], es[:, k])
        m, sd = exact.batch_mean_sigma(es[:, k])
        ref = exact.mean_energy(E, beta)
        assert abs(m - ref) < 5 * sd + 1e-9, ("<E>", k, m, ref, sd)
        mref = exact.marginals(N, E, beta)
        for i in range(N):
            mm, ss = exact.batch_mean_sigma(S[bits[:, k], i])
            assert abs(mm - mref[i]) < 5 * ss + 2e-3, ("<s_i>", k, i, mm, mref[i], ss)
    cnt = ch.counters()
    for k in range(sysm.K - 1):
        ref = exact.swap_acceptance(E, float(sysm.beta[k]), float(sysm.beta[k + 1]))
        att, acc = int(cnt["swap_att"][k]), int(cnt["swap_acc"][k])
        sd = np.sqrt(ref * (1 - ref) / att) * 3.0
        assert abs(acc / att - ref) < 5 * sd + 2e-3, (k, acc / att, ref, sd)
    assert ch.check_fields() == 0


PAIR_PINS = [pin_pairs_two_slices_is_canonical, pin_pairs_generator_use, pin_pairs_enumeration]
