"""Pins of the oracle against what the mathematics and libraries fix.

Each function raises AssertionError when the oracle disagrees.  They are run
by ``test_oracle_pins.py`` against the real oracle and by
``test_oracle_mutations.py`` against deliberately broken copies of it, to show
that a plausible mistake anywhere in the oracle fails at least one pin.
"""
from __future__ import annotations

import os

import numpy as np
from scipy import stats

import oracle
from gen import LayeredSystem, beta_ladder, make_chimera_system, make_random_system

from . import exact

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# --------------------------------------------------------------------- MT19937
def pin_mt_known_answer():
    for line in open(os.path.join(GOLDEN, "mt19937_known_answer.txt")):
        if line.startswith("#") or not line.strip():
            continue
        seed, idx, val = (int(t) for t in line.split())
        got = oracle.mt_stream(seed, idx)[idx - 1]
        assert int(got) == val, (seed, idx, int(got), val)


def pin_mt_matches_library():
    """numpy's legacy RandomState seeds MT19937 with init_genrand and returns raw words."""
    for r in (0, 1, 7, 4095):
        seed = 5489 + r
        n = 200_000 if r else 1_000_000
        ref = np.random.RandomState(seed).randint(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(oracle.mt_stream(seed, n), ref), seed


def pin_mt_window_continues_stream():
    """The 624-word window after c outputs, loaded into the library generator, continues the stream."""
    sysm = make_random_system(6, 6, seed=3, K=1)
    N, u, v, J, h = sysm.expand()
    for seed in (5489, 99):
        ch = oracle.Chain(N, u, v, J, h, sysm.beta, [seed], 1)
        for n_sw in (0, 1, 103, 104, 150):
            if n_sw:
                ch.sweeps(n_sw - (ch.sweeps_done), swap_every=0)
            win, used = ch.mt()
            assert used[0] == N * (1 + ch.sweeps_done)
            rs = np.random.RandomState()
            rs.set_state(("MT19937", win[0].copy(), 624))
            nxt = rs.randint(0, 2 ** 32, size=700, dtype=np.uint64).astype(np.uint32)
            ref = oracle.mt_stream(seed, 700, skip=int(used[0]))
            assert np.array_equal(nxt, ref), (seed, n_sw)


# ------------------------------------------------------------- cost function
def pin_energy_by_enumeration():
    for seed in (1, 2):
        sysm = make_random_system(9, 14, seed=seed, K=1)
        N, u, v, J, h = sysm.expand()
        E = exact.energies(N, u, v, J, h)
        ch = oracle.Chain(N, u, v, J, h, sysm.beta, [1], 1)
        S = exact.all_states(N)
        for x in (0, 1, 77, 255, 300, 511):
            ch.set_spins(0, S[x])
            assert ch.energy_of(0) == E[x], (x, ch.energy_of(0), E[x])
            assert ch.energy()[0] == E[x]


def pin_energy_all_up():
    sysm = make_chimera_system(2, 8, seed=5, K=1)
    N, u, v, J, h = sysm.expand()
    ch = oracle.Chain(N, u, v, J, h, sysm.beta, [1], 1)
    ch.set_spins(0, np.ones(N, np.int8))
    assert ch.energy_of(0) == -int(h.astype(np.int64).sum()) - int(J.astype(np.int64).sum())
    f = ch.fields()[0]
    deg_sum = np.zeros(N, np.int64)
    np.add.at(deg_sum, u, J.astype(np.int64))
    np.add.at(deg_sum, v, J.astype(np.int64))
    assert np.array_equal(f, h.astype(np.int64) + deg_sum)


def pin_incremental_fields():
    """Running local fields and energies equal a recomputation after every sweep."""
    sysm = make_chimera_system(2, 8, seed=11, K=6)
    ws = 5489 + np.arange(6)
    ch = oracle.Chain.from_system(sysm, ws, 7)
    assert ch.check_fields() == 0
    for _ in range(30):
        ch.sweeps(1, swap_every=1)
        assert ch.check_fields() == 0
        E = ch.energy()
        assert all(E[w] == ch.energy_of(w) for w in range(6))


# ------------------------------------------------------------ Metropolis sweep
def pin_sweep_transition_matrix():
    """Empirical one-sweep transitions of a 3-spin chain against the exact product kernel."""
    N, u, v, J, h = 3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), \
        np.array([2, -1], np.int8), np.array([1, -2, 1], np.int8)
    beta = 0.35
    ch = oracle.Chain(N, u, v, J, h, [beta], [4242], 1)
    s0 = ch.spins()[0]
    x0 = int(sum(1 << i for i in range(N) if s0[i] > 0))
    n = 300_000
    bits = ch.sweeps(n, swap_every=0, record_bits=True)["bits"][:, 0].astype(np.int64)
    prev = np.concatenate([[x0], bits[:-1]])
    C = np.zeros((8, 8))
    np.add.at(C, (prev, bits), 1)
    T = exact.metropolis_sweep_matrix(N, u, v, J, h, beta)
    chi2, dof = 0.0, 0
    for x in range(8):
        nx = C[x].sum()
        mask = T[x] > 0
        assert C[x][~mask].sum() == 0, "impossible transition observed"
        e = nx * T[x][mask]
        chi2 += float(((C[x][mask] - e) ** 2 / e).sum())
        dof += int(mask.sum()) - 1
    p = stats.chi2.sf(chi2, dof)
    assert p > 1e-5, (chi2, dof, p)


def _pt_run(sysm, n, seed0=5489, swap_every=1, burn=0.1):
    K = sysm.K
    ch = oracle.Chain.from_system(sysm, seed0 + np.arange(K), seed0 + 1000)
    rec = ch.sweeps(n, swap_every=swap_every, record_energy=True, record_bits=True)
    b = int(burn * n)
    return ch, rec["energy"][b:], rec["bits"][b:]


def _check_against_enumeration(sysm, n):
    N, u, v, J, h = sysm.expand()
    E = exact.energies(N, u, v, J, h)
    S = exact.all_states(N)
    ch, es, bits = _pt_run(sysm, n)
    for k in range(sysm.K):
        beta = float(sysm.beta[k])
        m, sd = exact.batch_mean_sigma(es[:, k])
        ref = exact.mean_energy(E, beta)
        assert abs(m - ref) < 5 * sd + 1e-9, ("<E>", k, m, ref, sd)
        # energy of the recorded state equals the recorded energy
        assert np.array_equal(E[bits[:, k].astype(np.int64)], es[:, k])
        spins = S[bits[:, k].astype(np.int64)]
        mref = exact.marginals(N, E, beta)
        for i in range(N):
            mm, ss = exact.batch_mean_sigma(spins[:, i])
            assert abs(mm - mref[i]) < 5 * ss + 2e-3, ("<s_i>", k, i, mm, mref[i], ss)
        levels, p = exact.energy_levels(E, beta)
        idx = np.searchsorted(levels, es[:, k])
        for j in np.argsort(-p)[:4]:
            series = (idx == j).astype(np.float64)
            mm, ss = exact.batch_mean_sigma(series)
            assert abs(mm - p[j]) < 5 * ss + 2e-3, ("P(E)", k, levels[j], mm, p[j], ss)
    return ch


def pin_enumeration_random_graph():
    sysm = make_random_system(10, 16, seed=21, K=5, beta_min=0.1, beta_max=1.2)
    _check_against_enumeration(sysm, 120_000)


def pin_enumeration_layered():
    """One K4,4 cell, two open Trotter slices (16 spins)."""
    sysm = make_chimera_system(1, 2, seed=8, K=5, ring=False, beta_min=0.1, beta_max=0.9)
    _check_against_enumeration(sysm, 100_000)


def pin_zero_coupling():
    """No edges: each spin is independent, <s_i> = tanh(beta h_i)."""
    N = 6
    h = np.array([1, -1, 2, -3, 3, -2], np.int8)
    beta = beta_ladder(3, 0.2, 0.8)
    sysm = LayeredSystem(S=N, M=1, ring=False, eu=np.zeros(0, np.int32), ev=np.zeros(0, np.int32),
                         eJ=np.zeros(0, np.int8), h=h, J_tau=np.zeros(N, np.int8), beta=beta)
    ch, es, bits = _pt_run(sysm, 60_000)
    S = exact.all_states(N)
    for k in range(3):
        spins = S[bits[:, k].astype(np.int64)]
        for i in range(N):
            mm, ss = exact.batch_mean_sigma(spins[:, i])
            ref = np.tanh(beta[k] * h[i])
            assert abs(mm - ref) < 5 * ss + 1e-3, (k, i, mm, ref)


def pin_ring_closed_form():
    """Periodic ring, uniform J = 1 and h = 1: <E> = -d ln Z / d beta by the transfer matrix.

    (At h = 0 the sequential sweep is not ergodic on a uniform ring: states in which
    every visited spin has dE <= 0 cycle deterministically, so time averages need not
    reach the Boltzmann values.  That is a property of the method, so the pin uses h = 1.)
    """
    M = 12
    eu = np.arange(M, dtype=np.int32)
    ev = ((np.arange(M) + 1) % M).astype(np.int32)
    beta = beta_ladder(4, 0.2, 1.0)
    sysm = LayeredSystem(S=M, M=1, ring=False, eu=eu, ev=ev, eJ=np.ones(M, np.int8),
                         h=np.ones(M, np.int8), J_tau=np.zeros(M, np.int8), beta=beta)
    N, u, v, J, h = sysm.expand()
    ch, es, bits = _pt_run(sysm, 80_000)
    for k in range(4):
        m, sd = exact.batch_mean_sigma(es[:, k])
        ref = exact.ring_mean_energy(M, 1.0, 1.0, float(beta[k]))
        assert abs(ref - exact.mean_energy(exact.energies(N, u, v, J, h), float(beta[k]))) < 1e-6
        assert abs(m - ref) < 5 * sd, (k, m, ref, sd)


# ------------------------------------------------------ parallel tempering
def pin_swap_acceptance():
    sysm = make_random_system(9, 13, seed=4, K=5, beta_min=0.1, beta_max=1.0)
    N, u, v, J, h = sysm.expand()
    E = exact.energies(N, u, v, J, h)
    n = 150_000
    ch, es, bits = _pt_run(sysm, n, burn=0.0)
    c = ch.counters()
    for k in range(sysm.K - 1):
        att, acc = int(c["swap_att"][k]), int(c["swap_acc"][k])
        ref = exact.swap_acceptance(E, float(sysm.beta[k]), float(sysm.beta[k + 1]))
        rate = acc / att
        sd = np.sqrt(ref * (1 - ref) / att) * 3.0  # generous: rounds are correlated
        assert abs(rate - ref) < 5 * sd + 2e-3, (k, rate, ref, sd)


def pin_swap_schedule_and_draws():
    """Even rounds try pairs (0,1),(2,3)..; odd rounds (1,2),(3,4)..; one swap draw per pair."""
    sysm = make_random_system(5, 4, seed=9, K=6)
    ch = oracle.Chain.from_system(sysm, 5489 + np.arange(6), 77)
    ch.sweeps(7, swap_every=1)
    c = ch.counters()
    assert list(c["swap_att"][:5]) == [4, 3, 4, 3, 4]
    win, used = ch.swap_mt()
    assert used == 4 * 3 + 3 * 2
    ch.sweeps(6, swap_every=3)  # rounds after sweeps 9 and 12 (counts continue)
    assert ch.rounds_done == 9
    wt, used_w = ch.mt()
    assert all(used_w == 5 * (1 + 13))


def pin_initial_spins_reading():
    """Initial spin i of a walker is +1 iff the top bit of its stream's i-th output is set."""
    sysm = make_chimera_system(1, 3, seed=2, K=3)
    ch = oracle.Chain.from_system(sysm, [11, 12, 13], 5)
    s = ch.spins()
    for w, seed in enumerate((11, 12, 13)):
        top = oracle.mt_stream(seed, sysm.N) >> 31
        assert np.array_equal(s[w], np.where(top == 1, 1, -1))


def pin_labels_consistent():
    sysm = make_random_system(8, 10, seed=12, K=7)
    ch = oracle.Chain.from_system(sysm, 5489 + np.arange(7), 78)
    for _ in range(50):
        ch.sweeps(1, swap_every=1)
        t, w = ch.labels()
        assert sorted(w) == list(range(7))
        assert all(t[w[k]] == k for k in range(7))


def pin_near_threshold_swaps():
    """Constructed decisions with exp(Delta) - u 2^-32 = +-1e-14 are counted once, on their
    pair, and decided as the exact comparison decides them; at 3e-12 they are not counted.
    The count is taken on the initial energies and after a sweep."""
    from . import near_case
    for offset, counted in ((1e-14, 1), (-1e-14, 1), (3e-12, 0), (-3e-12, 0)):
        for after in (False, True):
            nc = near_case.build(offset, after)
            assert (nc.gap > 0) == (offset > 0) and 0.5 * abs(offset) < abs(nc.gap) < 2 * abs(offset)
            ch = oracle.workload_chains(nc.workload)[0]
            if after:
                ch.sweeps(1, swap_every=1)
            else:
                ch.swap_round(0)
            c = ch.counters()
            assert list(c["swap_near"]) == [counted, 0, 0], (offset, after, c["swap_near"])
            assert list(c["swap_att"]) == [1, 0, 0]
            assert int(c["swap_acc"][0]) == int(nc.accept), (offset, after)
            t, w = ch.labels()
            assert list(w) == ([1, 0, 2] if nc.accept else [0, 1, 2])
            sw, used = ch.swap_mt()
            assert used == 1


ALL_PINS = [
    pin_mt_known_answer,
    pin_mt_matches_library,
    pin_mt_window_continues_stream,
    pin_energy_by_enumeration,
    pin_energy_all_up,
    pin_incremental_fields,
    pin_sweep_transition_matrix,
    pin_enumeration_random_graph,
    pin_enumeration_layered,
    pin_zero_coupling,
    pin_ring_closed_form,
    pin_swap_acceptance,
    pin_swap_schedule_and_draws,
    pin_labels_consistent,
    pin_initial_spins_reading,
    pin_near_threshold_swaps,
]
