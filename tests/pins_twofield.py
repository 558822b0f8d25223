"""Pins of the oracle's two-field form (the QMC models' separate in-slice and
tau fields) against what the mathematics fixes.

The two-field chain weighs a state s at slot k by exp(-a_k E_sp(s) + c_k B(s)),
with E_sp the cost of h and the in-slice edges and B the sum over tau edges of
J s s'.  Pins:
  - with a = c = beta (dyadic, so every product is exact) the chain is the
    one-field chain, draw for draw;
  - long runs match the enumerated law of a 16-spin two-slice system, and the
    swap acceptance matches its exact expectation;
  - a ring of tau edges matches its 2x2 transfer matrix;
  - the Trotter weights reproduce the quantum expectation of one spin in a
    transverse field as the number of slices grows.
Run by ``test_oracle_twofield.py`` and, against planted mistakes, by its
mutation audit.
"""
from __future__ import annotations

import numpy as np

import oracle
from gen import LayeredSystem, make_chimera_system

from . import exact

DYADIC_BETA = np.array([0.125, 0.25, 0.375, 0.5, 0.75, 1.0])


def _two_field_chain(sysm, a, c, seed0=5489, kind=oracle.ACCEPT_EXACT):
    K = sysm.K
    ch = oracle.Chain.from_system(sysm, seed0 + np.arange(K), seed0 + 1000)
    ch.set_acceptance(kind)
    return ch.set_two_field(oracle.tau_edge_mask(sysm), a, c)


def _split_energies(sysm):
    """E_total, E_sp and B of every state of a small layered system, by enumeration."""
    N, u, v, J, h = sysm.expand()
    tau = oracle.tau_edge_mask(sysm).astype(bool)
    S = exact.all_states(N)
    J64 = np.asarray(J, np.int64)
    prod = S[:, np.asarray(u)] * S[:, np.asarray(v)]
    B = (prod[:, tau] * J64[tau][None, :]).sum(1)
    E = exact.energies(N, u, v, J, h)
    return E, E + B, B, S


def _law(Esp, B, a, c):
    w = -a * (Esp - Esp.min()) + c * (B - B.min())
    p = np.exp(w - w.max())
    return p / p.sum()


# --------------------------------------------------------------- reductions
def pin_tf_equals_one_field():
    """a = c = beta: the two-field chain is the one-field chain (every product exact)."""
    for kind in (oracle.ACCEPT_EXACT, oracle.ACCEPT_FAST, oracle.ACCEPT_ACCURATE):
        sysm = make_chimera_system(2, 4, seed=31, K=len(DYADIC_BETA))
        sysm.beta = DYADIC_BETA.copy()
        one = oracle.Chain.from_system(sysm, 5489 + np.arange(sysm.K), 6489)
        one.set_acceptance(kind)
        two = _two_field_chain(sysm, DYADIC_BETA, DYADIC_BETA, kind=kind)
        for _ in range(6):
            one.sweeps(5, swap_every=1)
            two.sweeps(5, swap_every=1)
            assert np.array_equal(one.spins(), two.spins()), kind
            assert np.array_equal(one.energy(), two.energy()), kind
            assert np.array_equal(one.fields(), two.fields() + two.tau_fields()), kind
            assert np.array_equal(one.mt()[0], two.mt()[0])
            assert np.array_equal(one.labels()[0], two.labels()[0]), kind
            c1, c2 = one.counters(), two.counters()
            for key in ("flips", "swap_att", "swap_acc"):
                assert np.array_equal(c1[key], c2[key]), (kind, key)
        assert two.check_fields() == 0
        assert all(two.bond()[w] == two.bond_of(w) for w in range(sysm.K))


def pin_tf_threshold_matches_one_field():
    """The approximate threshold of a real cost change 2x equals the integer one at x = beta d."""
    for kind in (oracle.ACCEPT_FAST, oracle.ACCEPT_ACCURATE):
        for beta in (0.125, 0.375, 1.0):
            for d in range(1, 20):
                assert oracle.approx_threshold_x(beta * d, kind) == oracle.approx_threshold(beta, d, kind)


# ----------------------------------------------------- enumerated two-field law
def pin_tf_enumeration():
    """One K4,4 cell in two open slices (16 spins), Trotter-like weights, K = 4 slots."""
    sysm = make_chimera_system(1, 2, seed=12, K=4, ring=False, beta_min=0.3, beta_max=1.6)
    a, c = oracle.trotter_weights(sysm.beta, 2, 0.8)
    assert np.all(np.abs(a - c) > 0.05)  # the two weights differ: the tau field must use c
    E, Esp, B, S = _split_energies(sysm)
    N = sysm.N
    ch = _two_field_chain(sysm, a, c)
    n = 120_000
    rec = ch.sweeps(n, swap_every=1, record_energy=True, record_bits=True)
    b0 = n // 10
    es, bits = rec["energy"][b0:], rec["bits"][b0:].astype(np.int64)
    assert ch.check_fields() == 0
    for k in range(sysm.K):
        p = _law(Esp, B, a[k], c[k])
        assert np.array_equal(E[bits[:, k]], es[:, k])
        for name, val in (("E", E), ("B", B), ("Esp", Esp)):
            m, sd = exact.batch_mean_sigma(val[bits[:, k]])
            ref = float((p * val).sum())
            assert abs(m - ref) < 5 * sd + 1e-9, (name, k, m, ref, sd)
        mref = (p[:, None] * S).sum(0)
        for i in range(N):
            mm, ss = exact.batch_mean_sigma(S[bits[:, k], i])
            assert abs(mm - mref[i]) < 5 * ss + 2e-3, ("<s_i>", k, i, mm, mref[i], ss)
    # swap acceptance of each pair: E[min(1, exp(Delta))] over independent draws from the two laws
    cnt = ch.counters()
    for k in range(sysm.K - 1):
        pa, pb = _law(Esp, B, a[k], c[k]), _law(Esp, B, a[k + 1], c[k + 1])
        ia, ib = np.argsort(-pa)[:4000], np.argsort(-pb)[:4000]  # the states carrying the mass
        wa, wb = pa[ia] / pa[ia].sum(), pb[ib] / pb[ib].sum()
        delta = (a[k] - a[k + 1]) * (Esp[ia][:, None] - Esp[ib][None, :]) \
            - (c[k] - c[k + 1]) * (B[ia][:, None] - B[ib][None, :])
        ref = float((wa[:, None] * wb[None, :] * np.minimum(1.0, np.exp(np.minimum(delta, 0.0)))).sum())
        att, acc = int(cnt["swap_att"][k]), int(cnt["swap_acc"][k])
        sd = np.sqrt(ref * (1 - ref) / att) * 3.0
        assert abs(acc / att - ref) < 5 * sd + 5e-3, (k, acc / att, ref, sd)


# ------------------------------------------------------------ closed forms
def transfer_matrix_moments(M, h, a, c):
    """<s> and <s s'> of a ring of M spins with log weight a h sum s + c sum s s'
    (uniform field, unit tau couplings), from the 2x2 transfer matrix."""
    s = np.array([1.0, -1.0])
    T = np.exp(a * h * (s[:, None] + s[None, :]) / 2.0 + c * s[:, None] * s[None, :])
    T = T / np.linalg.eigvalsh(T).max()  # the moments are ratios: scale away overflow
    TM = np.linalg.matrix_power(T, M)
    Z = np.trace(TM)
    sz = np.diag(s)
    m1 = np.trace(sz @ TM) / Z
    m2 = np.trace(sz @ T @ sz @ np.linalg.matrix_power(T, M - 1)) / Z
    return float(m1), float(m2)


def pin_tf_transfer_matrix():
    """Ten copies of one spin joined in a ring by tau edges (J = 1), field h = 1:
    <s> and <s s'> from the transfer matrix, for weights that differ per slot."""
    M = 10
    eu = np.arange(M, dtype=np.int32)
    ev = ((np.arange(M) + 1) % M).astype(np.int32)
    beta = np.array([0.3, 0.6, 1.0, 1.5])
    sysm = LayeredSystem(S=M, M=1, ring=False, eu=eu, ev=ev, eJ=np.ones(M, np.int8),
                         h=np.ones(M, np.int8), J_tau=np.zeros(M, np.int8), beta=beta)
    a = beta / 4.0
    c = np.array([0.9, 0.5, 0.35, 0.2])
    ch = oracle.Chain.from_system(sysm, 5489 + np.arange(4), 6489)
    ch.set_two_field(np.ones(M, np.uint8), a, c)
    n = 150_000
    rec = ch.sweeps(n, swap_every=1, record_bits=True)
    bits = rec["bits"][n // 10:].astype(np.int64)
    S = exact.all_states(M)
    for k in range(4):
        spins = S[bits[:, k]]
        m1_ref, m2_ref = transfer_matrix_moments(M, 1.0, a[k], c[k])
        mm, ss = exact.batch_mean_sigma(spins.mean(1))
        assert abs(mm - m1_ref) < 5 * ss + 1e-3, ("<s>", k, mm, m1_ref, ss)
        bond = (spins * np.roll(spins, -1, axis=1)).mean(1)
        mm, ss = exact.batch_mean_sigma(bond)
        assert abs(mm - m2_ref) < 5 * ss + 1e-3, ("<ss'>", k, mm, m2_ref, ss)
        assert np.array_equal(ch.bond_of(ch.labels()[1][k]), ch.bond()[ch.labels()[1][k]])


def pin_trotter_quantum_limit():
    """One spin, H = -h sz - G sx: with the Trotter weights the ring of M copies gives
    <s> -> (h / w) tanh(beta w), w = sqrt(h^2 + G^2), with an error falling as 1/M^2."""
    for beta, h, G in ((1.0, 0.7, 1.3), (2.5, 0.4, 0.9), (0.6, 1.5, 0.5)):
        w = np.hypot(h, G)
        ref = h / w * np.tanh(beta * w)
        errs = []
        for M in (16, 64, 256):
            a, c = oracle.trotter_weights(np.array([beta]), M, G)
            m1, _ = transfer_matrix_moments(M, h, float(a[0]), float(c[0]))
            errs.append(abs(m1 - ref))
        assert errs[2] < 2e-4, (beta, h, G, errs)
        assert errs[1] < errs[0] and errs[2] < errs[1] / 8, (beta, h, G, errs)


TWO_FIELD_PINS = [
    pin_tf_equals_one_field,
    pin_tf_threshold_matches_one_field,
    pin_tf_enumeration,
    pin_tf_transfer_matrix,
    pin_trotter_quantum_limit,
]
