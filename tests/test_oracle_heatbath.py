"""Pins of the cell heat-bath oracle: the two-stage draw against the brute-force
conditional Boltzmann law, the sampled frequencies against it, and a chain of
sweeps plus heat-bath passes against exact enumeration (CPU)."""
import numpy as np
import pytest

import oracle
from gen import make_chimera_system
from oracle import heatbath as H
from oracle import learned as L

from . import exact


def _brute(b, J, beta):
    """exp(-beta E_c) over the 256 cell states, normalised, straight from E_c."""
    E = np.zeros(256)
    for byte in range(256):
        s = np.array([1 if (byte >> k) & 1 else -1 for k in range(8)])
        E[byte] = -float(b @ s) - sum(J[k, i] * s[k] * s[4 + i] for k in range(4) for i in range(4))
    p = np.exp(-beta * (E - E.min()))
    return p / p.sum()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_two_stage_law_is_the_conditional_boltzmann_law(seed):
    rng = np.random.default_rng(seed)
    b = rng.integers(-12, 13, 8)
    J = rng.integers(-3, 4, (4, 4))
    beta = float(rng.uniform(0.05, 1.5))
    assert np.allclose(H.two_stage_law(b, J, beta), _brute(b, J, beta), rtol=1e-10, atol=1e-15)


def test_two_stage_law_large_fields():
    """Fields large enough that plain exp would overflow FP32: the log-domain weights hold."""
    b = np.array([27, -25, 20, -18, 26, -27, 15, 9])
    J = np.array([[3, -3, 2, 1], [-2, 3, -3, 2], [1, 1, -1, 3], [-3, 2, 2, -2]])
    assert np.allclose(H.two_stage_law(b, J, 3.0), _brute(b, J, 3.0), rtol=1e-9, atol=1e-300)


def test_draw_frequencies():
    """The draw from uniform words reproduces the law (chi-squared over 256 states)."""
    from scipy import stats
    rng = np.random.default_rng(7)
    b = rng.integers(-4, 5, 8)
    J = rng.integers(-2, 3, (4, 4))
    beta = 0.4
    p = H.two_stage_law(b, J, beta)
    n = 30000
    counts = np.zeros(256)
    for t in range(n):
        counts[H.draw(b, J, beta, H.uniforms(3, 0, t, 0))] += 1
    e = n * p
    big = e >= 5
    chi2 = ((counts[big] - e[big]) ** 2 / e[big]).sum()
    assert stats.chi2.sf(chi2, big.sum() - 1) > 1e-5
    assert counts[~big].sum() <= 3 * e[~big].sum() + 20


def test_uniform_words_layout():
    u = H.uniforms(0x0123456789ABCDEF, 5, 9, 4)
    k = (0x89ABCDEF, 0x01234567)
    assert u[:4] == L.philox4x32((4, 5, 9, 0), k)
    assert u[4] == L.philox4x32((4, 5, 9, 1), k)[0]


def test_heatbath_chain_keeps_boltzmann():
    """Sweeps interleaved 1:1 with heat-bath passes on one cell x 2 open slices (16 spins):
    slot mean energies against exact enumeration; running energies stay exact."""
    K = 3
    sysm = make_chimera_system(1, 2, seed=8, K=K, ring=False, beta_min=0.2, beta_max=0.8)
    model = L.CellModel(sysm)
    ch = oracle.Chain.from_system(sysm, 9000 + np.arange(K), 9100)
    N, u, v, J, h = sysm.expand()
    E = exact.energies(N, u, v, J, h)
    es = []
    changed = 0
    for t in range(2000):
        ch.sweeps(1, swap_every=0)
        spins = ch.spins().astype(np.int64)
        energy = ch.energy().copy()
        temp_of, _ = ch.labels()
        changed += H.heatbath_pass(model, spins, energy, sysm.beta[temp_of], 55, list(range(K)), t).sum()
        for w in range(K):
            ch.set_spins(w, spins[w].astype(np.int8))
        assert np.array_equal(ch.energy(), energy)
        es.append(ch.energy()[np.argsort(temp_of)].copy())
    es = np.array(es)
    assert changed > 0
    burn = len(es) // 10
    for k in range(K):
        m, sd = exact.batch_mean_sigma(es[burn:, k], 20)
        ref = exact.mean_energy(E, float(sysm.beta[k]))
        assert abs(m - ref) < 5 * sd + 0.05, (k, m, ref, sd)
