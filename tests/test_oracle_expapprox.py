"""Pins of the paper's approximations of e^x (Sec. 2.4, Fig. 7, Appendix) as the
oracle implements them, against the figures the paper prints for them."""
import numpy as np

import oracle

LN2 = np.log(2.0)
SCALE = np.float32(2.0 * LN2 * LN2)  # the 2 ln^2 2 factor


def test_fast_unscaled_mean_error_is_0_0407():
    """Over one period the unscaled fast approximation (linear interpolation of 2^y between
    integers) overestimates on average by (2 ln^2 2)^-1 - 1, printed as 0.0407."""
    y = (np.arange(65536) + 0.5) / 65536
    x = (y * LN2).astype(np.float32)
    approx = oracle.exp_approx(x, oracle.ACCEPT_FAST).astype(np.float64) / float(SCALE)
    rel = approx / np.exp(x.astype(np.float64)) - 1.0
    assert abs(rel.mean() - 0.0407) < 5e-5
    assert abs(rel.mean() - (1.0 / (2 * LN2 * LN2) - 1.0)) < 5e-6


def test_fast_scaled_mean_error_is_zero():
    y = (np.arange(65536) + 0.5) / 65536
    for shift in (-40, -3, 0, 5):
        x = ((y + shift) * LN2).astype(np.float32)
        rel = oracle.exp_approx(x, oracle.ACCEPT_FAST) / np.exp(x.astype(np.float64)) - 1.0
        assert abs(rel.mean()) < 2e-5, shift
        assert -0.040 < rel.min() and rel.max() < 0.021


def test_fast_exact_at_powers_of_two():
    """The unscaled form is exact where e^x is a power of two (for |n| <= 12, where the FP32
    product x 2^23 log2 e still rounds to n 2^23)."""
    for n in range(-12, 13):
        x = np.float32(n * LN2)
        v = float(oracle.exp_approx(np.array([x]), oracle.ACCEPT_FAST)[0])
        assert v == float(np.float32(2.0 ** n * SCALE)), n


def test_accurate_error_bounds():
    """The 4th-root form has relative error within (-0.01, 0.005) on -31.5 ln 2 <= x < 32 ln 2,
    and is 0 below that range."""
    x = np.linspace(-31.5 * LN2, 32 * LN2, 200001)[:-1].astype(np.float32)
    rel = oracle.exp_approx(x, oracle.ACCEPT_ACCURATE) / np.exp(x.astype(np.float64)) - 1.0
    assert -0.0101 < rel.min() < -0.009
    assert 0.0045 < rel.max() < 0.0051
    assert abs(rel.mean()) < 1e-4
    assert float(oracle.exp_approx(np.array([np.float32(-31.6 * LN2)]), oracle.ACCEPT_ACCURATE)[0]) == 0.0


def test_approx_threshold_semantics():
    """u <= threshold iff u 2^-32 < p, for p = approx(-2 beta d) > 0."""
    rng = np.random.default_rng(3)
    for kind in (oracle.ACCEPT_FAST, oracle.ACCEPT_ACCURATE):
        for beta, d in ((0.1, 1), (0.37, 5), (1.3, 3), (2.9, 2)):
            p = float(oracle.exp_approx(np.array([np.float32(-2.0 * beta * d)]), kind)[0])
            assert p > 0
            t = oracle.approx_threshold(beta, d, kind)
            us = np.concatenate([rng.integers(0, 2**32, 2000), [t - 1, t, t + 1]]).astype(np.int64)
            us = us[(us >= 0) & (us < 2**32)]
            assert np.array_equal(us <= t, us * 2.0 ** -32 < p)
    # below the valid range p = 0 and only u = 0 passes
    assert oracle.approx_threshold(3.0, 60, oracle.ACCEPT_ACCURATE) == 0


def test_approximate_chains_against_enumeration(capsys):
    """16 spins (one K4,4 cell x 2 open slices), 4 temperatures, swaps every sweep: the exact
    test matches the Boltzmann means; the approximate tests are measured beside it (their
    stationary law is not the Boltzmann one; the deviations are printed, not asserted)."""
    from gen import make_chimera_system

    from . import exact
    sysm = make_chimera_system(1, 2, seed=8, K=4, ring=False, beta_min=0.3, beta_max=1.5)
    N, u, v, J, h = sysm.expand()
    E = exact.energies(N, u, v, J, h)
    report = {}
    for kind in (oracle.ACCEPT_EXACT, oracle.ACCEPT_FAST, oracle.ACCEPT_ACCURATE):
        ch = oracle.Chain.from_system(sysm, 7000 + np.arange(4), 7100).set_acceptance(kind)
        ch.sweeps(500, 1)
        rec = ch.sweeps(40000, 1, record_energy=True)["energy"]  # [t, slot]
        zs = []
        for k in range(4):
            m, sd = exact.batch_mean_sigma(rec[:, k].astype(np.float64), 40)
            zs.append((m - exact.mean_energy(E, float(sysm.beta[k]))) / sd)
        report[kind] = zs
    with capsys.disabled():
        print("\nslot mean energy - Boltzmann mean, in standard errors:",
              {k: [round(z, 1) for z in v] for k, v in report.items()})
    assert max(abs(z) for z in report[oracle.ACCEPT_EXACT]) < 5
