"""ESS estimator against the closed form of an AR(1) process:
tau_int = (1 + phi) / (2 (1 - phi)) (with the 1/2 convention)."""
import numpy as np
import pytest

from paper_1004_0024_amd import ess


@pytest.mark.parametrize("phi", [0.0, 0.5, 0.9, 0.97])
def test_tau_int_ar1(phi):
    rng = np.random.default_rng(int(phi * 100))
    n = 400_000
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0]
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    ref = (1 + phi) / (2 * (1 - phi))
    got = ess.tau_int(x)
    assert abs(got - ref) < 0.06 * ref + 0.02, (phi, got, ref)


def test_ess_constant_and_short():
    assert ess.tau_int(np.ones(100)) == 0.5
    x = np.random.default_rng(0).normal(size=1000)
    assert 700 < ess.ess(x, burn=0.0) < 1300


def test_compare_means_flags_a_shift_only():
    import numpy as np
    from paper_1004_0024_amd import learn

    class _S:
        beta = np.linspace(0.1, 3.0, 4)

    class _G:
        systems = [_S()] * 50

    rng = np.random.default_rng(1)
    a = rng.normal(size=(4000, 200))
    b = rng.normal(size=(4000, 200))
    r = learn.compare_means(_G(), a, b)
    assert r["frac_abs_z_below_4"] > 0.99
    assert all(0.4 < z < 1.0 for z in r["median_abs_z_by_slot"])  # |N(0,1)| has median 0.674
    b[:, 3::4] += 0.5
    r = learn.compare_means(_G(), a, b)
    assert r["median_abs_z_by_slot"][3] > 10 and r["frac_abs_z_below_4"] < 0.8
