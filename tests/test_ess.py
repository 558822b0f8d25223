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
