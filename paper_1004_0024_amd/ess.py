"""Effective sample size of a Markov-chain series (host-side analysis).

Integrated autocorrelation time by Sokal's automatic windowing: with the
normalised autocorrelation rho(t), tau(W) = 1/2 + sum_{t=1..W} rho(t), and the
window is the smallest W with W >= c * tau(W) (c = 5).  ESS = n / (2 tau).
"""
from __future__ import annotations

import numpy as np


def autocorrelation(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    x = x - x.mean()
    f = np.fft.rfft(x, n=2 * n)
    acov = np.fft.irfft(f * np.conj(f))[:n] / n
    if acov[0] <= 0:
        return np.zeros(n)
    return acov / acov[0]


def tau_int(x: np.ndarray, c: float = 5.0) -> float:
    rho = autocorrelation(x)
    n = rho.shape[0]
    if n < 2 or not np.any(rho):
        return 0.5
    taus = 0.5 + np.cumsum(rho[1:])
    w = np.arange(1, n)
    ok = w >= c * taus
    if not np.any(ok):
        return float(taus[-1])  # window never closed: the run is too short
    return float(max(taus[np.argmax(ok)], 0.5))


def ess(x: np.ndarray, burn: float = 0.2, c: float = 5.0) -> float:
    x = np.asarray(x)[int(burn * len(x)):]
    return len(x) / (2.0 * tau_int(x, c))


def slot_ess(series: np.ndarray, burn: float = 0.2) -> np.ndarray:
    """ESS per column of a [steps, slots] series of slot energies."""
    return np.array([ess(series[:, k], burn) for k in range(series.shape[1])])
