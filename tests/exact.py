"""Exact reference quantities for small Ising systems, by brute force.

Independent of the oracle and of the GPU path: the Boltzmann distribution is
enumerated over all 2^N spin states straight from the cost function
f(s) = -sum_i h_i s_i - sum_edges J_ij s_i s_j.
"""
from __future__ import annotations

import numpy as np


def all_states(N: int) -> np.ndarray:
    """[2^N, N] spins in {-1,+1}; row x has s_i = +1 iff bit i of x is set."""
    x = np.arange(2 ** N, dtype=np.int64)[:, None]
    return np.where((x >> np.arange(N)) & 1, 1, -1).astype(np.int64)


def energies(N, u, v, J, h) -> np.ndarray:
    S = all_states(N)
    e = -(S * np.asarray(h, np.int64)[None, :]).sum(1)
    e -= (S[:, np.asarray(u)] * S[:, np.asarray(v)] * np.asarray(J, np.int64)[None, :]).sum(1)
    return e


def boltzmann(E: np.ndarray, beta: float) -> np.ndarray:
    w = -beta * (E - E.min())
    p = np.exp(w - w.max())
    return p / p.sum()


def mean_energy(E, beta):
    return float((boltzmann(E, beta) * E).sum())


def energy_levels(E, beta):
    levels = np.unique(E)
    p = boltzmann(E, beta)
    return levels, np.array([p[E == l].sum() for l in levels])


def marginals(N, E, beta):
    p = boltzmann(E, beta)
    S = all_states(N)
    return (p[:, None] * S).sum(0)


def swap_acceptance(E, beta_a, beta_b):
    """E[min(1, exp((beta_a - beta_b)(E_a - E_b)))] with E_a ~ beta_a, E_b ~ beta_b independent."""
    la, pa = energy_levels(E, beta_a)
    lb, pb = energy_levels(E, beta_b)
    d = (beta_a - beta_b) * (la[:, None] - lb[None, :])
    return float((pa[:, None] * pb[None, :] * np.minimum(1.0, np.exp(np.minimum(d, 0.0)))).sum())


def metropolis_sweep_matrix(N, u, v, J, h, beta) -> np.ndarray:
    """Exact one-sweep transition matrix T[x, y]: single-site Metropolis kernels in order 0..N-1."""
    S = all_states(N)
    nbr = [[] for _ in range(N)]
    for a, b, j in zip(u, v, J):
        nbr[a].append((b, j))
        nbr[b].append((a, j))
    n = 2 ** N
    T = np.eye(n)
    for i in range(N):
        P = np.zeros((n, n))
        for x in range(n):
            s = S[x]
            field = h[i] + sum(j * s[b] for b, j in nbr[i])
            dE = 2 * s[i] * field
            a = min(1.0, float(np.exp(-beta * dE)))
            y = x ^ (1 << i)
            P[x, y] += a
            P[x, x] += 1 - a
        T = T @ P
    return T


def batch_mean_sigma(x: np.ndarray, n_batches: int = 40) -> tuple[float, float]:
    """Mean of a correlated series and its standard error from batch means."""
    x = np.asarray(x, np.float64)
    b = len(x) // n_batches
    bm = x[: b * n_batches].reshape(n_batches, b).mean(1)
    return float(x.mean()), float(bm.std(ddof=1) / np.sqrt(n_batches))


def ring_log_z(M: int, J: float, h: float, beta: float) -> float:
    """ln Z of a periodic 1-D ring of M spins, uniform J and h, by its 2x2 transfer matrix:
    Z = l+^M + l-^M,  l+- = e^{bJ} cosh(bh) +- sqrt(e^{2bJ} sinh^2(bh) + e^{-2bJ})."""
    a = np.exp(beta * J) * np.cosh(beta * h)
    r = np.sqrt(np.exp(2 * beta * J) * np.sinh(beta * h) ** 2 + np.exp(-2 * beta * J))
    lp, lm = a + r, a - r
    return float(M * np.log(lp) + np.log1p((lm / lp) ** M))


def ring_mean_energy(M: int, J: float, h: float, beta: float, step: float = 1e-5) -> float:
    """<E> = -d ln Z / d beta (central difference of the closed form)."""
    return -(ring_log_z(M, J, h, beta + step) - ring_log_z(M, J, h, beta - step)) / (2 * step)
