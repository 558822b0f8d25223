"""Synthetic QMC-style Ising instances: identical layers of a Chimera grid.

The paper's models are many (>= 64) identical copies of a small Ising model,
with edges joining corresponding spins of adjacent layers and the last layer
wrapping to the first (Section 3.1); every spin has 6, 7 or 8 neighbours and a
system has up to 32,768 spins (Section 1).  The 115 production instances used
for the timings (Section 4) are not available, so this module draws stand-ins
of the same shape:

* the layer ("slice") is an L x L grid of K4,4 unit cells, spin
  ``q = (y*L + x)*8 + k``; in-cell spins ``k < 4`` couple to every ``k' >= 4``
  of the same cell, ``k < 4`` couples to the same ``k`` in the cells above and
  below, ``k >= 4`` to the same ``k`` in the cells left and right (open grid);
* M slices; spin ``(m, q)`` has global index ``i = m*S + q`` with ``S = 8 L^2``;
  the Trotter ("tau") edge joins ``(m, q)`` and ``(m+1, q)``, and for a ring
  also ``(M-1, q)`` and ``(0, q)``;
* h and every J are int8, uniform over {-3,-2,-1,1,2,3}; one value per template
  spin / template edge, replicated in every slice (the layers are identical
  copies), and one tau coupling per template spin used for every slice pair.

Draw order from ``numpy.random.default_rng(instance_seed)``: h (S values), the
template edges in the order intra-cell, vertical, horizontal, then the tau
couplings (S values).  The inverse temperatures form a geometric ladder.
Walker r (global index over a workload) is seeded ``5489 + r``; system s's swap
stream is seeded ``5489 + R_total + s``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

VALUES = np.array([-3, -2, -1, 1, 2, 3], dtype=np.int8)


@lru_cache(maxsize=None)
def _chimera_template_cached(L: int):
    S, u, v = _chimera_template(L)
    u.setflags(write=False)
    v.setflags(write=False)
    return S, u, v


def chimera_template(L: int):
    """In-slice edges of an L x L grid of K4,4 cells: (S, u, v) with u < v."""
    S, u, v = _chimera_template_cached(L)
    return S, u.copy(), v.copy()


def _chimera_template(L: int):
    if L < 1:
        raise ValueError("L must be >= 1")
    us, vs = [], []
    cell = lambda y, x: (y * L + x) * 8  # noqa: E731
    for y in range(L):
        for x in range(L):
            c = cell(y, x)
            for k in range(4):
                for k2 in range(4, 8):
                    us.append(c + k)
                    vs.append(c + k2)
    for y in range(L - 1):
        for x in range(L):
            for k in range(4):
                us.append(cell(y, x) + k)
                vs.append(cell(y + 1, x) + k)
    for y in range(L):
        for x in range(L - 1):
            for k in range(4, 8):
                us.append(cell(y, x) + k)
                vs.append(cell(y, x + 1) + k)
    return 8 * L * L, np.array(us, np.int32), np.array(vs, np.int32)


def beta_ladder(K: int, beta_min: float = 0.1, beta_max: float = 3.0) -> np.ndarray:
    """Geometric ladder beta_k = beta_min * (beta_max/beta_min)^(k/(K-1))."""
    if K == 1:
        return np.array([beta_max], np.float64)
    k = np.arange(K, dtype=np.float64)
    return beta_min * (beta_max / beta_min) ** (k / (K - 1))


@dataclass
class LayeredSystem:
    """One Ising system given as M identical slices of an S-spin template.

    ``M == 1`` (no tau edges) describes an arbitrary graph on S spins.
    """

    S: int
    M: int
    ring: bool
    eu: np.ndarray  # int32 [E_t]  template in-slice edges, endpoints in [0, S)
    ev: np.ndarray  # int32 [E_t]
    eJ: np.ndarray  # int8  [E_t]
    h: np.ndarray  # int8  [S]
    J_tau: np.ndarray  # int8  [S]  coupling of (m,q)-(m+1,q); unused if M == 1
    beta: np.ndarray  # float64 [K]
    L: int = 0  # Chimera grid side (0 for a non-Chimera template)

    @property
    def N(self) -> int:
        return self.S * self.M

    @property
    def K(self) -> int:
        return int(self.beta.shape[0])

    def n_edges(self) -> int:
        tau = 0
        if self.M > 1:
            tau = self.S * (self.M if self.ring else self.M - 1)
        return int(self.eu.shape[0]) * self.M + tau

    def expand(self):
        """Full graph: (N, u, v, J, h) with edges listed slice by slice, tau last."""
        S, M = self.S, self.M
        m = np.arange(M, dtype=np.int64)[:, None] * S
        u = (self.eu[None, :].astype(np.int64) + m).ravel()
        v = (self.ev[None, :].astype(np.int64) + m).ravel()
        J = np.tile(self.eJ, M)
        if M > 1:
            npair = M if self.ring else M - 1
            q = np.arange(S, dtype=np.int64)
            a = (np.arange(npair, dtype=np.int64)[:, None] * S + q[None, :]).ravel()
            b = (((np.arange(npair, dtype=np.int64) + 1) % M)[:, None] * S + q[None, :]).ravel()
            u = np.concatenate([u, a])
            v = np.concatenate([v, b])
            J = np.concatenate([J, np.tile(self.J_tau, npair)])
        h = np.tile(self.h, M)
        return self.N, u.astype(np.int32), v.astype(np.int32), J.astype(np.int8), h.astype(np.int8)


def make_chimera_system(L: int, M: int, seed: int, K: int, ring: bool = True,
                        beta_min: float = 0.1, beta_max: float = 3.0) -> LayeredSystem:
    if ring and M < 3:
        raise ValueError("a ring of slices needs M >= 3 (M = 2 would double the tau edge)")
    S, eu, ev = chimera_template(L)
    rng = np.random.default_rng(seed)
    h = VALUES[rng.integers(0, 6, S)]
    eJ = VALUES[rng.integers(0, 6, eu.shape[0])]
    J_tau = VALUES[rng.integers(0, 6, S)]
    return LayeredSystem(S=S, M=M, ring=ring, eu=eu, ev=ev, eJ=eJ, h=h, J_tau=J_tau,
                         beta=beta_ladder(K, beta_min, beta_max), L=L)


def make_random_system(N: int, n_edges: int, seed: int, K: int, max_degree: int = 8,
                       beta_min: float = 0.1, beta_max: float = 3.0,
                       values=VALUES, zero_field: bool = False) -> LayeredSystem:
    """A random simple graph on N spins (one slice, no tau edges) with degree <= max_degree."""
    rng = np.random.default_rng(seed)
    deg = np.zeros(N, np.int64)
    seen = set()
    us, vs = [], []
    tries = 0
    while len(us) < n_edges and tries < 100000:
        tries += 1
        a, b = (int(t) for t in rng.integers(0, N, 2))
        if a == b:
            continue
        a, b = min(a, b), max(a, b)
        if (a, b) in seen or deg[a] >= max_degree or deg[b] >= max_degree:
            continue
        seen.add((a, b))
        deg[a] += 1
        deg[b] += 1
        us.append(a)
        vs.append(b)
    values = np.asarray(values, np.int8)
    h = values[rng.integers(0, len(values), N)]
    if zero_field:
        h = np.zeros(N, np.int8)
    eJ = values[rng.integers(0, len(values), len(us))]
    return LayeredSystem(S=N, M=1, ring=False, eu=np.array(us, np.int32), ev=np.array(vs, np.int32),
                         eJ=eJ.astype(np.int8), h=h.astype(np.int8), J_tau=np.zeros(N, np.int8),
                         beta=beta_ladder(K, beta_min, beta_max))


@dataclass
class Workload:
    """A batch of independent systems with their walker and swap-stream seeds."""

    name: str
    systems: list
    n_sweeps: int
    swap_every: int
    walker_seeds: np.ndarray = field(default=None)  # uint32 [R_total]
    swap_seeds: np.ndarray = field(default=None)  # uint32 [n_sys]
    walker_base: np.ndarray = field(default=None)  # int64 [n_sys + 1]

    def __post_init__(self):
        Ks = np.array([s.K for s in self.systems], np.int64)
        self.walker_base = np.concatenate([[0], np.cumsum(Ks)]).astype(np.int64)
        R = int(self.walker_base[-1])
        if self.walker_seeds is None:
            self.walker_seeds = (5489 + np.arange(R, dtype=np.int64)).astype(np.uint32)
        if self.swap_seeds is None:
            self.swap_seeds = (5489 + R + np.arange(len(self.systems), dtype=np.int64)).astype(np.uint32)

    @property
    def R(self) -> int:
        return int(self.walker_base[-1])

    def attempts_per_sweep(self) -> int:
        return int(sum(s.N * s.K for s in self.systems))

    def subset(self, idx, n_sweeps=None, swap_every=None) -> "Workload":
        """The chosen systems, keeping the seeds they have in the full workload."""
        idx = [int(i) for i in idx]
        ws = np.concatenate([self.walker_seeds[self.walker_base[i]:self.walker_base[i + 1]] for i in idx])
        return Workload(name=f"{self.name}[{len(idx)} of {len(self.systems)}]",
                        systems=[self.systems[i] for i in idx],
                        n_sweeps=self.n_sweeps if n_sweeps is None else n_sweeps,
                        swap_every=self.swap_every if swap_every is None else swap_every,
                        walker_seeds=ws, swap_seeds=self.swap_seeds[idx].copy())


def _uniform_batch(name, n_sys, L, M, K, seed_base, n_sweeps, swap_every=1):
    systems = [make_chimera_system(L, M, seed_base + s, K) for s in range(n_sys)]
    return Workload(name=name, systems=systems, n_sweeps=n_sweeps, swap_every=swap_every)


def _uneven_batch(name, n_sys, n_sweeps, shape_seed, seed_base, swap_every=1):
    rng = np.random.default_rng(shape_seed)
    Ls = rng.integers(2, 9, n_sys)
    Ms = rng.integers(8, 65, n_sys)
    Ks = rng.integers(16, 33, n_sys)
    systems = [make_chimera_system(int(Ls[s]), int(Ms[s]), seed_base + s, int(Ks[s])) for s in range(n_sys)]
    return Workload(name=name, systems=systems, n_sweeps=n_sweeps, swap_every=swap_every)


#: The five workload shapes: (builder, description).
CONFIGS = {
    "A": (lambda: _uniform_batch("A: L=2 M=8 N=256, 1 system x 16 walkers, 1000 sweeps",
                                 1, 2, 8, 16, 0, 1000),
          "latency / parity case"),
    "B": (lambda: _uniform_batch("B: L=8 M=64 N=32768, 256 systems x 32 walkers, 100 sweeps",
                                 256, 8, 64, 32, 1_000_000, 100),
          "plain throughput"),
    "C": (lambda: _uniform_batch("C: L=4 M=32 N=4096, 2048 systems x 32 walkers, 200 sweeps",
                                 2048, 4, 32, 32, 2_000_000, 200),
          "many replicas"),
    "D": (lambda: _uneven_batch("D: 2000 systems, L in 2..8, M in 8..64, K in 16..32, 1000 sweeps",
                                2000, 1000, 4000, 3_000_000),
          "batched uneven sizes"),
    "E": (lambda: _uniform_batch("E: L=4 M=32 N=4096, 256 systems x 32 walkers (learned proposal)",
                                 256, 4, 32, 32, 4_000_000, 100),
          "learned proposal"),
}


def make_workload(name: str) -> Workload:
    return CONFIGS[name][0]()
