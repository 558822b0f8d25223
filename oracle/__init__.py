"""Oracle -- TEST INFRASTRUCTURE ONLY.

Python wrapper over the plain C oracle in ``orc.c``; the learned-proposal
oracle is ``learned.py`` and the cell heat-bath oracle ``heatbath.py``.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library under ``paper_1004_0024_amd/``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "orc.c")]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, no hand-written SIMD)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-Wextra", "-o", tmp] + SOURCES + ["-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", LIB_PATH)  # a mutated build, for the pin audit
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(path)
        P = C.c_void_p
        i32, i64, u32 = C.c_int32, C.c_int64, C.c_uint32
        L.orc_mt_stream.argtypes = [u32, i64, i64, P]
        L.orc_new.argtypes = [i32, i32, P, P, P, P, i32, P, P, u32]
        L.orc_new.restype = P
        L.orc_free.argtypes = [P]
        L.orc_sweeps.argtypes = [P, i32, i32, P, P, P]
        L.orc_swap_round.argtypes = [P, i32]
        L.orc_run_many.argtypes = [i32, P, i32, i32, i32]
        for name in ("orc_N", "orc_K"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = i32
        for name in ("orc_sweeps_done", "orc_rounds_done", "orc_check_fields"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = i64
        L.orc_energy_of.argtypes = [P, i32]
        L.orc_energy_of.restype = i64
        for name in ("orc_get_spins", "orc_get_fields", "orc_get_energy"):
            getattr(L, name).argtypes = [P, P]
        L.orc_get_labels.argtypes = [P, P, P]
        L.orc_get_mt.argtypes = [P, P, P]
        L.orc_get_swap_mt.argtypes = [P, P, P]
        L.orc_get_counters.argtypes = [P, P, P, P, P]
        L.orc_set_spins.argtypes = [P, i32, P]
        L.orc_set_acceptance.argtypes = [P, i32]
        L.orc_exp_approx.argtypes = [C.c_float, i32]
        L.orc_exp_approx.restype = C.c_float
        L.orc_approx_threshold.argtypes = [C.c_double, i32, i32]
        L.orc_approx_threshold.restype = u32
        L.orc_approx_threshold_x.argtypes = [C.c_double, i32]
        L.orc_approx_threshold_x.restype = u32
        L.orc_set_two_field.argtypes = [P, P, i32, P, P]
        L.orc_set_two_field.restype = i32
        L.orc_bond_of.argtypes = [P, i32]
        L.orc_bond_of.restype = i64
        L.orc_get_bond.argtypes = [P, P]
        L.orc_get_tau_fields.argtypes = [P, P]
        L.orc_set_pairs.argtypes = [P, i32, i32, P]
        L.orc_set_pairs.restype = i32
        L.orc_get_pair_mt.argtypes = [P, P, P]
        _lib = L
    return _lib


ACCEPT_EXACT, ACCEPT_FAST, ACCEPT_ACCURATE = 0, 1, 2


def exp_approx(x, kind):
    """The paper's approximation of e^x (Sec. 2.4, Fig. 7), FP32, elementwise."""
    f = lib().orc_exp_approx
    return np.array([f(float(v), int(kind)) for v in np.ravel(x)], np.float32).reshape(np.shape(x))


def approx_threshold(beta, d, kind):
    return int(lib().orc_approx_threshold(float(beta), int(d), int(kind)))


def approx_threshold_x(x, kind):
    """Threshold of the approximate flip test for a real cost change 2x (two-field form)."""
    return int(lib().orc_approx_threshold_x(float(x), int(kind)))


def trotter_weights(beta, M, gamma):
    """Slot weights of the two-field form for a transverse field gamma, M slices.

    Suzuki-Trotter reading: a slice carries the classical cost at inverse
    temperature beta / M, and neighbouring copies of a spin are coupled by
    c = -1/2 ln tanh(beta gamma / M) (so that e^{c} + e^{-c} sigma_x is
    proportional to exp(beta gamma sigma_x / M)).  Returns (a, c) arrays.
    """
    beta = np.asarray(beta, np.float64)
    a = beta / float(M)
    c = -0.5 * np.log(np.tanh(beta * float(gamma) / float(M)))
    return a, c


def tau_edge_mask(system) -> np.ndarray:
    """Flags of the tau edges in the edge order of ``system.expand()`` (in-slice
    edges slice by slice, then the tau edges)."""
    N, u, v, J, h = system.expand()
    n_space = int(system.eu.shape[0]) * system.M
    m = np.zeros(len(u), np.uint8)
    m[n_space:] = 1
    return m


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def mt_stream(seed: int, n: int, skip: int = 0) -> np.ndarray:
    out = np.empty(n, np.uint32)
    lib().orc_mt_stream(seed, skip, n, _ptr(out))
    return out


class Chain:
    """One system under the oracle: K walkers + one swap stream."""

    def __init__(self, N, u, v, J, h, beta, walker_seeds, swap_seed):
        self._keep = [np.ascontiguousarray(u, np.int32), np.ascontiguousarray(v, np.int32),
                      np.ascontiguousarray(J, np.int8), np.ascontiguousarray(h, np.int8),
                      np.ascontiguousarray(beta, np.float64), np.ascontiguousarray(walker_seeds, np.uint32)]
        u_, v_, J_, h_, b_, ws_ = self._keep
        assert len(ws_) == len(b_) and len(h_) == N
        self.N, self.K = int(N), int(len(b_))
        self.h = self._keep[3]
        self._c = lib().orc_new(self.N, len(u_), _ptr(u_), _ptr(v_), _ptr(J_), _ptr(h_), self.K,
                                _ptr(b_), _ptr(ws_), int(swap_seed))
        if not self._c:
            raise ValueError("oracle rejected the system")

    @classmethod
    def from_system(cls, system, walker_seeds, swap_seed):
        N, u, v, J, h = system.expand()
        return cls(N, u, v, J, h, system.beta, walker_seeds, swap_seed)

    def __del__(self):
        c = getattr(self, "_c", None)
        if c:
            lib().orc_free(c)
            self._c = None

    def sweeps(self, n, swap_every=1, record_energy=False, record_bits=False, record_spins=False):
        K, N = self.K, self.N
        e = np.zeros((n, K), np.int32) if record_energy else None
        b = np.zeros((n, K), np.uint32) if record_bits else None
        ss = np.zeros((K, N), np.int64) if record_spins else None
        lib().orc_sweeps(self._c, n, swap_every,
                         _ptr(e) if e is not None else None,
                         _ptr(b) if b is not None else None,
                         _ptr(ss) if ss is not None else None)
        return {"energy": e, "bits": b, "slot_spin_sum": ss}

    def swap_round(self, parity):
        lib().orc_swap_round(self._c, parity)

    def spins(self):
        out = np.empty((self.K, self.N), np.int8)
        lib().orc_get_spins(self._c, _ptr(out))
        return out

    def fields(self):
        out = np.empty((self.K, self.N), np.int32)
        lib().orc_get_fields(self._c, _ptr(out))
        return out

    def energy(self):
        out = np.empty(self.K, np.int64)
        lib().orc_get_energy(self._c, _ptr(out))
        return out

    def labels(self):
        t = np.empty(self.K, np.int32)
        w = np.empty(self.K, np.int32)
        lib().orc_get_labels(self._c, _ptr(t), _ptr(w))
        return t, w

    def mt(self):
        win = np.empty((self.K, 624), np.uint32)
        used = np.empty(self.K, np.int64)
        lib().orc_get_mt(self._c, _ptr(win), _ptr(used))
        return win, used

    def swap_mt(self):
        win = np.empty(624, np.uint32)
        used = np.zeros(1, np.int64)
        lib().orc_get_swap_mt(self._c, _ptr(win), _ptr(used))
        return win, int(used[0])

    def counters(self):
        f = np.empty(self.K, np.uint64)
        a = np.empty(self.K, np.uint64)
        c = np.empty(self.K, np.uint64)
        n = np.empty(self.K, np.uint64)
        lib().orc_get_counters(self._c, _ptr(f), _ptr(a), _ptr(c), _ptr(n))
        return {"flips": f, "swap_att": a, "swap_acc": c, "swap_near": n, "near": int(n.sum())}

    def energy_of(self, w):
        return int(lib().orc_energy_of(self._c, w))

    def check_fields(self):
        return int(lib().orc_check_fields(self._c))

    def set_spins(self, w, s):
        s = np.ascontiguousarray(s, np.int8)
        lib().orc_set_spins(self._c, w, _ptr(s))

    def set_two_field(self, is_tau, a, c):
        """Switch to the two-field form: tau edges flagged by is_tau (edge order of the
        constructor), slot weights a[K], c[K]."""
        t = np.ascontiguousarray(is_tau, np.uint8)
        a_ = np.ascontiguousarray(a, np.float64)
        c_ = np.ascontiguousarray(c, np.float64)
        assert len(a_) == self.K and len(c_) == self.K
        self._keep += [t, a_, c_]
        if lib().orc_set_two_field(self._c, _ptr(t), len(t), _ptr(a_), _ptr(c_)) != 0:
            raise ValueError("oracle rejected the two-field form")
        return self

    def set_pairs(self, S, M, pair_seeds):
        """Switch to the layer-pair order (Sec. 3.2, Fig. 12c): M/2 generators per walker,
        seeded pair_seeds[w * M/2 + t]; the initial spins are redrawn from them."""
        ps = np.ascontiguousarray(pair_seeds, np.uint32)
        assert ps.shape == (self.K * (M // 2),)
        self._keep.append(ps)
        if lib().orc_set_pairs(self._c, int(S), int(M), _ptr(ps)) != 0:
            raise ValueError("oracle rejected the layer-pair order")
        self.pM = int(M)
        return self

    def pair_mt(self):
        n = self.K * (self.pM // 2)
        win = np.empty((n, 624), np.uint32)
        used = np.empty(n, np.int64)
        lib().orc_get_pair_mt(self._c, _ptr(win), _ptr(used))
        return win, used

    def bond(self):
        out = np.empty(self.K, np.int64)
        lib().orc_get_bond(self._c, _ptr(out))
        return out

    def bond_of(self, w):
        return int(lib().orc_bond_of(self._c, w))

    def tau_fields(self):
        out = np.empty((self.K, self.N), np.int32)
        lib().orc_get_tau_fields(self._c, _ptr(out))
        return out

    def set_acceptance(self, kind):
        """Flip test: ACCEPT_EXACT (exp), ACCEPT_FAST or ACCEPT_ACCURATE (Sec. 2.4 approximations)."""
        lib().orc_set_acceptance(self._c, int(kind))
        return self

    @property
    def sweeps_done(self):
        return int(lib().orc_sweeps_done(self._c))

    @property
    def rounds_done(self):
        return int(lib().orc_rounds_done(self._c))


def run_many(chains, n, swap_every, n_threads):
    arr = (C.c_void_p * len(chains))(*[c._c for c in chains])
    lib().orc_run_many(len(chains), arr, n, swap_every, n_threads)


def workload_chains(workload, idx=None):
    """Oracle chains for systems `idx` of a workload, with the workload's seeds."""
    idx = range(len(workload.systems)) if idx is None else idx
    out = []
    for s in idx:
        b0, b1 = workload.walker_base[s], workload.walker_base[s + 1]
        out.append(Chain.from_system(workload.systems[s], workload.walker_seeds[b0:b1],
                                     int(workload.swap_seeds[s])))
    return out
