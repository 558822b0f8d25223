"""ctypes binding of the C ABI (include/ising.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_FILE = os.path.join(HERE, "libising.so")

ISING_N_STATS = 8
STAT_NEAR, STAT_WAVE_STEPS, STAT_WAVE_FLIP, STAT_ATTEMPTS = 0, 1, 2, 3
_ERRORS = {-1: "E_INVAL", -2: "E_RANGE", -3: "E_SIZE", -4: "E_HIP", -5: "E_STATE"}


class IsingError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class SystemDesc(C.Structure):
    _fields_ = [
        ("spins_per_slice", C.c_int32), ("n_slices", C.c_int32), ("ring", C.c_int32),
        ("n_edges", C.c_int32), ("edge_u", C.c_void_p), ("edge_v", C.c_void_p),
        ("edge_J", C.c_void_p), ("h", C.c_void_p), ("J_tau", C.c_void_p),
        ("n_temps", C.c_int32), ("beta", C.c_void_p),
    ]


class StateStruct(C.Structure):
    _fields_ = [
        ("spins", C.c_void_p), ("mt", C.c_void_p), ("energy", C.c_void_p), ("temp_of", C.c_void_p),
        ("walker_at", C.c_void_p), ("swap_mt", C.c_void_p), ("flips", C.c_void_p),
        ("swap_att", C.c_void_p), ("swap_acc", C.c_void_p), ("stats", C.c_void_p), ("wsteps", C.c_void_p),
        ("bond", C.c_void_p), ("swap_near", C.c_void_p), ("sweeps", C.c_int64), ("rounds", C.c_int64),
    ]


_lib = None


def lib_path() -> str:
    return _LIB_FILE


def lib():
    """The loaded libising.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_FILE):
            raise ImportError(f"{_LIB_FILE} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(_LIB_FILE)
        P, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "ising_graph_bytes": ([P, i32, P], i32),
            "ising_load_graph": ([P, i32, P, sz, P, P], i32),
            "ising_free_graph": ([P], None),
            "ising_graph_info": ([P, P, i32], i32),
            "ising_spin_layout": ([P, P, P], i32),
            "ising_state_sizes": ([P, P], i32),
            "ising_init_state": ([P, P, P, P, P], i32),
            "ising_sweep": ([P, P, i32, i32, P, P], i32),
            "pt_swap": ([P, P, i32, P], i32),
            "ising_observables": ([P, P, P, P], i32),
            "ising_stats": ([P, P, P, P], i32),
            "ising_record_slots": ([P, P, P, P], i32),
            "ising_threshold_row": ([C.c_double, i32, P], i32),
            "ising_level_offsets": ([P, P, P], i32),
            "ising_last_error": ([], C.c_char_p),
            "ising_n_buckets": ([P], i32),
            "ising_bucket_info": ([P, i32, P, i32], i32),
            "ising_set_launch": ([P, i32, i32, i32, P], i32),
            "ising_capture": ([P, P, i32, i32, P, P, P], i32),
            "ising_replay_launch": ([P, P, P], i32),
            "ising_replay_free": ([P], None),
            "ising_autotune": ([P, P, i32, P, P, i32], i32),
            "ising_mlp_pack": ([P, P], i32),
            "ising_mlp_forward": ([P, P, i32, P, P], i32),
            "ising_mlp_grad": ([P, P, P, i32, P, P], i32),
            "ising_mlp_grad_noalloc": ([P, P, P, i32, P, P], i32),
            "ising_mlp_adam": ([P, C.c_float, P], i32),
            "ising_collect_cells": ([P, P, i64, i64, i32, P, P, P], i32),
            "ising_propose_cells": ([P, P, P, C.c_uint64, i64, P, P], i32),
            "ising_heatbath_cells": ([P, P, C.c_uint64, i64, P, P], i32),
            "ising_acceptance_row": ([C.c_double, i32, i32, P], i32),
            "ising_set_acceptance": ([P, i32, P], i32),
            "ising_refresh_energies": ([P, P, P], i32),
            "ising_set_two_field": ([P, P, P, P], i32),
            "ising_two_field_row": ([C.c_double, C.c_double, i32, i32, i32, P], i32),
            "ising_trotter_weights": ([P, i32, i32, C.c_double, P, P], i32),
            "ising_pairs_words": ([P, P], i32),
            "ising_pairs_init": ([P, P, P, P, P, P], i32),
            "ising_pairs_sweep": ([P, P, P, i32, i32, P], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise IsingError(rc, lib().ising_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _descs(systems):
    """ising_system_desc array for objects with S, M, ring, eu, ev, eJ, h, J_tau, beta."""
    keep, arr = [], (SystemDesc * len(systems))()
    for i, s in enumerate(systems):
        eu = np.ascontiguousarray(s.eu, np.int32)
        ev = np.ascontiguousarray(s.ev, np.int32)
        eJ = np.ascontiguousarray(s.eJ, np.int8)
        h = np.ascontiguousarray(s.h, np.int8)
        jt = np.ascontiguousarray(s.J_tau if s.J_tau is not None else np.zeros(s.S, np.int8), np.int8)
        beta = np.ascontiguousarray(s.beta, np.float64)
        keep += [eu, ev, eJ, h, jt, beta]
        arr[i] = SystemDesc(int(s.S), int(s.M), int(bool(s.ring)), int(eu.shape[0]), _np_ptr(eu), _np_ptr(ev),
                            _np_ptr(eJ), _np_ptr(h), _np_ptr(jt), int(beta.shape[0]), _np_ptr(beta))
    return arr, keep


def threshold_row(beta: float, dmax: int) -> np.ndarray:
    out = np.zeros(dmax + 1, np.uint32)
    _check(lib().ising_threshold_row(float(beta), int(dmax), _np_ptr(out)))
    return out


ACCEPT_EXACT, ACCEPT_FAST, ACCEPT_ACCURATE = 0, 1, 2


def acceptance_row(beta: float, dmax: int, kind: int) -> np.ndarray:
    """Threshold row of a flip-test variant (host only)."""
    out = np.zeros(dmax + 1, np.uint32)
    _check(lib().ising_acceptance_row(C.c_double(beta), int(dmax), int(kind), _np_ptr(out)))
    return out


def two_field_row(a: float, c: float, ds: int, dt: int, kind: int = ACCEPT_EXACT) -> np.ndarray:
    """Two-field threshold row of one slot (host only): [2 ds + 1, 2 dt + 1] over (d_sp, d_t)."""
    out = np.zeros((2 * ds + 1) * (2 * dt + 1), np.uint32)
    _check(lib().ising_two_field_row(C.c_double(a), C.c_double(c), int(ds), int(dt), int(kind), _np_ptr(out)))
    return out.reshape(2 * ds + 1, 2 * dt + 1)


def trotter_weights(beta, M: int, gamma: float):
    """Slot weights (a, c) of a transverse field gamma over M slices (host only)."""
    b = np.ascontiguousarray(beta, np.float64)
    a = np.zeros_like(b)
    c = np.zeros_like(b)
    _check(lib().ising_trotter_weights(_np_ptr(b), int(b.shape[0]), int(M), C.c_double(gamma), _np_ptr(a), _np_ptr(c)))
    return a, c


def level_offsets(system):
    arr, keep = _descs([system])
    f = np.zeros(int(system.S), np.int32)
    depth = C.c_int32(0)
    _check(lib().ising_level_offsets(C.byref(arr[0]), _np_ptr(f), C.byref(depth)))
    return f, int(depth.value)


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Graph:
    """Loaded systems: device tables in a torch buffer + the library handle."""

    def __init__(self, systems, device="cuda"):
        import torch
        self.systems = list(systems)
        arr, keep = _descs(self.systems)
        nbytes = C.c_size_t(0)
        _check(lib().ising_graph_bytes(arr, len(self.systems), C.byref(nbytes)))
        self.tables = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=device)
        base = self.tables.data_ptr()
        off = (-base) % 256
        self._handle = C.c_void_p()
        _check(lib().ising_load_graph(arr, len(self.systems), C.c_void_p(base + off), nbytes.value,
                                      _stream(), C.byref(self._handle)))
        info = np.zeros(6, np.int64)
        _check(lib().ising_graph_info(self._handle, _np_ptr(info), 6))
        self.n_sys, self.R, self.slots, self.spin_words, self.attempts_per_sweep, self.max_levels = \
            (int(x) for x in info)
        self.spin_word = np.zeros(self.R, np.int64)
        self.row_words = np.zeros(self.n_sys, np.int32)
        _check(lib().ising_spin_layout(self._handle, _np_ptr(self.spin_word), _np_ptr(self.row_words)))
        Ks = np.array([len(s.beta) for s in self.systems], np.int64)
        self.walker_base = np.concatenate([[0], np.cumsum(Ks)])

    def __del__(self):
        h = getattr(self, "_handle", None)
        if h and _lib is not None:
            _lib.ising_free_graph(h)
            self._handle = None

    @property
    def handle(self):
        return self._handle

    _BUCKET_KEYS = ["S", "systems", "walkers", "attempts", "tpw", "G", "cpt", "threads", "lds", "tiles", "ladder",
                    "stream", "work"]

    def buckets(self):
        out = []
        n = len(self._BUCKET_KEYS)
        for b in range(lib().ising_n_buckets(self._handle)):
            v = np.zeros(n, np.int64)
            _check(lib().ising_bucket_info(self._handle, b, _np_ptr(v), n))
            out.append(dict(zip(self._BUCKET_KEYS, (int(x) for x in v))))
        return out

    def set_acceptance(self, kind):
        """Flip-test variant for later sweeps: ACCEPT_EXACT, ACCEPT_FAST or ACCEPT_ACCURATE."""
        _check(lib().ising_set_acceptance(self.handle, int(kind), _stream()))

    def set_two_field(self, a=None, c=None):
        """Two-field form with slot weights a[slots], c[slots] (None, None: one-field form)."""
        if a is None and c is None:
            _check(lib().ising_set_two_field(self.handle, None, None, _stream()))
            return
        a_ = np.ascontiguousarray(a, np.float64)
        c_ = np.ascontiguousarray(c, np.float64)
        assert a_.shape == (self.slots,) and c_.shape == (self.slots,)
        _check(lib().ising_set_two_field(self.handle, _np_ptr(a_), _np_ptr(c_), _stream()))

    def set_launch(self, bucket, tpw, walkers_per_group):
        _check(lib().ising_set_launch(self._handle, int(bucket), int(tpw), int(walkers_per_group), _stream()))

    def autotune(self, scratch_state, reps=3):
        """Pick the fastest launch shape per bucket, timed on `scratch_state`."""
        rows = 64 * max(1, len(self.buckets()))
        rep = np.zeros((rows, 4), np.int64)
        n = lib().ising_autotune(self._handle, C.byref(scratch_state._s), int(reps), _stream(), _np_ptr(rep), rows)
        if n < 0:
            _check(n)
        return [dict(bucket=int(r[0]), tpw=int(r[1]), G=int(r[2]), ns_per_sweep=int(r[3])) for r in rep[:n]]


class State:
    """Chain state in torch device tensors, walker-major."""

    _FIELDS = ["spins", "mt", "energy", "temp_of", "walker_at", "swap_mt", "flips", "swap_att", "swap_acc",
               "stats", "wsteps", "bond", "swap_near"]

    def __init__(self, graph: Graph):
        import torch
        self.graph = graph
        counts = np.zeros(len(self._FIELDS), np.int64)
        _check(lib().ising_state_sizes(graph.handle, _np_ptr(counts)))
        dev = graph.tables.device
        dt = {"spins": torch.int32, "mt": torch.int32, "energy": torch.int32, "temp_of": torch.int32,
              "walker_at": torch.int32, "swap_mt": torch.int32, "flips": torch.int64, "swap_att": torch.int64,
              "swap_acc": torch.int64, "stats": torch.int64, "wsteps": torch.int64, "bond": torch.int32,
              "swap_near": torch.int64}
        self.t = {}
        for name, n in zip(self._FIELDS, counts):
            self.t[name] = torch.zeros(max(int(n), 1), dtype=dt[name], device=dev)
        self._s = StateStruct(*[C.c_void_p(self.t[n].data_ptr()) for n in self._FIELDS], -1, 0)

    @property
    def sweeps(self):
        return int(self._s.sweeps)

    @property
    def rounds(self):
        return int(self._s.rounds)

    def init(self, walker_seeds, swap_seeds):
        ws = np.ascontiguousarray(walker_seeds, np.uint32)
        ss = np.ascontiguousarray(swap_seeds, np.uint32)
        assert ws.shape[0] == self.graph.R and ss.shape[0] == self.graph.n_sys
        _check(lib().ising_init_state(self.graph.handle, C.byref(self._s), _np_ptr(ws), _np_ptr(ss), _stream()))
        return self

    def copy_from(self, other):
        """Make this state (of the same graph) a copy of `other`: device arrays and counters."""
        assert other.graph is self.graph
        for name in self._FIELDS:
            self.t[name].copy_(other.t[name])
        self._s.sweeps, self._s.rounds = other._s.sweeps, other._s.rounds
        return self

    def sweep(self, n_sweeps, swap_every=1, record=False):
        import torch
        e = None
        if record:
            e = torch.zeros((n_sweeps, self.graph.slots), dtype=torch.int32, device=self.graph.tables.device)
        _check(lib().ising_sweep(self.graph.handle, C.byref(self._s), int(n_sweeps), int(swap_every),
                                 C.c_void_p(e.data_ptr()) if e is not None else None, _stream()))
        return e

    def capture(self, n_sweeps, swap_every=1, stream=None, record=False):
        """A HIP graph of `n_sweeps` sweeps from the current counters (see Replay)."""
        return Replay(self, n_sweeps, swap_every, stream, record)

    def record(self, e_row):
        """e_row[slots] (device int32) = energy of the walker at each slot."""
        _check(lib().ising_record_slots(self.graph.handle, C.byref(self._s), C.c_void_p(e_row.data_ptr()), _stream()))

    def collect_cells(self, n, stride=1, offset=0):
        """Training rows (x [n,17] float32, y [n] uint8) from the current spins."""
        import torch
        dev = self.graph.tables.device
        x = torch.empty((n, 17), dtype=torch.float32, device=dev)
        y = torch.empty(n, dtype=torch.uint8, device=dev)
        _check(lib().ising_collect_cells(self.graph.handle, C.byref(self._s), int(stride), int(offset), int(n),
                                         C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), _stream()))
        return x, y

    def propose_cells(self, net, key, pass_index, moves=None):
        """One pass of learned cell moves (all colour classes)."""
        _check(lib().ising_propose_cells(self.graph.handle, C.byref(self._s), C.byref(net._s), C.c_uint64(key),
                                         int(pass_index), C.c_void_p(moves.data_ptr()) if moves is not None else None,
                                         _stream()))

    def heatbath_cells(self, key, pass_index, moves=None):
        """One pass of exact heat-bath cell moves (all colour classes)."""
        _check(lib().ising_heatbath_cells(self.graph.handle, C.byref(self._s), C.c_uint64(key), int(pass_index),
                                          C.c_void_p(moves.data_ptr()) if moves is not None else None, _stream()))

    # ---- layer-pair order (the paper's GPU layout, Sec. 3.2) ----
    def pairs_init(self, pair_seeds, swap_seeds):
        """Start the layer-pair chain: generator lanes seeded from pair_seeds (one per
        pair of slices of every walker, walker-major), swap streams from swap_seeds."""
        import torch
        words = C.c_int64(0)
        _check(lib().ising_pairs_words(self.graph.handle, C.byref(words)))
        self.pair_lanes = int(words.value) // 624
        self.t["pair_mt"] = torch.zeros(max(int(words.value), 1), dtype=torch.int32, device=self.graph.tables.device)
        ps = np.ascontiguousarray(pair_seeds, np.uint32)
        ss = np.ascontiguousarray(swap_seeds, np.uint32)
        assert ps.shape == (self.pair_lanes,) and ss.shape == (self.graph.n_sys,)
        _check(lib().ising_pairs_init(self.graph.handle, C.byref(self._s), C.c_void_p(self.t["pair_mt"].data_ptr()),
                                      _np_ptr(ps), _np_ptr(ss), _stream()))
        return self

    def pairs_sweep(self, n_sweeps, swap_every=1):
        _check(lib().ising_pairs_sweep(self.graph.handle, C.byref(self._s), C.c_void_p(self.t["pair_mt"].data_ptr()),
                                       int(n_sweeps), int(swap_every), _stream()))

    def pair_windows(self, system):
        """[lanes of `system`][624] words of its generator lanes, oldest first (each lane
        of the system has delivered 2 S (1 + sweeps) outputs).  Storage: slot k of lane l
        at ((k // 4) * lanes + l) * 4 + k % 4."""
        l0 = 0
        for sysm in self.graph.systems[:system]:
            l0 += len(sysm.beta) * (int(sysm.M) // 2)
        sysm = self.graph.systems[system]
        lanes = len(sysm.beta) * (int(sysm.M) // 2)
        blocks = self.t["pair_mt"][: 624 * self.pair_lanes].view(156, self.pair_lanes, 4)[:, l0:l0 + lanes, :]
        a = blocks.cpu().numpy().view(np.uint32).transpose(1, 0, 2).reshape(lanes, 624)
        n = 2 * int(sysm.S) * (1 + self.sweeps)
        return np.ascontiguousarray(a[:, (n + np.arange(624)) % 624])

    def refresh_energies(self):
        """Recompute the running cost and tau-bond sum of every walker from its spins."""
        _check(lib().ising_refresh_energies(self.graph.handle, C.byref(self._s), _stream()))

    def swap(self, parity):
        _check(lib().pt_swap(self.graph.handle, C.byref(self._s), int(parity), _stream()))

    def stats(self):
        """Totals: near-threshold swaps, wavefront steps, steps with a flip, attempts,
        flips, swap attempts, accepted swaps."""
        out = np.zeros(ISING_N_STATS, np.uint64)
        _check(lib().ising_stats(self.graph.handle, C.byref(self._s), _np_ptr(out), _stream()))
        keys = ["near", "wave_steps", "wave_flip_steps", "attempts", "flips", "swap_att", "swap_acc"]
        return {k: int(v) for k, v in zip(keys, out)}

    def observables(self):
        import torch
        obs = torch.zeros((self.graph.R, 6), dtype=torch.int32, device=self.graph.tables.device)
        _check(lib().ising_observables(self.graph.handle, C.byref(self._s), C.c_void_p(obs.data_ptr()), _stream()))
        return obs

    # ---- host views of the device state (for tests and reports) ----
    def host(self, name):
        return self.t[name].cpu().numpy()

    def spins_pm(self, systems=None):
        """Spins as +-1 int8 arrays, one [K, N] array per requested system."""
        g = self.graph
        words = self.host("spins").view(np.uint32)
        out = []
        for s in (range(g.n_sys) if systems is None else systems):
            sysm = g.systems[s]
            S, M, K = int(sysm.S), int(sysm.M), len(sysm.beta)
            SW = int(g.row_words[s])
            w0 = int(g.walker_base[s])
            base = g.spin_word[w0]
            blk = words[base: base + K * M * SW].reshape(K, M, SW)
            bits = np.unpackbits(blk.view(np.uint8).reshape(K, M, SW * 4), axis=2, bitorder="little")[:, :, :S]
            out.append((bits.astype(np.int8) * 2 - 1).reshape(K, S * M))
        return out

    def mt_window(self):
        return self.host("mt").view(np.uint32).reshape(self.graph.R, 624)

    def swap_window(self):
        return self.host("swap_mt").view(np.uint32).reshape(self.graph.n_sys, 624)


class Replay:
    """A captured sweep loop; launch() replays it on the capture stream."""

    def __init__(self, state, n_sweeps, swap_every, stream, record):
        import torch
        self.state = state
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.e = None
        if record:
            self.e = torch.zeros((n_sweeps, state.graph.slots), dtype=torch.int32,
                                 device=state.graph.tables.device)
        self._h = C.c_void_p()
        torch.cuda.current_stream().synchronize()
        _check(lib().ising_capture(state.graph.handle, C.byref(state._s), int(n_sweeps), int(swap_every),
                                   C.c_void_p(self.e.data_ptr()) if self.e is not None else None,
                                   C.c_void_p(self.stream.cuda_stream), C.byref(self._h)))

    def launch(self):
        _check(lib().ising_replay_launch(self._h, C.byref(self.state._s), C.c_void_p(self.stream.cuda_stream)))
        return self.e

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.ising_replay_free(h)
            self._h = None


class MlpStruct(C.Structure):
    _fields_ = [("w", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p), ("grad", C.c_void_p),
                ("part", C.c_void_p), ("wb", C.c_void_p), ("step", C.c_int64)]


MLP_PARAMS, MLP_PACKED, MLP_PARTS = 19848, 43008, 128


class Mlp:
    """Network of the learned cell proposal: FP32 master weights, Adam moments, BF16 copies."""

    def __init__(self, params, device="cuda"):
        import torch
        p = torch.as_tensor(np.asarray(params, np.float32)).to(device)
        assert p.numel() == MLP_PARAMS
        self.w = p.contiguous()
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.grad = torch.zeros_like(self.w)
        self.part = torch.zeros(MLP_PARTS * (MLP_PARAMS + 1), dtype=torch.float32, device=device)
        self.wb = torch.zeros(MLP_PACKED, dtype=torch.int16, device=device)
        self._s = MlpStruct(self.w.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.grad.data_ptr(),
                            self.part.data_ptr(), self.wb.data_ptr(), 0)
        _check(lib().ising_mlp_pack(C.byref(self._s), _stream()))

    def forward(self, x):
        import torch
        x = x.contiguous().float()
        out = torch.empty((x.shape[0], 8), dtype=torch.float32, device=x.device)
        _check(lib().ising_mlp_forward(C.byref(self._s), C.c_void_p(x.data_ptr()), int(x.shape[0]),
                                       C.c_void_p(out.data_ptr()), _stream()))
        return out

    def grad_step(self, x, y):
        """Writes self.grad; returns the mean loss (device scalar)."""
        import torch
        x = x.contiguous().float()
        y = y.contiguous().to(torch.uint8)
        loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        _check(lib().ising_mlp_grad(C.byref(self._s), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                    int(x.shape[0]), C.c_void_p(loss.data_ptr()), _stream()))
        return loss

    def grad_step_noalloc(self, x, y, loss):
        """The same step with the library's own partial-gradient rows (nothing allocated by
        the library; x, y and the device scalar `loss` are the caller's)."""
        _check(lib().ising_mlp_grad_noalloc(C.byref(self._s), C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                            int(x.shape[0]), C.c_void_p(loss.data_ptr()), _stream()))

    def adam(self, lr):
        _check(lib().ising_mlp_adam(C.byref(self._s), C.c_float(lr), _stream()))

    @property
    def steps(self):
        return int(self._s.step)
