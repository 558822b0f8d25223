"""Helpers for the GPU parity tests: run the HIP path and the oracle on the same
seeded inputs and compare them element by element."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


def make_state(workload):
    import paper_1004_0024_amd as pa
    g = pa.Graph(workload.systems)
    st = pa.State(g).init(workload.walker_seeds, workload.swap_seeds)
    return g, st


def compare_system(st, s, ch, what=""):
    """Bit-exact comparison of system s of the GPU state with oracle chain `ch`."""
    g = st.graph
    w0, w1 = int(g.walker_base[s]), int(g.walker_base[s + 1])
    gs = st.spins_pm([s])[0]
    os_ = ch.spins()
    if not np.array_equal(gs, os_):
        bad = np.argwhere(gs != os_)
        raise AssertionError(f"{what} system {s}: {len(bad)} spins differ, first {bad[:5].tolist()}")
    win, used = ch.mt()
    assert np.array_equal(st.mt_window()[w0:w1], win), f"{what} system {s}: MT windows differ"
    assert np.array_equal(st.host("energy")[w0:w1].astype(np.int64), ch.energy()), \
        f"{what} system {s}: energies differ"
    t, wa = ch.labels()
    assert np.array_equal(st.host("temp_of")[w0:w1], t), f"{what} system {s}: temp_of differs"
    slot0 = w0  # slots are laid out like walkers (K per system)
    assert np.array_equal(st.host("walker_at")[slot0:slot0 + (w1 - w0)], wa), f"{what} system {s}: walker_at"
    sw, sused = ch.swap_mt()
    assert np.array_equal(st.swap_window()[s], sw), f"{what} system {s}: swap stream differs"
    c = ch.counters()
    assert np.array_equal(st.host("flips")[w0:w1].astype(np.uint64), c["flips"]), f"{what} flips"
    assert np.array_equal(st.host("swap_att")[slot0:slot0 + (w1 - w0)].astype(np.uint64), c["swap_att"])
    assert np.array_equal(st.host("swap_acc")[slot0:slot0 + (w1 - w0)].astype(np.uint64), c["swap_acc"])
    gnear = st.host("swap_near")[slot0:slot0 + (w1 - w0)].astype(np.uint64)
    assert np.array_equal(gnear, c["swap_near"]), \
        f"{what} system {s}: near-threshold swap counts differ: gpu {gnear.tolist()} oracle {c['swap_near'].tolist()}"
    if c["near"]:
        say(f"{what} system {s}: near-threshold swap decisions at pairs", np.nonzero(c["swap_near"])[0].tolist())
    return c["near"]


def chains_for(workload, idx):
    return oracle.workload_chains(workload, idx)
