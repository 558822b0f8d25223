"""Two-field form (the QMC models' separate in-slice and tau fields) on the GPU
against the oracle's two-field chains, element by element: spins, MT19937
windows, running cost, tau-bond sums, labels, swap streams and counters."""
import dataclasses

import numpy as np
import pytest

import oracle
from gen import Workload, make_chimera_system, make_workload

from .gpu_util import chains_for, compare_system, make_state, say

pytestmark = pytest.mark.gpu


def _weights(wl, gamma):
    """Per-slot Trotter weights of every system (its own M), concatenated in slot order."""
    a, c = [], []
    for s in wl.systems:
        sa, sc = oracle.trotter_weights(s.beta, s.M, gamma)
        a.append(sa)
        c.append(sc)
    return np.concatenate(a), np.concatenate(c)


def _two_field_chains(wl, idx, a, c, kind=0):
    chains = chains_for(wl, idx)
    for s, ch in zip(idx, chains):
        b0, b1 = int(wl.walker_base[s]), int(wl.walker_base[s + 1])
        ch.set_acceptance(kind)
        ch.set_two_field(oracle.tau_edge_mask(wl.systems[s]), a[b0:b1], c[b0:b1])
    return chains


def _compare(st, s, ch, what):
    near = compare_system(st, s, ch, what)
    g = st.graph
    w0, w1 = int(g.walker_base[s]), int(g.walker_base[s + 1])
    assert np.array_equal(st.host("bond")[w0:w1].astype(np.int64), ch.bond()), f"{what} system {s}: bond sums"
    return near


def _run(wl, idx, a, c, steps, swap_every=1, kind=0, shape=None):
    say(wl.name, "two-field", "compare", list(idx), "steps", steps, "swap_every", swap_every, "kind", kind,
        "shape", shape)
    g, st = make_state(wl)
    if kind:
        g.set_acceptance(kind)
    g.set_two_field(a, c)
    if shape is not None:
        g.set_launch(0, *shape)
    chains = _two_field_chains(wl, idx, a, c, kind)
    for s, ch in zip(idx, chains):
        _compare(st, s, ch, "after init")
    for n in steps:
        st.sweep(n, swap_every)
        for s, ch in zip(idx, chains):
            ch.sweeps(n, swap_every)
            _compare(st, s, ch, f"after {st.sweeps} sweeps")
    obs = st.observables().cpu().numpy()
    assert np.array_equal(obs[:, 0], obs[:, 2]), "running cost = recomputed cost"
    assert np.array_equal(obs[:, 4], obs[:, 5]), "running tau-bond sum = recomputed"
    return g, st


MIXED = [("L2 ring M=8 K=8", make_chimera_system(2, 8, 41, 8)),
         ("L3 ring M=5 K=7 (ragged rows)", make_chimera_system(3, 5, 42, 7)),
         ("L1 open M=2 K=5", make_chimera_system(1, 2, 43, 5, ring=False)),
         ("L4 open M=6 K=6", make_chimera_system(4, 6, 44, 6, ring=False)),
         ("L8 ring M=4 K=3", make_chimera_system(8, 4, 45, 3))]


@pytest.mark.parametrize("name,sysm", MIXED, ids=[m[0] for m in MIXED])
def test_two_field_parity_shapes(name, sysm):
    wl = Workload(name, [sysm], 0, 1)
    a, c = _weights(wl, 0.9)
    _run(wl, [0], a, c, [1, 2, 9])


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_two_field_parity_mixed_batch(kind):
    """Several template sizes in one graph, Trotter weights, every flip-test variant."""
    wl = Workload("two-field batch", [m[1] for m in MIXED], 0, 1)
    a, c = _weights(wl, 1.3)
    _run(wl, list(range(len(MIXED))), a, c, [1, 4, 15], kind=kind)


@pytest.mark.parametrize("swap_every,steps", [(0, [3, 4]), (3, [2, 5, 7])])
def test_two_field_swap_cadence(swap_every, steps):
    wl = Workload("cadence", [make_chimera_system(2, 6, 46, 6)], 0, swap_every)
    a, c = _weights(wl, 0.5)
    _run(wl, [0], a, c, steps, swap_every=swap_every)


def test_two_field_unit_tau_couplings():
    """The transverse-field Ising reading: every tau coupling +1."""
    sysm = dataclasses.replace(make_chimera_system(4, 16, 47, 12), J_tau=np.ones(128, np.int8))
    wl = Workload("unit tau", [sysm], 0, 1)
    a, c = _weights(wl, 2.0)
    _run(wl, [0], a, c, [1, 20])


@pytest.mark.parametrize("tpw,G", [(16, 9), (16, 4), (32, 1), (64, 2), (128, 1)])
def test_two_field_launch_shapes(tpw, G):
    """Every launch shape (columns per thread 1..8, wavefront and workgroup sync)."""
    wl = Workload("shape S=128", [make_chimera_system(4, 9, 48, 9)], 0, 1)
    a, c = _weights(wl, 0.7)
    _run(wl, [0], a, c, [2, 1], shape=(tpw, G))


def test_two_field_with_equal_weights_is_the_one_field_chain():
    """a = c = beta (dyadic): the two-field GPU chain equals the one-field GPU chain."""
    beta = np.array([0.125, 0.25, 0.375, 0.5, 0.75, 1.0])
    systems = [dataclasses.replace(make_chimera_system(2, 8, 49 + i, 6), beta=beta.copy()) for i in range(3)]
    wl = Workload("equal weights", systems, 0, 1)
    g1, st1 = make_state(wl)
    g2, st2 = make_state(wl)
    b = np.concatenate([s.beta for s in systems])
    g2.set_two_field(b, b)
    for n in (1, 5, 30):
        st1.sweep(n, 1)
        st2.sweep(n, 1)
        for name in ("spins", "mt", "energy", "temp_of", "walker_at", "swap_mt", "flips", "swap_acc"):
            assert np.array_equal(st1.host(name), st2.host(name)), name


def test_two_field_graph_replay_and_switch_back():
    """Captured two-field loops replay bit-exactly; switching back restores the one-field form."""
    import torch
    wl = Workload("replay", [make_chimera_system(2, 8, 50, 8), make_chimera_system(3, 6, 51, 5)], 0, 1)
    a, c = _weights(wl, 1.1)
    g, st = make_state(wl)
    g.set_two_field(a, c)
    chains = _two_field_chains(wl, [0, 1], a, c)
    rp = st.capture(10, 1)
    for _ in range(3):
        rp.launch()
        rp.stream.synchronize()
        torch.cuda.synchronize()
        st.observables()  # eager work between replays
        for s, ch in enumerate(chains):
            ch.sweeps(10, 1)
            _compare(st, s, ch, f"replay, {st.sweeps} sweeps")
    assert not any(b["ladder"] for b in g.buckets())
    g.set_two_field(None, None)
    st.sweep(3, 1)
    obs = st.observables().cpu().numpy()
    assert np.array_equal(obs[:, 0], obs[:, 2])


def test_two_field_refused_for_cell_moves():
    import paper_1004_0024_amd as pa
    wl = Workload("refuse", [make_chimera_system(2, 4, 52, 4)], 0, 1)
    a, c = _weights(wl, 1.0)
    g, st = make_state(wl)
    g.set_two_field(a, c)
    with pytest.raises(pa.IsingError) as e:
        st.heatbath_cells(1, 0)
    assert e.value.code == -5


def test_two_field_config_B_full_size_sampled():
    """The throughput workload in the two-field form (unit tau couplings, gamma = 1):
    the full 256-system graph in the launch shape the benchmark times, two systems compared."""
    wl = make_workload("B")
    wl.systems = [dataclasses.replace(s, J_tau=np.ones(s.S, np.int8)) for s in wl.systems]
    a, c = _weights(wl, 1.0)
    _run(wl, [0, 255], a, c, [1, 2])


def test_switch_to_two_field_mid_run():
    """One-field sweeps, then the two-field form on the same state (tau-bond sums refreshed),
    against oracle chains that switch at the same sweep."""
    wl = Workload("switch", [make_chimera_system(2, 8, 53, 8), make_chimera_system(4, 4, 54, 6)], 0, 1)
    say(wl.name, "one-field then two-field")
    g, st = make_state(wl)
    chains = chains_for(wl, [0, 1])
    st.sweep(7, 1)
    for s, ch in enumerate(chains):
        ch.sweeps(7, 1)
        compare_system(st, s, ch, "one-field")
    a, c = _weights(wl, 0.8)
    g.set_two_field(a, c)
    st.refresh_energies()
    for s, ch in enumerate(chains):
        b0, b1 = int(wl.walker_base[s]), int(wl.walker_base[s + 1])
        ch.set_two_field(oracle.tau_edge_mask(wl.systems[s]), a[b0:b1], c[b0:b1])
        _compare(st, s, ch, "after the switch")
    for n in (1, 6):
        st.sweep(n, 1)
        for s, ch in enumerate(chains):
            ch.sweeps(n, 1)
            _compare(st, s, ch, f"two-field, {st.sweeps} sweeps")


def test_two_field_autotune_keeps_the_chain():
    """Launch shapes tuned in the two-field form (no whole-ladder shapes) leave the chain unchanged."""
    import paper_1004_0024_amd as pa
    wl = Workload("tune two-field", [make_chimera_system(4, 8, 55, 8), make_chimera_system(2, 8, 56, 16)], 0, 1)
    say(wl.name)
    a, c = _weights(wl, 0.6)
    g = pa.Graph(wl.systems)
    g.set_two_field(a, c)
    scratch = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    rows = g.autotune(scratch, reps=2)
    assert len(rows) > 4 and all(r["ns_per_sweep"] > 0 for r in rows)
    assert not any(b["ladder"] for b in g.buckets())
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    chains = _two_field_chains(wl, [0, 1], a, c)
    st.sweep(6, 1)
    for s, ch in enumerate(chains):
        ch.sweeps(6, 1)
        _compare(st, s, ch, "after autotune")
