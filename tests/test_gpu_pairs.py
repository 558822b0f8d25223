"""Layer-pair order (the paper's GPU layout, Sec. 3.2 and Fig. 12c) on the GPU
against the oracle's layer-pair chains, element by element: spins, every pair
generator's 624-word window, energies, labels, swap streams and counters."""
import numpy as np
import pytest

from gen import Workload, make_chimera_system, make_workload

from .gpu_util import chains_for, say

pytestmark = pytest.mark.gpu


def _pair_seeds(wl):
    lanes = sum(s.K * (s.M // 2) for s in wl.systems)
    return (100_000 + np.arange(lanes)).astype(np.uint32)


def _lane_base(wl):
    return np.concatenate([[0], np.cumsum([s.K * (s.M // 2) for s in wl.systems])]).astype(np.int64)


def _setup(wl, idx, kind=0):
    import paper_1004_0024_amd as pa
    g = pa.Graph(wl.systems)
    if kind:
        g.set_acceptance(kind)
    st = pa.State(g)
    seeds = _pair_seeds(wl)
    st.pairs_init(seeds, wl.swap_seeds)
    lb = _lane_base(wl)
    chains = chains_for(wl, idx)
    for s, ch in zip(idx, chains):
        ch.set_acceptance(kind)
        ch.set_pairs(wl.systems[s].S, wl.systems[s].M, seeds[lb[s]:lb[s + 1]])
    return g, st, chains, lb


def _compare(wl, st, s, ch, lb, what):
    g = st.graph
    w0, w1 = int(g.walker_base[s]), int(g.walker_base[s + 1])
    gs, os_ = st.spins_pm([s])[0], ch.spins()
    if not np.array_equal(gs, os_):
        bad = np.argwhere(gs != os_)
        raise AssertionError(f"{what} system {s}: {len(bad)} spins differ, first {bad[:5].tolist()}")
    win, used = ch.pair_mt()
    assert np.array_equal(st.pair_windows(s), win), f"{what} system {s}: pair generators"
    assert np.array_equal(st.host("energy")[w0:w1].astype(np.int64), ch.energy()), f"{what} system {s}: energies"
    t, wa = ch.labels()
    assert np.array_equal(st.host("temp_of")[w0:w1], t), f"{what} system {s}: temp_of"
    assert np.array_equal(st.host("walker_at")[w0:w1], wa), f"{what} system {s}: walker_at"
    assert np.array_equal(st.swap_window()[s], ch.swap_mt()[0]), f"{what} system {s}: swap stream"
    c = ch.counters()
    assert np.array_equal(st.host("flips")[w0:w1].astype(np.uint64), c["flips"]), f"{what} flips"
    assert np.array_equal(st.host("swap_att")[w0:w1].astype(np.uint64), c["swap_att"]), f"{what} swap_att"
    assert np.array_equal(st.host("swap_acc")[w0:w1].astype(np.uint64), c["swap_acc"]), f"{what} swap_acc"


def _run(wl, idx, steps, swap_every=1, kind=0):
    say(wl.name, "layer pairs", "compare", list(idx), "steps", steps, "swap_every", swap_every, "kind", kind)
    g, st, chains, lb = _setup(wl, idx, kind)
    for s, ch in zip(idx, chains):
        _compare(wl, st, s, ch, lb, "after init")
    for n in steps:
        st.pairs_sweep(n, swap_every)
        for s, ch in zip(idx, chains):
            ch.sweeps(n, swap_every)
            _compare(wl, st, s, ch, lb, f"after {st.sweeps} sweeps")
    obs = st.observables().cpu().numpy()
    assert np.array_equal(obs[:, 0], obs[:, 2]), "running cost = recomputed cost"
    return g, st


CASES = [("A: L2 M8 K16", make_chimera_system(2, 8, 0, 16)),
         ("L1 open M2 K5 (the canonical order)", make_chimera_system(1, 2, 71, 5, ring=False)),
         ("L3 ring M6 K7 (S=72, ragged words)", make_chimera_system(3, 6, 72, 7)),
         ("L4 open M6 K6", make_chimera_system(4, 6, 73, 6, ring=False)),
         ("L8 ring M4 K3", make_chimera_system(8, 4, 74, 3))]


@pytest.mark.parametrize("name,sysm", CASES, ids=[c[0] for c in CASES])
def test_pairs_parity_shapes(name, sysm):
    wl = Workload(name, [sysm], 0, 1)
    _run(wl, [0], [1, 2, 9])


def test_pairs_parity_mixed_batch():
    """Several template sizes and both ring and open slices in one graph (one launch per class)."""
    systems = [c[1] for c in CASES] + [make_chimera_system(2, 10, 76, 12), make_chimera_system(4, 2, 77, 9, ring=False)]
    wl = Workload("pairs batch", systems, 0, 1)
    _run(wl, list(range(len(systems))), [1, 5, 20])


@pytest.mark.parametrize("swap_every,steps", [(0, [3, 4]), (3, [2, 5, 7]), (2, [1, 1, 6])])
def test_pairs_swap_cadence(swap_every, steps):
    wl = Workload("cadence", [make_chimera_system(2, 6, 78, 6)], 0, swap_every)
    _run(wl, [0], steps, swap_every=swap_every)


@pytest.mark.parametrize("kind", [1, 2])
def test_pairs_approximate_acceptance(kind):
    wl = Workload("approx", [make_chimera_system(2, 8, 79, 12), make_chimera_system(3, 4, 80, 8)], 0, 1)
    _run(wl, [0, 1], [1, 7, 30], kind=kind)


def test_pairs_long_ladder_swaps_across_wavefronts():
    """150 walkers: a swap round has 74 or 75 pairs, so the threads that draw
    and decide them span two wavefronts (the stream window is read by all of
    them before any output is stored)."""
    wl = Workload("long ladder", [make_chimera_system(2, 4, 83, 150)], 0, 1)
    _run(wl, [0], [1, 2, 7])


def test_pairs_config_A_long_run():
    wl = make_workload("A")
    _run(wl, [0], [1] * 5 + [995])


def test_pairs_config_B_full_size_sampled():
    wl = make_workload("B")
    _run(wl, [0, 255], [1, 2])


def test_pairs_config_C_full_size_sampled():
    wl = make_workload("C")
    _run(wl, [0, 2047], [2])


def test_pairs_rejects_odd_slices_and_two_field():
    import paper_1004_0024_amd as pa
    g = pa.Graph([make_chimera_system(2, 5, 81, 4)])
    st = pa.State(g)
    with pytest.raises(pa.IsingError) as e:
        st.pairs_init(np.arange(8, dtype=np.uint32), np.array([1], np.uint32))
    assert e.value.code == -2
    g2 = pa.Graph([make_chimera_system(2, 4, 82, 4)])
    b = g2.systems[0].beta
    g2.set_two_field(b, b)
    st2 = pa.State(g2)
    with pytest.raises(pa.IsingError) as e:
        st2.pairs_init(np.arange(8, dtype=np.uint32), np.array([1], np.uint32))
    assert e.value.code == -5
