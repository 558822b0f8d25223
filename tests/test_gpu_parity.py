"""HIP path against the oracle, element by element, on the same seeded inputs.

Bit-exact: spins, MT19937 windows, energies, temperature labels, swap streams
and counters (every quantity of the chain is an integer or a bit; the one
floating-point decision, the swap test, is made in IEEE double on both sides
and near-threshold cases are counted).
"""
import numpy as np
import pytest

from gen import Workload, make_chimera_system, make_random_system, make_workload

from .gpu_util import chains_for, compare_system, make_state, say

pytestmark = pytest.mark.gpu


def _run_compare(wl, idx, steps, swap_every, record=False):
    """steps: list of sweep counts; compare the sampled systems after each."""
    say(wl.name, "systems", len(wl.systems), "compare", list(idx), "steps", steps, "swap_every", swap_every)
    g, st = make_state(wl)
    chains = chains_for(wl, idx)
    for s, ch in zip(idx, chains):
        compare_system(st, s, ch, "after init")
    near = 0
    for n in steps:
        e = st.sweep(n, swap_every, record=record)
        near = 0  # the counts are cumulative: keep the last comparison's total
        for s, ch in zip(idx, chains):
            rec = ch.sweeps(n, swap_every, record_energy=record)
            near += compare_system(st, s, ch, f"after {st.sweeps} sweeps")
            if record:
                w0, w1 = int(g.walker_base[s]), int(g.walker_base[s + 1])
                assert np.array_equal(e.cpu().numpy()[:, w0:w1], rec["energy"]), "energy series"
    return g, st, near


def test_parity_config_A_every_sweep():
    """One system, 16 walkers, swaps after every sweep: compare after each of the
    first 40 sweeps, then after the remaining 960 (1000 in all)."""
    wl = make_workload("A")
    g, st, near = _run_compare(wl, [0], [1] * 40 + [960], 1)
    say("near-threshold swap decisions, oracle", near, "gpu", st.stats()["near"])
    assert st.stats()["near"] == near
    assert st.sweeps == 1000 and st.rounds == 1000


def test_parity_config_A_energy_series():
    wl = make_workload("A")
    _run_compare(wl, [0], [5, 60], 1, record=True)


@pytest.mark.parametrize("swap_every,steps", [(0, [3, 4]), (3, [2, 5, 7]), (2, [1, 1, 6])])
def test_parity_swap_cadence(swap_every, steps):
    wl = Workload("cadence L=2 M=6 K=6", [make_chimera_system(2, 6, 77, 6)], 0, swap_every)
    _run_compare(wl, [0], steps, swap_every)


@pytest.mark.parametrize("name,sysm", [
    ("L1 open M=2", make_chimera_system(1, 2, 8, 5, ring=False)),
    ("L1 ring M=3", make_chimera_system(1, 3, 9, 4)),
    ("L3 ring M=5 S=72 (ragged rows)", make_chimera_system(3, 5, 10, 7)),
    ("L5 open M=4 S=200", make_chimera_system(5, 4, 11, 3, ring=False)),
    ("L6 ring M=3 S=288 chained MT", make_chimera_system(6, 3, 12, 2)),
    ("random graph N=10 M=1", make_random_system(10, 16, 21, 5)),
    ("random graph N=37 deg 8", make_random_system(37, 140, 5, 3)),
    ("single spin K=1", make_random_system(1, 0, 3, 1)),
])
def test_parity_shapes(name, sysm):
    wl = Workload(name, [sysm], 0, 1)
    _run_compare(wl, [0], [1, 2, 9], 1)


def test_parity_uneven_batch():
    """Systems of every template size in one graph (one launch per size bucket)."""
    systems = [make_chimera_system(L, M, 500 + i, K)
               for i, (L, M, K) in enumerate([(2, 8, 16), (3, 9, 17), (4, 8, 20), (2, 13, 32), (5, 8, 16),
                                              (6, 8, 18), (7, 8, 16), (8, 8, 19), (4, 11, 31), (3, 8, 25)])]
    wl = Workload("uneven", systems, 0, 1)
    _run_compare(wl, list(range(len(systems))), [1, 3], 1)


def test_parity_config_B_full_size_sampled():
    """Full 256-system graph of the throughput workload; two systems compared."""
    wl = make_workload("B")
    _run_compare(wl, [0, 255], [1, 2], 1)


def test_parity_config_C_full_size_sampled():
    wl = make_workload("C")
    _run_compare(wl, [0, 1023, 2047], [2], 1)


def test_parity_config_D_sampled():
    wl = make_workload("D")
    idx = [int(i) for i in np.linspace(0, len(wl.systems) - 1, 6)]
    _run_compare(wl, idx, [2], 1)


def test_pt_swap_standalone_and_observables():
    wl = Workload("swap", [make_chimera_system(2, 5, 3, 9), make_random_system(12, 20, 4, 6)], 0, 1)
    g, st = make_state(wl)
    chains = chains_for(wl, [0, 1])
    st.sweep(3, 0)
    for ch in chains:
        ch.sweeps(3, 0)
    for parity in (1, 0, 1):
        st.swap(parity)
        for ch in chains:
            ch.swap_round(parity)
    for s, ch in enumerate(chains):
        compare_system(st, s, ch, "after pt_swap")
    obs = st.observables().cpu().numpy()
    for s, ch in enumerate(chains):
        w0 = int(g.walker_base[s])
        spins = ch.spins()
        for w in range(ch.K):
            assert obs[w0 + w, 0] == ch.energy_of(w)
            assert obs[w0 + w, 1] == int(spins[w].astype(np.int64).sum())
            assert obs[w0 + w, 2] == int(ch.energy()[w])
            assert obs[w0 + w, 3] == int(ch.labels()[0][w])


def test_sweep_zero_and_errors():
    import paper_1004_0024_amd as pa
    wl = Workload("zero", [make_chimera_system(1, 3, 1, 2)], 0, 1)
    g, st = make_state(wl)
    ch = chains_for(wl, [0])[0]
    st.sweep(0, 1)
    compare_system(st, 0, ch, "after zero sweeps")
    with pytest.raises(pa.IsingError) as e:
        st.sweep(-1, 1)
    assert e.value.code == -1
    with pytest.raises(pa.IsingError):
        st.swap(2)


def test_stats_counters():
    wl = make_workload("A")
    g, st = make_state(wl)
    st.sweep(10, 1)
    stats = st.stats()
    assert stats["attempts"] == 10 * 256 * 16
    assert 0 < stats["wave_flip_steps"] <= stats["wave_steps"]
    assert stats["flips"] == int(st.host("flips").sum())
    ch = chains_for(wl, [0])[0]
    ch.sweeps(10, 1)
    c = ch.counters()
    assert stats["flips"] == int(c["flips"].sum())
    assert stats["swap_att"] == int(c["swap_att"].sum()) and stats["swap_acc"] == int(c["swap_acc"].sum())


@pytest.mark.parametrize("tpw,G", [(512, 1), (256, 2), (128, 3), (64, 1), (64, 4)])
def test_parity_launch_shapes_large_template(tpw, G):
    """Every launch shape gives the same chain (8x8 cells, S = 512)."""
    wl = Workload("shape S=512", [make_chimera_system(8, 6, 31, 5), make_chimera_system(8, 7, 32, 3)], 0, 1)
    say(wl.name, "tpw", tpw, "G", G)
    g, st = make_state(wl)
    g.set_launch(0, tpw, G)
    chains = chains_for(wl, [0, 1])
    for n in (1, 3):
        st.sweep(n, 1)
        for s, ch in enumerate(chains):
            ch.sweeps(n, 1)
            compare_system(st, s, ch, f"tpw={tpw} G={G}")


@pytest.mark.parametrize("tpw,G", [(16, 4), (16, 9), (32, 8), (64, 2), (128, 1)])
def test_parity_launch_shapes_small_template(tpw, G):
    wl = Workload("shape S=128", [make_chimera_system(4, 9, 33, 9)], 0, 1)
    say(wl.name, "tpw", tpw, "G", G)
    g, st = make_state(wl)
    g.set_launch(0, tpw, G)
    ch = chains_for(wl, [0])[0]
    for n in (2, 1):
        st.sweep(n, 1)
        ch.sweeps(n, 1)
        compare_system(st, 0, ch, f"tpw={tpw} G={G}")


def test_launch_shape_rejected():
    import paper_1004_0024_amd as pa
    wl = Workload("shape S=512", [make_chimera_system(8, 4, 31, 2)], 0, 1)
    g, st = make_state(wl)
    before = g.buckets()[0]
    for tpw, G in [(32, 2), (48, 1), (1024, 2), (64, 0)]:
        with pytest.raises(pa.IsingError) as e:
            g.set_launch(0, tpw, G)
        assert e.value.code == -2
    assert g.buckets()[0] == before


@pytest.mark.parametrize("kind", [1, 2])
def test_parity_approximate_acceptance(kind):
    """The paper's approximate flip tests (Fig. 7, fast and accurate): GPU chains with the
    approximate threshold rows against oracle chains with the same test, bit for bit."""
    import paper_1004_0024_amd as pa
    wl = Workload("approx accept", [make_chimera_system(2, 8, 91, 12), make_chimera_system(3, 6, 92, 8)], 0, 1)
    g, st = make_state(wl)
    g.set_acceptance(kind)
    chains = [ch.set_acceptance(kind) for ch in chains_for(wl, [0, 1])]
    for n in (1, 7, 40):
        st.sweep(n, 1)
        for s, ch in enumerate(chains):
            ch.sweeps(n, 1)
            compare_system(st, s, ch, f"kind {kind} after {st.sweeps} sweeps")
    g.set_acceptance(pa.ACCEPT_EXACT)
    st.sweep(5, 1)
    for s, ch in enumerate(chains):
        ch.set_acceptance(0).sweeps(5, 1)
        compare_system(st, s, ch, "back to the exact test")
