"""Runtime around the sweep on the GPU: captured sweep loops (HIP graphs),
the launch-shape autotuner, checkpoint / resume.  Every chain is checked
against the oracle bit for bit."""
import numpy as np
import pytest

from gen import Workload, make_chimera_system, make_workload

from .gpu_util import chains_for, compare_system, make_state, say

pytestmark = pytest.mark.gpu


def _small():
    return Workload("runtime", [make_chimera_system(2, 6, 41, 6), make_chimera_system(3, 5, 42, 5)], 0, 1)


def test_graph_replay_matches_oracle():
    """Replays of one captured 8-sweep loop (an even number of swap rounds, so
    every replay starts in the captured phase), with eager work between them."""
    import torch
    wl = _small()
    say("graph replay", wl.name)
    g, st = make_state(wl)
    chains = chains_for(wl, [0, 1])
    rep = st.capture(8, swap_every=1, record=True)
    for k in range(3):
        e = rep.launch()
        rep.stream.synchronize()
        recs = [ch.sweeps(8, 1, record_energy=True)["energy"] for ch in chains]
        for s, ch in enumerate(chains):
            compare_system(st, s, ch, f"replay {k}")
            w0, w1 = int(g.walker_base[s]), int(g.walker_base[s + 1])
            assert np.array_equal(e.cpu().numpy()[:, w0:w1], recs[s])
        st.observables()  # eager work between replays
        torch.cuda.synchronize()
    assert st.sweeps == 24 and st.rounds == 24


def test_graph_replay_rejects_other_phase():
    import paper_1004_0024_amd as pa
    wl = _small()
    g, st = make_state(wl)
    rep = st.capture(4, swap_every=1)
    st.sweep(1, 1)  # now one swap round ahead of the capture
    with pytest.raises(pa.IsingError) as e:
        rep.launch()
    assert e.value.code == -5
    odd = st.capture(3, swap_every=1)  # an odd number of rounds flips the phase
    odd.launch()
    odd.stream.synchronize()
    with pytest.raises(pa.IsingError):
        odd.launch()


def test_autotune_keeps_the_chain():
    import paper_1004_0024_amd as pa
    wl = Workload("tune", [make_chimera_system(4, 8, 51, 8), make_chimera_system(2, 8, 52, 16)], 0, 1)
    say("autotune", wl.name)
    g = pa.Graph(wl.systems)
    scratch = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    rows = g.autotune(scratch, reps=2)
    assert len(rows) > 4 and all(r["ns_per_sweep"] > 0 for r in rows)
    for bi, b in enumerate(g.buckets()):
        best = min((r for r in rows if r["bucket"] == bi), key=lambda r: r["ns_per_sweep"])
        assert (b["tpw"], b["G"]) == (best["tpw"], best["G"])
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    chains = chains_for(wl, [0, 1])
    st.sweep(5, 1)
    for s, ch in enumerate(chains):
        ch.sweeps(5, 1)
        compare_system(st, s, ch, "after autotune")


def test_autotune_ladder_graph_keeps_the_chain():
    """A graph whose buckets all hold whole ladders is tuned on 16-sweep launches
    with the swap rounds inside the kernel: the tuned shapes stay ladder shapes,
    the fastest trial is kept, and the chain (swaps in the kernel, cadences 1
    and 2) is the oracle's."""
    import paper_1004_0024_amd as pa
    wl = Workload("tune ladders", [make_chimera_system(2, 8, 53, 16), make_chimera_system(2, 5, 54, 12)], 0, 1)
    say("autotune", wl.name)
    g = pa.Graph(wl.systems)
    assert all(b["ladder"] == 1 for b in g.buckets())
    scratch = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    rows = g.autotune(scratch, reps=2)
    assert len(rows) >= 2 and all(r["ns_per_sweep"] > 0 for r in rows)
    assert all(b["ladder"] == 1 for b in g.buckets())
    for bi, b in enumerate(g.buckets()):
        best = min((r for r in rows if r["bucket"] == bi), key=lambda r: r["ns_per_sweep"])
        assert (b["tpw"], b["G"]) == (best["tpw"], best["G"])
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    chains = chains_for(wl, [0, 1])
    for n, every in ((7, 1), (6, 2)):
        st.sweep(n, every)
        for s, ch in enumerate(chains):
            ch.sweeps(n, every)
            compare_system(st, s, ch, f"after ladder autotune, {n} sweeps, swap every {every}")


def test_checkpoint_resume_bit_identical():
    """Saving every state buffer and the two counters, then resuming, continues
    the chain exactly as an uninterrupted run."""
    import paper_1004_0024_amd as pa
    wl = _small()
    g, st = make_state(wl)
    st.sweep(5, 2)
    ckpt = {k: v.clone() for k, v in st.t.items()}
    counters = (st.sweeps, st.rounds)
    st.sweep(6, 2)
    ref = {k: v.cpu().numpy() for k, v in st.t.items()}
    st2 = pa.State(g)
    for k, v in ckpt.items():
        st2.t[k].copy_(v)
    st2._s.sweeps, st2._s.rounds = counters
    st2.sweep(6, 2)
    for k, v in st2.t.items():
        assert np.array_equal(v.cpu().numpy(), ref[k]), k
    chains = chains_for(wl, [0, 1])
    for s, ch in enumerate(chains):
        ch.sweeps(11, 2)
        compare_system(st2, s, ch, "resumed")


def test_record_slots_matches_observables():
    """ising_record_slots writes the running energy of the walker at each slot."""
    import torch
    import paper_1004_0024_amd as pa
    wl = make_workload("C").subset(range(3), n_sweeps=7)
    _, st = make_state(wl)
    st.sweep(7, 1)
    e = torch.full((st.graph.slots,), -7, dtype=torch.int32, device="cuda")
    st.record(e)
    obs = st.observables().cpu().numpy()
    got = e.cpu().numpy()
    want = np.zeros_like(got)
    base = st.graph.walker_base
    sys_of = np.repeat(np.arange(len(base) - 1), np.diff(base))
    want[base[sys_of] + obs[:, 3]] = obs[:, 2]  # obs[:, 3] is the slot within the system
    assert np.array_equal(got, want)
    assert np.array_equal(obs[:, 0], obs[:, 2])


@pytest.mark.parametrize("ladder", [True, False])
def test_in_kernel_swap_rounds_match_oracle(ladder):
    """Whole ladders in one workgroup (swap rounds inside the sweep kernel, one launch per
    call) and the same systems split over workgroups (swap kernel between sweeps): both
    chains equal the oracle's, with swap cadences 1 and 3 and a graph replay."""
    wl = Workload("ladder", [make_chimera_system(2, 5, 51, 12), make_chimera_system(2, 4, 52, 9)], 0, 1)
    g, st = make_state(wl)
    if not ladder:
        g.set_launch(0, 32, 4)
    say("buckets", g.buckets())
    assert all(b["ladder"] == (1 if ladder else 0) for b in g.buckets())
    chains = chains_for(wl, [0, 1])
    for n, every in ((1, 1), (7, 1), (5, 3), (4, 3)):
        st.sweep(n, every)
        for s, ch in enumerate(chains):
            ch.sweeps(n, every)
            compare_system(st, s, ch, f"ladder={ladder} {n} sweeps, swap every {every}")
    # a captured loop of 6 sweeps with swaps every 3, replayed twice
    rep = st.capture(6, swap_every=3)
    for _ in range(2):
        rep.launch()
        rep.stream.synchronize()
        for s, ch in enumerate(chains):
            ch.sweeps(6, 3)
            compare_system(st, s, ch, f"ladder={ladder} replay")
