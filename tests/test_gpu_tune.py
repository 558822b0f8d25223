"""Runtime choices on the GPU that change how fast, not what, the chain samples:
the swap-cadence tuner (scored by effective samples per second) and the spread
of several buckets over streams (chain unchanged, checked against the oracle)."""
import numpy as np
import pytest

from gen import Workload, make_chimera_system

from .gpu_util import chains_for, compare_system, make_state, say

pytestmark = pytest.mark.gpu


def test_swap_cadence_tuner():
    """The tuner leaves the state alone, scores every candidate, picks the one with the
    most effective samples per second, and the chain at that cadence is the oracle's."""
    import paper_1004_0024_amd as pa
    wl = Workload("cadence tuner", [make_chimera_system(2, 8, 60 + i, 16) for i in range(4)], 0, 1)
    g, st = make_state(wl)
    st.sweep(200, 1)
    before = st.host("spins").copy()
    res = pa.tune.swap_cadence(st, (1, 3), steps=400)
    say("cadence trials", res["trials"], "best", res["best"])
    assert np.array_equal(st.host("spins"), before) and st.sweeps == 200
    assert [t["swap_every"] for t in res["trials"]] == [1, 3]
    assert all(t["ess_per_s"] > 0 and t["ms_per_step"] > 0 for t in res["trials"])
    assert res["best"] == max(res["trials"], key=lambda t: t["ess_per_s"])["swap_every"]
    chains = chains_for(wl, range(4))
    for ch in chains:
        ch.sweeps(200, 1)
    st.sweep(30, res["best"])
    for s, ch in enumerate(chains):
        ch.sweeps(30, res["best"])
        compare_system(st, s, ch, f"cadence {res['best']}")


def test_buckets_spread_over_streams_keep_the_chain():
    """Eight template sizes (eight buckets) on at most four streams, largest first, before
    and after the autotuner re-spreads them by measured time; captured and eager loops."""
    import paper_1004_0024_amd as pa
    systems = [make_chimera_system(L, M, 700 + i, K)
               for i, (L, M, K) in enumerate([(1, 9, 5), (2, 8, 16), (3, 9, 7), (4, 8, 9), (5, 8, 6),
                                              (6, 8, 5), (7, 8, 4), (8, 8, 3), (2, 13, 11), (4, 11, 8)])]
    wl = Workload("streams", systems, 0, 1)
    g, st = make_state(wl)
    assert len(g.buckets()) == 8  # one per template size
    chains = chains_for(wl, range(len(systems)))
    st.sweep(3, 1)
    for ch in chains:
        ch.sweeps(3, 1)
    for s, ch in enumerate(chains):
        compare_system(st, s, ch, "attempt-weighted streams")
    scratch = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    g.autotune(scratch, reps=1)
    rep = st.capture(4, swap_every=1)
    rep.launch()
    rep.stream.synchronize()
    for ch in chains:
        ch.sweeps(4, 1)
    for s, ch in enumerate(chains):
        compare_system(st, s, ch, "time-weighted streams, captured")


@pytest.mark.parametrize("L,M,K,tpw,G", [
    (3, 6, 8, 72, 8),     # 72-spin walkers back to back: 9 wavefronts, walkers straddle them
    (3, 6, 8, 72, 3),     # 216 threads: the last wavefront partly idle
    (3, 6, 5, 128, 2),    # a multiple of 64 above S
    (5, 5, 5, 200, 4),
    (6, 4, 4, 288, 2),
    (6, 4, 4, 320, 1),
    (6, 4, 4, 144, 3),    # ceil(S / 2): two columns per thread
    (7, 4, 3, 196, 2),
    (8, 3, 2, 576, 1),    # more threads than spins
])
def test_threads_per_walker_not_a_power_of_two(L, M, K, tpw, G):
    """Shapes with a thread count per walker above 64 that is not a power of two keep the
    chain, the MT windows and every counter (a wavefront that holds two walkers splits its flip
    count between them by a lane mask) bit for bit; swap rounds after single sweeps and a 7-sweep launch."""
    wl = Workload(f"tpw {tpw} G {G}", [make_chimera_system(L, M, 800 + L, K)], 0, 1)
    g, st = make_state(wl)
    g.set_launch(0, tpw, G)
    b = g.buckets()[0]
    say("shape", {k: b[k] for k in ("S", "tpw", "G", "cpt", "threads", "lds")})
    assert (b["tpw"], b["G"]) == (tpw, min(G, K))
    ch = chains_for(wl, [0])[0]
    st.sweep(3, 1)
    ch.sweeps(3, 1)
    compare_system(st, 0, ch, "single sweeps")
    st.sweep(7, 0)
    ch.sweeps(7, 0)
    compare_system(st, 0, ch, "7-sweep launch")
    st.sweep(2, 1)
    ch.sweeps(2, 1)
    compare_system(st, 0, ch, "after")
