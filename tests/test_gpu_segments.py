"""Long calls cut into launches whose 32-bit per-launch counters cannot wrap.

The real cut comes after about 10^5 sweeps of the largest systems; the
environment cap ISING_LAUNCH_SWEEPS_MAX lowers it so that short calls run as
several launches.  The chain must not notice: spins, MT windows, labels, swap
streams and every counter match the oracle bit for bit, with the swap rounds
inside the sweep kernel (their parity carried across launches), with a swap
kernel between launches, in captured loops, and in the layer-pair order."""
import pytest

from gen import Workload, make_chimera_system

from .gpu_util import chains_for, compare_system, make_state, say
from . import test_gpu_pairs as tp

pytestmark = pytest.mark.gpu


@pytest.fixture
def cap3(monkeypatch):
    monkeypatch.setenv("ISING_LAUNCH_SWEEPS_MAX", "3")


def test_segments_without_swaps(cap3):
    wl = Workload("segments, no swaps", [make_chimera_system(3, 6, 31, 4)], 0, 0)
    g, st = make_state(wl)
    g.set_launch(0, 128, 1)
    assert g.buckets()[0]["ladder"] == 0
    ch = chains_for(wl, [0])[0]
    st.sweep(10, 0)  # launches of 3, 3, 3, 1 sweeps
    ch.sweeps(10, 0)
    compare_system(st, 0, ch, "10 sweeps in launches of at most 3")
    st.sweep(12, 5)  # 3, 2 | swap | 3, 2 | swap | 2 (the swap kernel between launches)
    ch.sweeps(12, 5)
    compare_system(st, 0, ch, "swap rounds every 5 sweeps, launches of at most 3")
    assert st.sweeps == 22 and st.rounds == ch.rounds_done


def test_segments_with_rounds_in_the_kernel(cap3):
    wl = Workload("segments, ladder", [make_chimera_system(2, 8, 32, 16)], 0, 2)
    g, st = make_state(wl)
    assert g.buckets()[0]["ladder"] == 1  # the default shape holds the whole ladder
    ch = chains_for(wl, [0])[0]
    for n, every in ((11, 2), (7, 1), (5, 3)):
        st.sweep(n, every)
        ch.sweeps(n, every)
        say("ladder segments", n, every, "rounds", st.rounds)
        compare_system(st, 0, ch, f"{n} sweeps, a round after every {every}")
        assert st.rounds == ch.rounds_done


def test_segments_captured(cap3):
    wl = Workload("segments, captured", [make_chimera_system(2, 8, 33, 16)], 0, 1)
    g, st = make_state(wl)
    ch = chains_for(wl, [0])[0]
    rep = st.capture(8, swap_every=1)  # launches of 3, 3, 2 sweeps, rounds inside
    for _ in range(2):
        rep.launch()
        rep.stream.synchronize()
        ch.sweeps(8, 1)
        compare_system(st, 0, ch, "captured 8-sweep loop in launches of at most 3")


def test_segments_layer_pairs(cap3):
    wl = Workload("segments, layer pairs", [make_chimera_system(2, 8, 34, 12)], 0, 1)
    g, st, chains, lb = tp._setup(wl, [0])
    st.pairs_sweep(10, 1)
    chains[0].sweeps(10, 1)
    tp._compare(wl, st, 0, chains[0], lb, "layer pairs, 10 sweeps in launches of at most 3")
