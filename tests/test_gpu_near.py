"""The FP64 swap step's near-threshold count on the GPU, on constructed decisions.

A swap decision lands within 1e-12 of its threshold essentially never on random
inputs, so these cases are built (tests/near_case.py): the first decision of
round 0 has exp(Delta) - u 2^-32 = +-1e-14 (counted, and decided the way the
exact comparison decides it) or 3e-12 (not counted).  Each case runs through
the standalone swap kernel (pt_swap on the initial spins, and a sweep followed
by its swap round in a launch shape without in-kernel rounds) and through the
swap round inside the sweep kernel of a whole-ladder workgroup; the chain,
including the per-pair counts, is compared with the oracle.
"""
import numpy as np
import pytest

from .gpu_util import chains_for, compare_system, make_state, say
from . import near_case

pytestmark = pytest.mark.gpu

CASES = [(1e-14, 1), (-1e-14, 1), (3e-12, 0)]


def _check(st, ch, nc, counted, what):
    compare_system(st, 0, ch, what)
    gnear = st.host("swap_near").astype(np.int64)
    assert gnear.tolist() == [counted, 0, 0], (what, gnear.tolist())
    assert st.stats()["near"] == counted
    assert int(st.host("swap_acc")[0]) == int(nc.accept), what
    assert st.host("walker_at").tolist() == ([1, 0, 2] if nc.accept else [0, 1, 2])


@pytest.mark.parametrize("offset,counted", CASES)
def test_near_threshold_pt_swap(offset, counted):
    nc = near_case.build(offset, after_sweep=False)
    say("near-threshold pt_swap, offset", offset, "u", nc.u, "delta", nc.delta, "gap", nc.gap)
    g, st = make_state(nc.workload)
    ch = chains_for(nc.workload, [0])[0]
    st.swap(0)
    ch.swap_round(0)
    _check(st, ch, nc, counted, f"pt_swap offset {offset}")


@pytest.mark.parametrize("offset,counted", CASES)
def test_near_threshold_swap_kernel_after_sweep(offset, counted):
    nc = near_case.build(offset, after_sweep=True)
    say("near-threshold swap kernel after a sweep, offset", offset, "gap", nc.gap)
    g, st = make_state(nc.workload)
    g.set_launch(0, 16, 1)  # one walker per workgroup: no whole ladder, rounds in swap_kernel
    assert g.buckets()[0]["ladder"] == 0
    ch = chains_for(nc.workload, [0])[0]
    st.sweep(1, 1)
    ch.sweeps(1, 1)
    _check(st, ch, nc, counted, f"swap kernel offset {offset}")


@pytest.mark.parametrize("offset,counted", CASES)
def test_near_threshold_ladder_round(offset, counted):
    nc = near_case.build(offset, after_sweep=True)
    say("near-threshold in-kernel ladder round, offset", offset, "gap", nc.gap)
    g, st = make_state(nc.workload)
    assert g.buckets()[0]["ladder"] == 1  # the default shape holds the whole ladder
    ch = chains_for(nc.workload, [0])[0]
    st.sweep(1, 1)
    ch.sweeps(1, 1)
    _check(st, ch, nc, counted, f"ladder round offset {offset}")
    # later rounds add no further counts on either side
    st.sweep(5, 1)
    ch.sweeps(5, 1)
    compare_system(st, 0, ch, "5 more sweeps")
