"""The learned proposal end to end on the GPU: training on samples of the plain
chain lowers the held-out loss and raises the acceptance of cell moves; copies
of a state run identical chains; the effective-sample estimate of a chain."""
import numpy as np
import pytest

from gen import make_workload
from gen.mlp import initial_params

from .gpu_util import say

pytestmark = pytest.mark.gpu


def _setup(n_sys=16, burn=400):
    import paper_1004_0024_amd as pa
    wl = make_workload("E").subset(range(n_sys))
    g = pa.Graph(wl.systems)
    st = pa.State(g).init(wl.walker_seeds, wl.swap_seeds)
    st.sweep(burn, 1)
    return pa, g, st


def _acceptance(pa, g, base, net, key=5):
    import torch
    s2 = pa.State(g).copy_from(base)
    mv = torch.zeros((g.R, 2), dtype=torch.int64, device="cuda")
    s2.propose_cells(net, key, 0, mv)
    m = mv.sum(0).cpu().numpy()
    return float(m[1]) / float(m[0])


def test_training_raises_acceptance():
    from paper_1004_0024_amd import learn
    pa, g, st = _setup()
    x, y = learn.collect(st, 1 << 17, snapshots=4, sweeps_between=5)
    xh, yh = learn.collect(st, 1 << 13, snapshots=1, sweeps_between=7)
    base = pa.State(g).copy_from(st)
    net0 = pa.Mlp(initial_params(11))
    net = pa.Mlp(initial_params(11))
    held0 = float(net.grad_step(xh, yh).item())
    losses = learn.train(net, x, y, batch=4096, epochs=3, lr=2e-3)
    held1 = float(net.grad_step(xh, yh).item())
    a0, a1 = _acceptance(pa, g, base, net0), _acceptance(pa, g, base, net)
    say("held-out loss", held0, "->", held1, "acceptance", a0, "->", a1, "steps", len(losses))
    assert len(losses) == 3 * ((1 << 17) // 4096)
    assert held1 < 0.6 * held0
    assert a1 > 3.0 * a0 and a1 > 0.15


def test_copied_state_runs_the_same_chain():
    import torch
    pa, g, st = _setup(n_sys=4, burn=20)
    net = pa.Mlp(initial_params(2))
    a = pa.State(g).copy_from(st)
    b = pa.State(g).copy_from(st)
    for s in (a, b):
        s.sweep(3, 1)
        s.propose_cells(net, 3, 0)
        s.sweep(2, 1)
    torch.cuda.synchronize()
    for name in pa.State._FIELDS:
        assert torch.equal(a.t[name], b.t[name]), name
    assert a.sweeps == b.sweeps == st.sweeps + 5 and a.rounds == b.rounds


def test_run_records_energies_and_ess():
    from paper_1004_0024_amd import learn
    pa, g, st = _setup(n_sys=2, burn=50)
    r = learn.run(st, 200, None)
    e = r["e"]
    assert e.shape == (200, g.slots)
    obs = st.observables().cpu().numpy()
    base = g.walker_base
    sys_of = np.repeat(np.arange(len(base) - 1), np.diff(base))
    last = np.zeros(g.slots, np.int64)
    last[base[sys_of] + obs[:, 3]] = obs[:, 2]
    assert np.array_equal(e[-1], last)
    s = learn.ess_summary(g, e)
    assert 0 < s["coldest_total"] <= 2 * 160 and s["median_slot"] > 0


def test_timed_cell_passes_leave_the_chain_unchanged():
    """HIP events around each cell pass (learn.run's time_cells, which the benchmark
    uses to time the kernels where the chains run them) give one positive time per
    pass and the same chain as the untimed run."""
    from paper_1004_0024_amd import learn
    pa, g, st = _setup(n_sys=2, burn=50)
    net = pa.Mlp(initial_params(3))
    a, b = pa.State(g).copy_from(st), pa.State(g).copy_from(st)
    ra = learn.run(a, 30, net, pass0=7)
    rb = learn.run(b, 30, net, pass0=7, time_cells=True)
    assert np.array_equal(ra["e"], rb["e"]) and np.array_equal(a.host("spins"), b.host("spins"))
    assert "cell_pass_ms" not in ra
    assert len(rb["cell_pass_ms"]) == 30 and min(rb["cell_pass_ms"]) > 0
    rh = learn.run(pa.State(g).copy_from(st), 12, None, heatbath=True, cell_every=4, time_cells=True)
    assert len(rh["cell_pass_ms"]) == 3 and min(rh["cell_pass_ms"]) > 0
