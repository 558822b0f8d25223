"""Exact heat-bath cell moves on the GPU: one pass against the oracle, the law of
one draw against the conditional Boltzmann law, and a chain against enumeration."""
import numpy as np
import pytest

from gen import LayeredSystem, Workload, chimera_template, make_chimera_system
from oracle import heatbath as H
from oracle import learned as L

from . import exact
from .gpu_util import chains_for, make_state, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ring", [True, False])
def test_one_pass_agrees_with_oracle(ring):
    """Same state and uniforms: the GPU pass (FP32 weights) and the oracle pass (FP64) draw
    the same cell for nearly every cell; energies stay exact."""
    import torch
    wl = Workload("hb pass", [make_chimera_system(3, 5 if ring else 4, 71, 6, ring=ring)], 0, 1)
    g, st = make_state(wl)
    st.sweep(4, 1)
    ch = chains_for(wl, [0])[0]
    ch.sweeps(4, 1)
    moves = torch.zeros((g.R, 2), dtype=torch.int64, device="cuda")
    st.heatbath_cells(key=321, pass_index=11, moves=moves)
    gspins = st.spins_pm([0])[0]
    sysm = wl.systems[0]
    model = L.CellModel(sysm)
    spins = ch.spins().astype(np.int64)
    energy = ch.energy().copy()
    temp_of, _ = ch.labels()
    changed = H.heatbath_pass(model, spins, energy, sysm.beta[temp_of], 321, list(range(sysm.K)), 11)
    diff = sum(not np.array_equal(gspins[w][model.cell_spins(*c)], spins[w][model.cell_spins(*c)])
               for w in range(sysm.K) for c in model.cells)
    ncells = sysm.K * len(model.cells)
    say("heat-bath cells differing", diff, "of", ncells, "changed", int(changed.sum()))
    assert diff <= max(2, ncells // 200)
    mv = moves.cpu().numpy()
    assert int(mv[:, 0].sum()) == ncells
    assert abs(int(mv[:, 1].sum()) - int(changed.sum())) <= max(2, ncells // 200)
    obs = st.observables().cpu().numpy()
    assert np.array_equal(obs[:, 0], obs[:, 2])


def test_one_draw_law():
    """4,096 walkers of one 8-spin cell at one beta (16 systems x 256 walkers): one pass
    draws from the exact conditional law whatever the start (chi-squared)."""
    from scipy import stats
    S, eu, ev = chimera_template(1)
    rng = np.random.default_rng(12)
    vals = np.array([-3, -2, -1, 1, 2, 3], np.int8)
    beta = 0.3
    sysm = LayeredSystem(S=S, M=1, ring=False, eu=eu, ev=ev, eJ=vals[rng.integers(0, 6, len(eu))],
                         h=vals[rng.integers(0, 6, S)], J_tau=np.zeros(S, np.int8), beta=np.full(256, beta), L=1)
    wl = Workload("one cell", [sysm] * 16, 0, 0)
    g, st = make_state(wl)
    model = L.CellModel(sysm)
    idx = model.cell_spins(0, 0, 0)
    law = H.two_stage_law(model.h[idx], H.cell_couplings(model, idx), beta)
    counts = np.zeros(256)
    for t in range(4):
        st.heatbath_cells(key=9, pass_index=t)
        np.add.at(counts, st.host("spins").view(np.uint32) & 0xFF, 1)
    N, u, v, J, h = sysm.expand()
    Ecell = exact.energies(N, u, v, J, h)
    assert np.array_equal(st.host("energy"), Ecell[st.host("spins").view(np.uint32) & 0xFF])
    n = counts.sum()
    e = n * law
    big = e >= 5
    chi2 = ((counts[big] - e[big]) ** 2 / e[big]).sum()
    pval = stats.chi2.sf(chi2, big.sum() - 1)
    say("heat-bath draw chi2", chi2, "dof", big.sum() - 1, "p", pval)
    assert pval > 1e-5
    assert counts[~big].sum() <= 3 * e[~big].sum() + 20


def test_heatbath_chain_keeps_boltzmann():
    """Sweeps interleaved 1:1 with heat-bath passes (swaps every step) on 16 spins, 16
    copies: slot mean energies against enumeration."""
    sysm = make_chimera_system(1, 2, seed=8, K=4, ring=False, beta_min=0.2, beta_max=1.0)
    wl = Workload("hb chain", [sysm] * 16, 0, 1)
    g, st = make_state(wl)
    n = 1500
    series = []
    for t in range(n):
        st.sweep(1, 1)
        st.heatbath_cells(key=79, pass_index=t)
        wat = st.host("walker_at").reshape(16, 4)
        en = st.host("energy").reshape(16, 4)
        series.append(np.take_along_axis(en, wat, axis=1))
    obs = st.observables().cpu().numpy()
    assert np.array_equal(obs[:, 0], obs[:, 2])
    N, u, v, J, h = sysm.expand()
    E = exact.energies(N, u, v, J, h)
    series = np.array(series)[n // 10:]
    for k in range(4):
        m, sd = exact.batch_mean_sigma(series[:, :, k].mean(1), 20)
        ref = exact.mean_energy(E, float(sysm.beta[k]))
        say("slot", k, "mean", m, "exact", ref, "sd", sd)
        assert abs(m - ref) < 5 * sd + 0.05
