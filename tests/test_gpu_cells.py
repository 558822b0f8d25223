"""Learned cell moves on the GPU: training rows, one pass against the oracle,
exactness of the Metropolis-Hastings moves by enumeration, energy bookkeeping."""
import numpy as np
import pytest

from gen import LayeredSystem, Workload, chimera_template, make_chimera_system
from gen.mlp import initial_params
from oracle import learned as L

from . import exact
from .gpu_util import chains_for, make_state, say

pytestmark = pytest.mark.gpu


def _sharp(seed):
    p = initial_params(seed).astype(np.float64)
    p[-8 - 8 * 128:-8] *= 6.0
    return p


def test_collect_cells_matches_oracle():
    import torch
    wl = Workload("collect", [make_chimera_system(3, 5, 61, 4), make_chimera_system(2, 4, 62, 3, ring=False)], 0, 1)
    g, st = make_state(wl)
    st.sweep(3, 1)
    chains = chains_for(wl, [0, 1])
    for ch in chains:
        ch.sweeps(3, 1)
    total = sum(s.M * s.L * s.L * s.K for s in wl.systems)
    x, y = st.collect_cells(total, stride=1, offset=0)
    x, y = x.cpu().numpy(), y.cpu().numpy()
    row = 0
    for s, (sysm, ch) in enumerate(zip(wl.systems, chains)):
        model = L.CellModel(sysm)
        spins = ch.spins().astype(np.int64)
        temp_of, _ = ch.labels()
        for w in range(sysm.K):
            for (m, yy, xx) in model.cells:
                idx = model.cell_spins(m, yy, xx)
                b = model.boundary(spins[w], idx)
                ref = L.features(b[None, :], [sysm.beta[temp_of[w]]])[0]
                assert np.allclose(x[row], ref, rtol=0, atol=1e-6), (s, w, m, yy, xx)
                assert y[row] == sum(1 << k for k, i in enumerate(idx) if spins[w][i] > 0)
                row += 1
    # stride / offset wrap around the cell list
    x2, y2 = st.collect_cells(7, stride=5, offset=total - 3)
    for i in range(7):
        assert y2.cpu().numpy()[i] == y[(total - 3 + 5 * i) % total]


def test_one_pass_agrees_with_oracle():
    """Same state, network and uniforms: the GPU pass (BF16 network) and the oracle pass
    (the same network in the BF16 mirror) take the same decision for nearly every cell."""
    import torch
    wl = Workload("pass", [make_chimera_system(4, 6, 63, 8)], 0, 1)
    g, st = make_state(wl)
    st.sweep(5, 1)
    ch = chains_for(wl, [0])[0]
    ch.sweeps(5, 1)
    params = _sharp(9)
    import paper_1004_0024_amd as pa
    net = pa.Mlp(params)
    moves = torch.zeros((g.R, 2), dtype=torch.int64, device="cuda")
    st.propose_cells(net, key=123, pass_index=7, moves=moves)
    gspins = st.spins_pm([0])[0]
    sysm = wl.systems[0]
    model = L.CellModel(sysm)
    spins = ch.spins().astype(np.int64)
    energy = ch.energy().copy()
    temp_of, _ = ch.labels()
    acc = L.learned_pass(model, spins, energy, sysm.beta[temp_of], params, 123, list(range(sysm.K)), 7,
                         forward_fn=L.forward_bf16)
    diff_cells = 0
    for w in range(sysm.K):
        for (m, yy, xx) in model.cells:
            idx = model.cell_spins(m, yy, xx)
            if not np.array_equal(gspins[w][idx], spins[w][idx]):
                diff_cells += 1
    ncells = sysm.K * len(model.cells)
    say("cells differing after one pass", diff_cells, "of", ncells, "accepted", int(acc.sum()))
    assert diff_cells <= max(2, ncells // 200)
    mv = moves.cpu().numpy()
    assert int(mv[:, 0].sum()) == ncells
    assert abs(int(mv[:, 1].sum()) - int(acc.sum())) <= max(2, ncells // 200)
    obs = st.observables().cpu().numpy()
    assert np.array_equal(obs[:, 0], obs[:, 2]), "running energy must equal the recomputed cost"


def _single_cell(seed, K, beta):
    S, eu, ev = chimera_template(1)
    rng = np.random.default_rng(seed)
    vals = np.array([-3, -2, -1, 1, 2, 3], np.int8)
    return LayeredSystem(S=S, M=1, ring=False, eu=eu, ev=ev, eJ=vals[rng.integers(0, 6, len(eu))],
                         h=vals[rng.integers(0, 6, S)], J_tau=np.zeros(S, np.int8),
                         beta=np.full(K, beta), L=1)


def test_cell_move_one_step_kernel():
    """256 walkers of one 8-spin cell, all reset to the same state before every pass:
    the law of the outcome against the exact Metropolis-Hastings kernel."""
    import torch
    from scipy import stats
    import paper_1004_0024_amd as pa
    K, beta = 256, 0.35
    sysm = _single_cell(3, K, beta)
    wl = Workload("one cell", [sysm], 0, 0)
    g, st = make_state(wl)
    params = _sharp(4)
    net = pa.Mlp(params)
    N, u, v, J, h = sysm.expand()
    Ecell = exact.energies(N, u, v, J, h)
    S = exact.all_states(N)
    logits, _ = L.forward(L.unpack(params), L.features(h[None, :].astype(np.int64), [beta]))
    lp, lm = L.log_sigmoid(logits[0]), L.log_sigmoid(-logits[0])
    logq = np.where(S > 0, lp[None, :], lm[None, :]).sum(1)
    for start in (5, 170):
        a = np.minimum(1.0, np.exp(-beta * (Ecell - Ecell[start]) + logq[start] - logq))
        T = np.exp(logq) * a
        T[start] = 0.0
        T[start] = 1.0 - T.sum()
        counts = np.zeros(256)
        n_pass = 60
        for t in range(n_pass):
            st.t["spins"].fill_(start)
            st.t["energy"].fill_(int(Ecell[start]))
            st.propose_cells(net, key=5, pass_index=1000 * start + t)
            words = st.host("spins").view(np.uint32) & 0xFF
            e = st.host("energy")
            assert np.array_equal(e, Ecell[words]), "energy bookkeeping"
            np.add.at(counts, words, 1)
        n = K * n_pass
        expct = n * T
        big = expct >= 5
        chi2 = ((counts[big] - expct[big]) ** 2 / expct[big]).sum()
        pval = stats.chi2.sf(chi2, big.sum() - 1)
        say("one-step kernel start", start, "chi2", chi2, "dof", big.sum() - 1, "p", pval)
        assert pval > 1e-5
        assert counts[~big].sum() <= max(30, 3 * expct[~big].sum() + 10)


def test_learned_chain_keeps_boltzmann():
    """Plain sweeps interleaved 1:1 with learned passes (swaps every step) on 16 spins,
    16 independent copies: slot mean energies against enumeration."""
    import paper_1004_0024_amd as pa
    sysm = make_chimera_system(1, 2, seed=8, K=4, ring=False, beta_min=0.2, beta_max=1.0)
    wl = Workload("learned chain", [sysm] * 16, 0, 1)
    g, st = make_state(wl)
    net = pa.Mlp(_sharp(10))
    n = 1500
    series = []
    for t in range(n):
        st.sweep(1, 1)
        st.propose_cells(net, key=78, pass_index=t)
        wat = st.host("walker_at").reshape(16, 4)
        en = st.host("energy").reshape(16, 4)
        series.append(np.take_along_axis(en, wat, axis=1))
    obs = st.observables().cpu().numpy()
    assert np.array_equal(obs[:, 0], obs[:, 2])
    N, u, v, J, h = sysm.expand()
    E = exact.energies(N, u, v, J, h)
    series = np.array(series)[n // 10:]  # [t, copy, slot]
    for k in range(4):
        m, sd = exact.batch_mean_sigma(series[:, :, k].mean(1), 20)
        ref = exact.mean_energy(E, float(sysm.beta[k]))
        say("slot", k, "mean", m, "exact", ref, "sd", sd)
        assert abs(m - ref) < 5 * sd + 0.05
