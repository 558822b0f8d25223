"""Pins of the learned-proposal oracle: library routines, finite differences,
and exactness of the Metropolis-Hastings cell moves by enumeration (CPU)."""
import numpy as np
import pytest
import torch

import oracle
from gen import make_chimera_system
from gen.mlp import N_PARAMS, initial_params
from oracle import learned as L

from . import exact


def test_philox_known_answers():
    """Philox4x32-10 against the known-answer vectors published with the generator."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_known_answers.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert L.philox4x32(v[0:4], v[4:6]) == v[6:10]
    # fewer rounds give other words (the round count is taken from the argument)
    assert L.philox4x32([0] * 4, [0, 0], rounds=7) != [int(x, 16) for x in rows[0][6:10]]


def test_cell_uniforms_layout():
    """Blocks 0, 1 give the proposal words, word 0 of block 2 the acceptance word."""
    key = 0x0123456789ABCDEF
    u = L.cell_uniforms(key, 77, 5, 9)
    k = (0x89ABCDEF, 0x01234567)
    assert u[:4] == L.philox4x32((9, 77, 5, 0), k)
    assert u[4:8] == L.philox4x32((9, 77, 5, 1), k)
    assert u[8] == L.philox4x32((9, 77, 5, 2), k)[0]
    assert len(set(u)) == 9


def test_forward_matches_torch():
    p = L.unpack(initial_params(3))
    rng = np.random.default_rng(0)
    x = rng.normal(size=(50, 17))
    lin = [torch.nn.Linear(17, 128).double(), torch.nn.Linear(128, 128).double(), torch.nn.Linear(128, 8).double()]
    with torch.no_grad():
        for layer, (w, b) in zip(lin, [("W1", "b1"), ("W2", "b2"), ("W3", "b3")]):
            layer.weight.copy_(torch.from_numpy(p[w]))
            layer.bias.copy_(torch.from_numpy(rng.normal(size=p[b].shape)))
            p[b] = layer.bias.numpy().copy()
        ref = lin[2](torch.relu(lin[1](torch.relu(lin[0](torch.from_numpy(x)))))).numpy()
    got, _ = L.forward(p, x)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    flat = initial_params(5).astype(np.float64)
    flat[-8:] = rng.normal(size=8) * 0.1
    p = L.unpack(flat)
    x = L.features(rng.integers(-12, 13, size=(40, 8)), rng.uniform(0.1, 3.0, 40))
    y = rng.integers(0, 2, size=(40, 8)).astype(np.float64)
    logits, cache = L.forward(p, x)
    g = L.pack(L.backward(p, cache, logits, y))
    idx = rng.choice(N_PARAMS, 300, replace=False)
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        num = (L.nll(L.forward(L.unpack(fp), x)[0], y) - L.nll(L.forward(L.unpack(fm), x)[0], y)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)) + 1e-9, (i, num, g[i])


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(2)
    a = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, 10000), [0.0, -0.0, 1.0, 3.0e38]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(L.bf16(a), ref)


def test_adam_matches_torch():
    rng = np.random.default_rng(3)
    w0 = rng.normal(size=64)
    opt = L.Adam(w0, lr=1e-2)
    t = torch.tensor(w0, requires_grad=True)
    topt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(20):
        g = rng.normal(size=64)
        opt.step(g)
        topt.zero_grad()
        t.grad = torch.tensor(g)
        topt.step()
    assert np.allclose(opt.w, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_mirror_close_to_fp64():
    rng = np.random.default_rng(4)
    p = L.unpack(initial_params(6))
    x = L.features(rng.integers(-12, 13, size=(256, 8)), rng.uniform(0.1, 3.0, 256))
    y = rng.integers(0, 2, size=(256, 8)).astype(np.float64)
    l64, c64 = L.forward(p, x)
    l16, c16 = L.forward_bf16(p, x)
    assert np.abs(l16 - l64).max() < 2e-2 * (1 + np.abs(l64).max())
    g64 = L.pack(L.backward(p, c64, l64, y))
    g16 = L.pack(L.backward_bf16(p, c16, l16, y))
    cos = g64 @ g16 / np.linalg.norm(g64) / np.linalg.norm(g16)
    assert cos > 0.999


def _run_learned_chain(params, n_steps, sweeps_per_step, seed0=9000, K=3):
    sysm = make_chimera_system(1, 2, seed=8, K=K, ring=False, beta_min=0.2, beta_max=0.8)
    model = L.CellModel(sysm)
    ch = oracle.Chain.from_system(sysm, seed0 + np.arange(K), seed0 + 100)
    N, u, v, J, h = sysm.expand()
    E = exact.energies(N, u, v, J, h)
    es = []
    acc_total = 0
    for t in range(n_steps):
        if sweeps_per_step:
            ch.sweeps(sweeps_per_step, swap_every=0)
        spins = ch.spins().astype(np.int64)
        energy = ch.energy().copy()
        temp_of, _ = ch.labels()
        betas = sysm.beta[temp_of]
        acc_total += L.learned_pass(model, spins, energy, betas, params, 77, list(range(K)), t).sum()
        for w in range(K):
            ch.set_spins(w, spins[w].astype(np.int8))
        assert np.array_equal(ch.energy(), energy), "running energy of the cell moves"
        es.append(ch.energy()[np.argsort(temp_of)].copy())
    return sysm, E, np.array(es), acc_total


def _sharp_params(seed):
    p = initial_params(seed).astype(np.float64)
    p[-8 - 8 * 128:-8] *= 6.0  # a peaked proposal, far from uniform
    return p


def _single_cell_system(seed):
    from gen import LayeredSystem, chimera_template
    S, eu, ev = chimera_template(1)
    rng = np.random.default_rng(seed)
    vals = np.array([-3, -2, -1, 1, 2, 3], np.int8)
    return LayeredSystem(S=S, M=1, ring=False, eu=eu, ev=ev, eJ=vals[rng.integers(0, 6, len(eu))],
                         h=vals[rng.integers(0, 6, S)], J_tau=np.zeros(S, np.int8),
                         beta=np.array([0.35]), L=1)


def test_learned_move_one_step_kernel():
    """One cell move from a fixed state, repeated with fresh uniforms: the empirical law of
    the outcome against the exact Metropolis-Hastings kernel
    T(s->s') = q(s') min(1, pi(s') q(s) / (pi(s) q(s'))), by enumeration of the 256 cell states."""
    from scipy import stats
    sysm = _single_cell_system(3)
    model = L.CellModel(sysm)
    params = _sharp_params(4)
    p = L.unpack(params)
    beta = float(sysm.beta[0])
    N, u, v, J, h = sysm.expand()
    Ecell = exact.energies(N, u, v, J, h)          # the whole graph is the cell: b = h
    S = exact.all_states(N)
    logits, _ = L.forward(p, L.features(h[None, :].astype(np.int64), [beta]))
    lp = L.log_sigmoid(logits[0])
    lm = L.log_sigmoid(-logits[0])
    logq = np.where(S > 0, lp[None, :], lm[None, :]).sum(1)
    rng = np.random.default_rng(5)
    for start in rng.choice(256, 3, replace=False):
        a = np.minimum(1.0, np.exp(-beta * (Ecell - Ecell[start]) + logq[start] - logq))
        T = np.exp(logq) * a
        T[start] = 0.0
        T[start] = 1.0 - T.sum()
        n = 20000
        counts = np.zeros(256)
        for t in range(n):
            spins = S[start][None, :].copy()
            energy = np.array([Ecell[start]])
            L.learned_pass(model, spins, energy, [beta], params, 11, [0], t)
            x = int(sum(1 << i for i in range(N) if spins[0][i] > 0))
            assert energy[0] == Ecell[x]
            counts[x] += 1
        expct = n * T
        big = expct >= 5
        assert counts[~big].sum() <= max(30, 3 * expct[~big].sum() + 10)
        chi2 = ((counts[big] - expct[big]) ** 2 / expct[big]).sum()
        pval = stats.chi2.sf(chi2, big.sum() - 1)
        assert pval > 1e-5, (start, chi2, big.sum(), pval)


@pytest.mark.parametrize("sweeps", [1])
def test_learned_moves_keep_boltzmann(sweeps):
    """Cell moves interleaved 1:1 with sweeps sample the Boltzmann law: slot mean energies
    against exact enumeration (random, untrained network)."""
    params = initial_params(21)
    sysm, E, es, acc = _run_learned_chain(params, 2000, sweeps)
    assert acc > 0
    burn = len(es) // 10
    for k in range(sysm.K):
        m, sd = exact.batch_mean_sigma(es[burn:, k], 20)
        ref = exact.mean_energy(E, float(sysm.beta[k]))
        assert abs(m - ref) < 5 * sd + 0.05, (k, m, ref, sd)
