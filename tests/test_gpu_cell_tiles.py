"""Cell moves over a batch of unlike systems, so that the 64-row tiles of a colour
class cross walkers and systems: walkers of 72 rows (a tile holds the end of one
walker and the start of the next), of 4 rows (many walkers per tile), a ring of
odd length (four colour classes), and a system with no grid of cells (no rows).
Each system's pass is compared with the oracle's, with the global walker index
as the generator's counter, for the exact heat-bath draw and the learned
proposal."""
import numpy as np
import pytest

from gen import Workload, make_chimera_system, make_random_system
from gen.mlp import initial_params
from oracle import heatbath as H
from oracle import learned as L

from .gpu_util import chains_for, make_state, say

pytestmark = pytest.mark.gpu

SYSTEMS = [make_chimera_system(4, 9, 81, 7, ring=False),  # 16 cells x 9 slices: 72 rows per walker and class
           make_random_system(12, 18, 82, 3),          # no cells
           make_chimera_system(2, 3, 83, 5),           # 4 cells x 3 slices, ring of odd length: 4 classes
           make_chimera_system(3, 5, 84, 6, ring=False)]


def _run(kind):
    import torch

    import paper_1004_0024_amd as pa
    wl = Workload(f"cell tiles {kind}", SYSTEMS, 0, 1)
    g, st = make_state(wl)
    st.sweep(3, 1)
    idx = list(range(len(SYSTEMS)))
    chains = chains_for(wl, idx)
    for ch in chains:
        ch.sweeps(3, 1)
    moves = torch.zeros((g.R, 2), dtype=torch.int64, device="cuda")
    params = initial_params(21).astype(np.float64)
    if kind == "heatbath":
        st.heatbath_cells(key=555, pass_index=3, moves=moves)
    else:
        st.propose_cells(pa.Mlp(params), key=555, pass_index=3, moves=moves)
    mv = moves.cpu().numpy()
    obs = st.observables().cpu().numpy()
    assert np.array_equal(obs[:, 0], obs[:, 2]), "running energy must equal the recomputed cost"
    for s, (sysm, ch) in enumerate(zip(SYSTEMS, chains)):
        w0, w1 = int(wl.walker_base[s]), int(wl.walker_base[s + 1])
        gspins = st.spins_pm([s])[0]
        if getattr(sysm, "L", 0) == 0:  # no cells: untouched
            assert np.array_equal(gspins, ch.spins()), f"system {s} without cells changed"
            assert not mv[w0:w1].any()
            continue
        model = L.CellModel(sysm)
        spins = ch.spins().astype(np.int64)
        energy = ch.energy().copy()
        temp_of, _ = ch.labels()
        ids = list(range(w0, w1))
        if kind == "heatbath":
            hit = H.heatbath_pass(model, spins, energy, sysm.beta[temp_of], 555, ids, 3)
        else:
            hit = L.learned_pass(model, spins, energy, sysm.beta[temp_of], params, 555, ids, 3,
                                 forward_fn=L.forward_bf16)
        diff = sum(not np.array_equal(gspins[w][model.cell_spins(*c)], spins[w][model.cell_spins(*c)])
                   for w in range(sysm.K) for c in model.cells)
        ncells = sysm.K * len(model.cells)
        say(kind, "system", s, "cells", ncells, "differing", diff, "moved", int(hit.sum()))
        assert diff <= max(2, ncells // 200), f"system {s}: {diff} of {ncells} cells differ"
        assert int(mv[w0:w1, 0].sum()) == ncells, f"system {s}: rows visited"
        assert np.array_equal(mv[w0:w1, 0], np.full(sysm.K, len(model.cells))), f"system {s}: rows per walker"
        assert abs(int(mv[w0:w1, 1].sum()) - int(hit.sum())) <= max(2, ncells // 200)


def test_heatbath_pass_over_unlike_systems():
    _run("heatbath")


def test_learned_pass_over_unlike_systems():
    _run("learned")
