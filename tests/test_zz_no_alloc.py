"""The gradient step that allocates nothing (ising_mlp_grad_noalloc) against the
ordinary one (ising_mlp_grad, caller scratch), through the C ABI: two calls in a
row, the second with a smaller batch, each bit for bit equal to the ordinary
step on the same batch."""
import numpy as np
import pytest

from .gpu_util import say

pytestmark = pytest.mark.gpu


def _batch(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    x = np.zeros((n, 17), np.float32)
    x[:, 8:16] = rng.integers(-12, 13, (n, 8)) / 8.0  # boundary fields / 8
    x[:, 16] = rng.uniform(0.1, 3.0, n)                # beta
    y = rng.integers(0, 256, n).astype(np.uint8)
    return torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()


def test_noalloc_gradient_matches_the_scratch_entry_point():
    import torch

    import paper_1004_0024_amd as pa
    from gen.mlp import initial_params
    net = pa.Mlp(initial_params(5))
    batches = [_batch(4096, 1), _batch(777, 2)]  # second call smaller
    refs = []
    for x, y in batches:
        loss = net.grad_step(x, y)
        refs.append((net.grad.clone(), loss.clone()))
    for (x, y), (g_ref, l_ref) in zip(batches, refs):
        say("noalloc gradient, rows", x.shape[0])
        net.grad.fill_(float("nan"))
        loss = torch.full((1,), float("nan"), device="cuda")
        net.grad_step_noalloc(x, y, loss)
        torch.cuda.synchronize()
        assert torch.equal(net.grad, g_ref), f"gradient differs at {x.shape[0]} rows"
        assert torch.equal(loss, l_ref)
