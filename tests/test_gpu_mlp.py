"""Network kernels of the learned proposal (BF16 MFMA, FP32 sums) against the
oracle's BF16 mirror and FP64 reference."""
import numpy as np
import pytest

from gen.mlp import initial_params
from oracle import learned as L

from .gpu_util import say

pytestmark = pytest.mark.gpu


def _data(n, seed):
    rng = np.random.default_rng(seed)
    b = rng.integers(-20, 21, size=(n, 8))
    beta = rng.uniform(0.1, 3.0, n)
    x = L.features(b, beta)
    y = rng.integers(0, 2, size=(n, 8))
    ybytes = (y * (1 << np.arange(8))).sum(1).astype(np.uint8)
    return x, y.astype(np.float64), ybytes


def _params(seed):
    p = initial_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed + 1)
    p[-8:] = rng.normal(size=8) * 0.3
    p[128 * 17:128 * 17 + 128] = rng.normal(size=128) * 0.1  # b1
    return p


@pytest.mark.parametrize("n", [1, 31, 32, 33, 1000])
def test_forward_matches_bf16_mirror(n):
    import torch
    import paper_1004_0024_amd as pa
    say("mlp forward n", n)
    p = _params(1)
    x, _, _ = _data(n, 2)
    net = pa.Mlp(p)
    got = net.forward(torch.from_numpy(x).float().cuda()).cpu().numpy().astype(np.float64)
    ref16, _ = L.forward_bf16(L.unpack(p), x)
    ref64, _ = L.forward(L.unpack(p), x)
    scale = 1.0 + np.abs(ref64).max()
    assert np.abs(got - ref16).max() < 2e-3 * scale, np.abs(got - ref16).max()
    assert np.abs(got - ref64).max() < 2e-2 * scale


@pytest.mark.parametrize("n", [32, 45, 4096])
def test_gradient_matches_oracle(n):
    import torch
    import paper_1004_0024_amd as pa
    say("mlp grad n", n)
    p = _params(3)
    x, y, yb = _data(n, 4)
    net = pa.Mlp(p)
    loss = net.grad_step(torch.from_numpy(x).float().cuda(), torch.from_numpy(yb).cuda())
    g = net.grad.cpu().numpy().astype(np.float64)
    pp = L.unpack(p)
    l16, c16 = L.forward_bf16(pp, x)
    g16 = L.pack(L.backward_bf16(pp, c16, l16, y))
    l64, c64 = L.forward(pp, x)
    g64 = L.pack(L.backward(pp, c64, l64, y))
    cos16 = g @ g16 / np.linalg.norm(g) / np.linalg.norm(g16)
    cos64 = g @ g64 / np.linalg.norm(g) / np.linalg.norm(g64)
    assert cos16 > 0.9999 and cos64 > 0.999, (cos16, cos64)
    assert np.linalg.norm(g - g16) < 2e-2 * np.linalg.norm(g16)
    # each parameter block separately
    o = 0
    for name, shape in [("W1", (128, 17)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
                        ("W3", (8, 128)), ("b3", (8,))]:
        k = int(np.prod(shape))
        assert np.linalg.norm(g[o:o + k] - g16[o:o + k]) < 3e-2 * np.linalg.norm(g16[o:o + k]) + 1e-7, name
        o += k
    assert abs(float(loss.item()) - L.nll(l64, y)) < 1e-2 * abs(L.nll(l64, y))


def test_adam_step_matches_oracle():
    import torch
    import paper_1004_0024_amd as pa
    p = _params(5)
    x, y, yb = _data(256, 6)
    net = pa.Mlp(p)
    opt = L.Adam(p.copy(), lr=1e-3)
    for step in range(3):
        net.grad_step(torch.from_numpy(x).float().cuda(), torch.from_numpy(yb).cuda())
        g = net.grad.cpu().numpy().astype(np.float64)
        net.adam(1e-3)
        opt.step(g)
    w = net.w.cpu().numpy().astype(np.float64)
    assert np.abs(w - opt.w).max() < 1e-5
    assert net.steps == 3


def test_training_reduces_loss():
    """Rows whose targets follow the inputs (spin k = sign of b_k): the loss falls."""
    import torch
    import paper_1004_0024_amd as pa
    rng = np.random.default_rng(7)
    b = rng.integers(-6, 7, size=(4096, 8))
    b[b == 0] = 1
    x = L.features(b, rng.uniform(0.5, 2.0, 4096))
    y = (b > 0).astype(np.uint8)
    yb = (y * (1 << np.arange(8))).sum(1).astype(np.uint8)
    net = pa.Mlp(initial_params(8))
    xt, yt = torch.from_numpy(x).float().cuda(), torch.from_numpy(yb).cuda()
    first = float(net.grad_step(xt, yt).item())
    for _ in range(150):
        net.grad_step(xt, yt)
        net.adam(3e-3)
    last = float(net.grad_step(xt, yt).item())
    say("loss", first, "->", last)
    assert last < 0.5 * first


@pytest.mark.parametrize("n", [4113, 9000])
def test_gradient_many_workgroups_reproducible(n):
    """More tiles than partial-gradient slots (some workgroups take several tiles):
    the gradient matches the mirror and two calls agree bit for bit."""
    import torch
    import paper_1004_0024_amd as pa
    p = _params(9)
    x, y, yb = _data(n, 10)
    net = pa.Mlp(p)
    xt, yt = torch.from_numpy(x).float().cuda(), torch.from_numpy(yb).cuda()
    l1 = net.grad_step(xt, yt).clone()
    g1 = net.grad.clone()
    l2 = net.grad_step(xt, yt)
    assert torch.equal(g1, net.grad) and torch.equal(l1, l2)
    g = g1.cpu().numpy().astype(np.float64)
    pp = L.unpack(p)
    l16, c16 = L.forward_bf16(pp, x)
    g16 = L.pack(L.backward_bf16(pp, c16, l16, y))
    assert g @ g16 / np.linalg.norm(g) / np.linalg.norm(g16) > 0.9999
    assert abs(float(l1.item()) - L.nll(L.forward(pp, x)[0], y)) < 1e-2
