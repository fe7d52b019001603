"""The hand-written adjoint through torch.autograd: against the oracle's
adjoint for the same upstream gradient, against float64 finite differences of
the loss on 64x64 crops, and torch's gradcheck."""
import numpy as np
import pytest
import torch

import oracle
from paper_1708_07853_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def D():
    import paper_1708_07853_amd as d
    return d


def band_weights(w, h, levels):
    """2^k on the three H bands of level k, 0 on LL_L (packed layout)."""
    m = np.zeros((h, w), dtype=np.float32)
    sz = [(w, h)]
    for _ in range(levels):
        sz.append(((sz[-1][0] + 1) // 2, (sz[-1][1] + 1) // 2))
    for k in range(1, levels + 1):
        (wp, hp), (wk, hk) = sz[k - 1], sz[k]
        m[:hp, :wp] = 2.0 ** k
        m[:hk, :wk] = 0.0
    return m


def loss_oracle(x64, levels, m):
    return float(np.sum(m * np.abs(oracle.fwd(x64, levels))))


def test_function_matches_entry_points():
    d = D()
    x = torch.from_numpy(synth.channel_batch(2, 3, 96, 80)).cuda().requires_grad_()
    y = d.DWT2Function.apply(x, 3)
    assert torch.equal(y.detach(), d.fwd(x.detach(), 3))
    g = torch.randn_like(y)
    (gx,) = torch.autograd.grad(y, x, g)
    assert torch.equal(gx, d.bwd(g, 3))


def test_weighted_l1_gradient_equals_oracle_adjoint():
    """Config-5 shape: 32 x 3 x 1024 x 1024, 4 levels, loss sum_k 2^k |H_k|_1.
    The gradient is W^T (m * sign(c)); the oracle applies W^T to that same g."""
    d = D()
    levels = 4
    x = torch.from_numpy(synth.channel_batch(32, 3, 1024, 1024)).cuda().requires_grad_()
    m = torch.from_numpy(band_weights(1024, 1024, levels)).cuda()
    c = d.DWT2Function.apply(x, levels)
    loss = (m * c.abs()).sum()
    loss.backward()
    g = (m * torch.sign(c.detach()))
    for b, ch in [(0, 0), (17, 2), (31, 1)]:
        ref = oracle.adj(g[b, ch].cpu().numpy().astype(np.float64), levels)
        assert float(np.abs(x.grad[b, ch].cpu().numpy() - ref).max()) <= 2e-4


def test_loss_gradient_against_fd_on_crops():
    d = D()
    levels = 4
    img = synth.image(1024, 1024, 5000)
    rng = np.random.default_rng(5)
    m = band_weights(64, 64, levels)
    for _ in range(4):
        y0, x0 = (int(v) for v in rng.integers(0, 1024 - 64, size=2))
        # a small perturbation keeps every coefficient away from |.|'s kink
        crop = img[y0:y0 + 64, x0:x0 + 64].astype(np.float64) + rng.uniform(-0.3, 0.3, size=(64, 64))
        coeff = oracle.fwd(crop, levels)
        h = 1e-6
        if np.abs(coeff).min() < 100 * h:
            continue
        xt = torch.from_numpy(crop.astype(np.float32)).cuda().requires_grad_()
        c = d.DWT2Function.apply(xt, levels)
        (torch.from_numpy(m).cuda() * c.abs()).sum().backward()
        grad = xt.grad.cpu().numpy()
        for (py, px) in rng.integers(0, 64, size=(24, 2)):
            e = np.zeros_like(crop)
            e[py, px] = h
            fd = (loss_oracle(crop + e, levels, m) - loss_oracle(crop - e, levels, m)) / (2 * h)
            assert abs(fd - grad[py, px]) <= 2e-4 * max(1.0, abs(fd)), (py, px, fd, grad[py, px])


def test_linear_functional_fd():
    """phi(x) = <g, W x> with random g: its gradient is exactly W^T g."""
    d = D()
    levels = 4
    rng = np.random.default_rng(6)
    g = rng.normal(size=(64, 64))
    x = synth.image(64, 64, 77).astype(np.float64)
    grad = d.bwd(torch.from_numpy(g.astype(np.float32)).cuda(), levels).cpu().numpy()
    for (py, px) in rng.integers(0, 64, size=(32, 2)):
        e = np.zeros_like(x)
        e[py, px] = 1.0
        fd = (np.vdot(g, oracle.fwd(x + e, levels)) - np.vdot(g, oracle.fwd(x - e, levels))) / 2
        assert abs(fd - grad[py, px]) <= 2e-4 * max(1.0, abs(fd))


def test_torch_gradcheck_float32():
    d = D()
    x = torch.from_numpy(synth.image(13, 16, 3)).cuda().requires_grad_()
    assert torch.autograd.gradcheck(lambda t: d.DWT2Function.apply(t, 2), (x,), eps=0.5, atol=2e-3, rtol=1e-3)
