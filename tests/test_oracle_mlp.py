"""Pins of the FP64 MLP reference: central finite differences, torch's CPU
autograd on the same function, and torch's CPU Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp


def _problem(d=5, h=7, n=23, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.n_params(d, h)) * 0.4
    X = rng.standard_normal((n, d))
    y = rng.standard_normal(n)
    return p, X, y, d, h


def test_gradient_finite_differences():
    p, X, y, d, h = _problem()
    _, g = mlp.loss_and_grad(p, X, y, d, h)
    eps = 1e-6
    for i in range(0, len(p), 3):
        e = np.zeros_like(p)
        e[i] = eps
        fd = (mlp.loss_and_grad(p + e, X, y, d, h)[0] - mlp.loss_and_grad(p - e, X, y, d, h)[0]) / (2 * eps)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_matches_torch_autograd():
    p, X, y, d, h = _problem(d=4, h=6, n=17, seed=3)
    W1, b1, W2, b2, W3, b3 = [torch.tensor(np.array(a), dtype=torch.float64, requires_grad=True)
                              for a in mlp.unpack(p, d, h)]
    Xt, yt = torch.tensor(X), torch.tensor(y)
    out = torch.nn.functional.linear(torch.tanh(torch.nn.functional.linear(
        torch.tanh(torch.nn.functional.linear(Xt, W1, b1)), W2, b2)), W3.unsqueeze(0), b3.reshape(1))
    loss = 0.5 * torch.mean((out.squeeze(1) - yt) ** 2)
    loss.backward()
    ref = torch.cat([W1.grad.reshape(-1), b1.grad, W2.grad.reshape(-1), b2.grad, W3.grad,
                     b3.grad.reshape(1)]).numpy()
    l, g = mlp.loss_and_grad(p, X, y, d, h)
    assert l == pytest.approx(loss.item(), rel=1e-13)
    np.testing.assert_allclose(g, ref, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(mlp.forward(p, X, d, h), out.detach().numpy()[:, 0], rtol=1e-13)


def test_adam_matches_torch():
    rng = np.random.default_rng(1)
    p = rng.standard_normal(11)
    m = np.zeros(11)
    v = np.zeros(11)
    pt = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=3e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.standard_normal(11)
        p, m, v = mlp.adam_step(p, g, m, v, t, 3e-2)
        opt.zero_grad()
        pt.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)
