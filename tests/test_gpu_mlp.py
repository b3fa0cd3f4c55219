"""GPU parity of the selector's regressor (include/tn_mlp.h) against the FP64
reference in oracle/mlp.py.

The device keeps parameters and activations in FP32 and sums gradient partials
in FP64.  Bars, derived from FP32 rounding through two tanh layers of width
<= 64 (unit roundoff 6e-8, <= 64-term dot products, |activations| <= 1):
predictions within 1e-4 (1 + |f|); gradients within 1e-4 in relative 2-norm;
one Adam step exact to 1e-5 lr wherever the oracle gradient is not tiny
(|g| > 1e-3 max|g|), and a valid step (|dp| <= lr (1 + 1e-5)) elsewhere, since
the first Adam step is lr g / (|g| + 1e-8) and flips with the sign of g.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    return T


def _data(n, d, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    w = rng.standard_normal(d) / np.sqrt(d)
    y = (np.sin(2.0 * X @ w) + 0.1 * rng.standard_normal(n)).astype(np.float32)
    return X, y


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_layout_and_seeded_init(T):
    from oracle import mlp
    a, b, c = T.MLP(20, 64, seed=3), T.MLP(20, 64, seed=3), T.MLP(20, 64, seed=4)
    assert a.num_params == mlp.n_params(20, 64)
    pa, pb, pc = a.params(), b.params(), c.params()
    assert np.array_equal(pa, pb) and not np.array_equal(pa, pc)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(pa, 20, 64)
    # Glorot-uniform bounds, zero biases
    assert np.abs(W1).max() <= np.sqrt(6.0 / 84) and np.abs(W2).max() <= np.sqrt(6.0 / 128)
    assert np.abs(W3).max() <= np.sqrt(6.0 / 65)
    assert not b1.any() and not b2.any() and b3 == 0.0


@pytest.mark.parametrize("n,d,h", [(1, 20, 64), (63, 20, 64), (1000, 20, 64), (777, 7, 33), (300, 40, 96)])
def test_predict_matches_oracle(T, n, d, h):
    from oracle import mlp
    net = T.MLP(d, h, seed=n)
    rng = np.random.default_rng(n)
    p = (rng.standard_normal(net.num_params) * 0.3).astype(np.float32)
    net.set_params(p)
    X, _ = _data(n, d, n + 1)
    got = net.predict(_dev(X)).cpu().numpy().astype(np.float64)
    ref = mlp.forward(p, X, d, h)
    assert np.all(np.abs(got - ref) <= 1e-4 * (1 + np.abs(ref)))


def test_predict_empty(T):
    import torch
    net = T.MLP(5, 8, seed=1)
    out = net.predict(torch.empty((0, 5), dtype=torch.float32, device="cuda"))
    assert out.numel() == 0


@pytest.mark.parametrize("n,d,h", [(1, 20, 64), (200, 20, 64), (4096, 20, 64), (129, 3, 17)])
def test_grad_matches_oracle(T, n, d, h):
    from oracle import mlp
    net = T.MLP(d, h, seed=7 + n)
    X, y = _data(n, d, 11 + n)
    g, loss = net.grad(_dev(X), _dev(y))
    p = net.params()
    lref, gref = mlp.loss_and_grad(p, X, y, d, h)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss - lref) <= 1e-4 * max(lref, 1e-3)
    assert np.linalg.norm(g - gref) <= 1e-4 * np.linalg.norm(gref)


def test_adam_steps_match_oracle(T):
    from oracle import mlp
    d, h, n, lr = 20, 64, 500, 1e-3
    net = T.MLP(d, h, seed=21)
    X, y = _data(n, d, 22)
    p0 = net.params().astype(np.float64)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    Xd, yd = _dev(X), _dev(y)
    for t in range(1, 4):
        _, g = mlp.loss_and_grad(p, X, y, d, h)
        pn, m, v = mlp.adam_step(p, g, m, v, t, lr)
        net.step(Xd, yd, lr)
        got = net.params().astype(np.float64)
        big = np.abs(g) > 1e-3 * np.abs(g).max()
        assert big.mean() > 0.5
        if t == 1:
            assert np.all(np.abs((got - pn)[big]) <= 1e-5 * lr + 1e-7 * np.abs(pn[big]))
            assert np.all(np.abs(got - p) <= lr * (1 + 1e-5) + 1e-7 * np.abs(p))
        else:
            # the moments now carry each side's own rounding: compare in norm
            assert np.linalg.norm((got - pn)[big]) <= 1e-3 * lr * np.sqrt(big.sum())
        p = got
    l3, _ = mlp.loss_and_grad(p, X, y, d, h)
    l0, _ = mlp.loss_and_grad(p0, X, y, d, h)
    assert l3 < l0


def test_training_reduces_loss_and_reports_it(T):
    from oracle import mlp
    d, h, n = 20, 64, 6000
    X, y = _data(n, d, 31)
    net = T.MLP(d, h, seed=32)
    l0, _ = mlp.loss_and_grad(net.params(), X, y, d, h)
    losses = net.train(_dev(X), _dev(y), batch=1000, epochs=60, lr=3e-3)
    assert losses.shape == (60,) and np.all(np.isfinite(losses))
    lend, _ = mlp.loss_and_grad(net.params(), X, y, d, h)
    assert lend < 0.2 * l0
    assert losses[-1] < 0.3 * losses[0]
    # the reported epoch loss is the running mean over the epoch's batches; the
    # last epoch's should sit close to the final full-data loss
    assert abs(losses[-1] - lend) <= 0.25 * lend + 1e-3


def test_too_large_is_rejected(T):
    with pytest.raises(T.TNError):
        T.MLP(256, 128, seed=0)
    with pytest.raises(T.TNError):
        T.MLP(0, 8, seed=0)
