"""FP64 reference of the selector's regressor (TEST INFRASTRUCTURE ONLY).

A 3-layer perceptron f(x) = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3 with the
parameter layout of include/tn_mlp.h, the loss L = 0.5 mean((f(X) - y)^2), its
gradient by the chain rule written out layer by layer, and one bias-corrected
Adam step (Kingma & Ba 2015: beta1 0.9, beta2 0.999, eps 1e-8).  Plain numpy
in float64; shares no code with the device kernels.
"""
import numpy as np


def n_params(d, h):
    return h * d + h + h * h + h + h + 1


def unpack(p, d, h):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + h * d].reshape(h, d); o += h * d
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    W3 = p[o:o + h]; o += h
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def forward(p, X, d, h):
    W1, b1, W2, b2, W3, b3 = unpack(p, d, h)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3 + b3


def loss_and_grad(p, X, y, d, h):
    W1, b1, W2, b2, W3, b3 = unpack(p, d, h)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = X.shape[0]
    a1 = X @ W1.T + b1
    h1 = np.tanh(a1)
    a2 = h1 @ W2.T + b2
    h2 = np.tanh(a2)
    out = h2 @ W3 + b3
    r = out - y
    loss = 0.5 * np.mean(r * r)
    dout = r / n                          # dL/dout
    gW3 = h2.T @ dout
    gb3 = dout.sum()
    dh2 = np.outer(dout, W3)
    da2 = dh2 * (1.0 - h2 * h2)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (1.0 - h1 * h1)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return loss, g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """Step t (1-based): returns updated (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
