"""CPU pins of the oracle's earlier cross-correlation estimator (Examples 2-3
of the Methods section) and of the all-ones-chain variance behind Lemma 7.

The estimator: one count sketch C_e per contraction, used by both of its
modes; tensor sketches of every tensor; e_1^T (y_1 star ... star y_p) with the
circular cross-correlation of Def. 9 applied left to right.

Pins that do not restate the oracle:
  * Def. 9 by hand and through Lemma 1 (F(x star y) = conj(F x) o F y), with
    numpy's FFT;
  * a single contraction reduces to the count-sketch inner product
    (C x)^T (C y) of Lemma 2, per seed;
  * exact enumeration over all fully random hash functions: unbiased on the
    chain of Example 2 and on an even ring (every contraction joins an
    unconjugated and a conjugated tensor); on odd cycles (the triangle of
    Example 3, a ring of five) the mean is gcd(2, m)/m times tc -- the
    contraction whose two tensors are both unconjugated (or both conjugated)
    only survives at the frequencies j with 2j = 0 mod m (derived here: for
    that contraction E[s(i) s(i') w^(j(h(i) + h(i')))] = [i = i'] [2j = 0 mod m]);
  * the all-ones chain of Lemma 7 (q contractions, n indices each): with
    V_i = F C_i 1, the proof rewrites the estimate as
    (1/m) sum_j prod_i |V_i[j]|^2, and for one count sketch
    E|V[j]|^2 |V[j']|^2 = n^2 + n (n - 1) ([j + j' = 0] + [j = j']) (mod m),
    so Var = (1/m^2) sum_{j,j'} (n^2 + n(n-1)([j+j'=0] + [j=j']))^q - n^(2q)
    (derived here).  Enumeration must reproduce it, for the cross-correlation
    chain and for Method 1 alike (on a chain the two have one distribution).
    Lemma 7's bound (3^q / (2 m^2) - 1) n^(2q) holds once n is at least about
    q, but not at n = m = 2, q = 4, where the exact variance 1920 is below its
    2336.
"""
import math

import numpy as np
import pytest

import tn_workloads as W


def ones_chain(q, n):
    """Lemma 7's network: vector, q - 1 matrices, vector, all ones; contraction
    i joins the second mode of tensor i with the first of tensor i + 1."""
    orders = [1] + [2] * (q - 1) + [1]
    edges = [(2 * i, 2 * i + 1) for i in range(q)]
    data = [np.ones(n)] + [np.ones((n, n)) for _ in range(q - 1)] + [np.ones(n)]
    return W.Network(orders, [n] * (2 * q), edges, data)


def chain_variance(q, n, m):
    """Closed form of the all-ones chain's estimator variance (see above)."""
    tot = 0.0
    for j in range(m):
        for jj in range(m):
            g = n * n + n * (n - 1) * (((j + jj) % m == 0) + (j == jj))
            tot += float(g) ** q
    return tot / (m * m) - float(n) ** (2 * q)


def test_circ_xcorr_definition_and_lemma1(orc):
    x = np.array([1.0, 2.0, 3.0])
    y = np.array([4.0, 5.0, 6.0])
    # (x star y)_j = sum_i x_i y_{(i + j) mod 3}
    assert np.allclose(orc.circ_xcorr(x, y), [1 * 4 + 2 * 5 + 3 * 6, 1 * 5 + 2 * 6 + 3 * 4, 1 * 6 + 2 * 4 + 3 * 5])
    rng = np.random.default_rng(3)
    for m in (1, 2, 7, 16):
        a, b = rng.standard_normal(m), rng.standard_normal(m)
        lhs = np.fft.fft(orc.circ_xcorr(a, b))
        assert np.allclose(lhs, np.conj(np.fft.fft(a)) * np.fft.fft(b), atol=1e-12)


@pytest.mark.parametrize("seed", [0, 5, 9])
def test_single_contraction_is_count_sketch_inner_product(orc, seed):
    rng = np.random.default_rng(seed)
    x, y = rng.standard_normal(20), rng.standard_normal(20)
    net = W.Network([1, 1], [20, 20], [(0, 1)], [x, y])
    for r in range(4):
        h, s = orc.hash_table(seed, r, 0, 20, 8)
        cx, cy = np.zeros(8), np.zeros(8)
        np.add.at(cx, h, s * x)
        np.add.at(cy, h, s * y)
        got = orc.xcorr_estimate(net, 8, seed, r)["estimate"]
        assert got == pytest.approx(float(cx @ cy), rel=1e-12, abs=1e-12)


def test_unbiased_on_chain_and_even_ring(orc):
    rng = np.random.default_rng(1)
    x, Y, z = rng.standard_normal(2), rng.standard_normal((2, 2)), rng.standard_normal(2)
    chain = W.Network([1, 2, 1], [2, 2, 2, 2], [(0, 1), (2, 3)], [x, Y, z])
    for m in (3, 4):
        mean, _, _ = orc.xcorr_enumerate(chain, m)
        assert mean == pytest.approx(float(x @ Y @ z), rel=1e-12, abs=1e-13)
    ring4 = W.ring(4, 2, seed=5)
    mean, _, _ = orc.xcorr_enumerate(ring4, 3)
    assert mean == pytest.approx(orc.tc_full(ring4), rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("m", [3, 4])
def test_biased_on_odd_cycles(orc, m):
    tri = W.triangle(2, seed=3)
    tc = orc.tc_full(tri)
    mean, _, _ = orc.xcorr_enumerate(tri, m)
    assert mean == pytest.approx(math.gcd(2, m) / m * tc, rel=1e-12, abs=1e-13)
    assert abs(mean - tc) > 0.3 * abs(tc)
    # Method 1 on the same network stays unbiased (Lemma 6)
    assert orc.m1_enumerate(tri, m)[0] == pytest.approx(tc, rel=1e-12, abs=1e-13)


def test_biased_on_five_ring(orc):
    ring5 = W.ring(5, 2, seed=6)
    tc = orc.tc_full(ring5)
    mean, _, _ = orc.xcorr_enumerate(ring5, 2)
    assert mean == pytest.approx(tc, rel=1e-12, abs=1e-13)    # gcd(2, 2)/2 = 1: no bias at m = 2
    ring5b = W.ring(5, 1, seed=6)
    mean, _, _ = orc.xcorr_enumerate(ring5b, 4)
    assert mean == pytest.approx(0.5 * orc.tc_full(ring5b), rel=1e-12, abs=1e-13)


@pytest.mark.parametrize("q,n,m", [(2, 2, 2), (2, 2, 3), (4, 2, 2), (2, 3, 4)])
def test_all_ones_chain_exact_variance(orc, q, n, m):
    net = ones_chain(q, n)
    mean, var, _ = orc.xcorr_enumerate(net, m)
    assert mean == pytest.approx(float(n) ** q, rel=1e-12)
    assert var == pytest.approx(chain_variance(q, n, m), rel=1e-10)
    mean1, var1, _ = orc.m1_enumerate(net, m)
    assert mean1 == pytest.approx(mean, rel=1e-12) and var1 == pytest.approx(var, rel=1e-10)


def test_lemma7_bound_needs_moderate_n():
    """The lower bound against the closed form.  For fixed n the closed form
    grows like ((3 - 2/n) n^2)^q, so the bound (which grows like 3^q n^(2q))
    needs n to grow with q: it fails at n = m = 2, q = 4 (exact 1920 < 2336)
    and, for instance, at n = 4, q = 10, m = 16, and holds for n >= q at every
    even q up to 12 and m in {2, 4, 16}."""
    def bound(q, n, m):
        return (3.0 ** q / (2.0 * m * m) - 1.0) * float(n) ** (2 * q)
    assert chain_variance(4, 2, 2) == 1920.0 and bound(4, 2, 2) == 2336.0
    assert chain_variance(10, 4, 16) < bound(10, 4, 16)
    for m in (2, 4, 16):
        for q in range(2, 13, 2):
            for n in (q, 2 * q, 8 * q):
                assert chain_variance(q, n, m) >= bound(q, n, m), (q, n, m)
