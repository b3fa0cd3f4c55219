"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these compare the oracle with itself: each checks it against a closed
form, a library routine for a special case, the literal definition, an exact
enumeration over all hash functions, or the paper's statistical statements.
"""
import json
import math
import os

import numpy as np
import pytest

import tn_workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
P31 = 2**31 - 1


# --------------------------------------------------------------------------
# Hash family
# --------------------------------------------------------------------------

def test_splitmix64_reference_vectors(orc):
    vals = [int(l) for l in open(os.path.join(GOLD, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    state = 1234567
    for v in vals:
        assert orc.mix(state) == v
        state = (state + 0x9E3779B97F4A7C15) % 2**64


def _py_mix(x):
    z = (x + 0x9E3779B97F4A7C15) % 2**64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) % 2**64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) % 2**64
    return z ^ (z >> 31)


@pytest.mark.parametrize("seed,sample,stream", [(0, 0, 0), (7, 123, 5), (2**63 + 11, 99999, 1 << 62)])
def test_hash_family_exact_integers(orc, seed, sample, stream):
    """The C tables equal an arbitrary-precision evaluation of the stated family
    (no 64-bit overflow in the mod-P polynomial arithmetic)."""
    key = _py_mix(_py_mix(_py_mix(seed) ^ sample) ^ stream)
    raw = [_py_mix(key ^ j) >> 33 for j in range(6)]
    a0, a1 = raw[0] % P31, 1 + raw[1] % (P31 - 1)
    c = [r % P31 for r in raw[2:]]
    assert orc.hash_coeffs(seed, sample, stream) == [a0, a1] + c
    for m in (1, 3, 256, 4096, 65536):
        h, s = orc.hash_table(seed, sample, stream, 300, m)
        for i in range(0, 300, 7):
            assert h[i] == ((a1 * i + a0) % P31) % m
            poly = (c[3] * i**3 + c[2] * i**2 + c[1] * i + c[0]) % P31
            assert s[i] == (1 if poly % 2 == 0 else -1)


def test_hash_family_statistics(orc):
    """Buckets uniform, signs balanced and pairwise/4-wise uncorrelated over draws
    (Def. 10-11)."""
    m, n, R = 16, 6, 6000
    H = np.zeros((R, n), np.int64)
    S = np.zeros((R, n), np.int64)
    for r in range(R):
        H[r], S[r] = orc.hash_table(3, r, 0, n, m)
    counts = np.bincount(H.ravel(), minlength=m)
    expected = H.size / m
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert chi2 < 60.0          # 15 dof; p ~ 1e-7 cutoff
    assert abs(S.mean()) < 5 / math.sqrt(S.size)
    for (i, j) in [(0, 1), (2, 5)]:
        assert abs((S[:, i] * S[:, j]).mean()) < 5 / math.sqrt(R)
        assert abs((H[:, i] == H[:, j]).mean() - 1 / m) < 5 * math.sqrt(1 / m / R)
    assert abs((S[:, 0] * S[:, 1] * S[:, 2] * S[:, 3]).mean()) < 5 / math.sqrt(R)


# --------------------------------------------------------------------------
# Exact contraction
# --------------------------------------------------------------------------

def test_golden_triangle(orc):
    g = json.load(open(os.path.join(GOLD, "triangle_2x2_int.json")))
    net = W.triangle(2).with_data([np.array(g[k], dtype=np.float64) for k in "ABC"])
    assert orc.tc_full(net) == g["expected"]
    assert orc.tc_literal(net) == g["expected"]


def test_golden_example5_ones(orc):
    g = json.load(open(os.path.join(GOLD, "example5_ones.json")))
    net = W.example5(n=g["n"], dist="ones")
    assert orc.tc_full(net) == g["expected"]
    for root in range(net.p):
        assert orc.tc_tree(net, root) == g["expected"]


@pytest.mark.parametrize("n", [3, 5, 8])
def test_triangle_is_trace(orc, n):
    net = W.triangle(n, seed=n)
    A, B, C = net.data
    assert orc.tc_full(net) == pytest.approx(np.trace(A @ B @ C), rel=1e-12, abs=1e-12)


def test_ring_is_trace(orc):
    net = W.ring(5, 4, seed=3)
    ref = np.trace(np.linalg.multi_dot(net.data))
    assert orc.tc_full(net) == pytest.approx(ref, rel=1e-12)


def test_dot_and_matrix_product(orc):
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(7), rng.standard_normal(7)
    dot = W.Network([1, 1], [7, 7], [(0, 1)], [x, y])
    assert orc.tc_full(dot) == pytest.approx(float(x @ y), rel=1e-13)
    A, B = rng.standard_normal((3, 4)), rng.standard_normal((4, 5))
    mm = W.Network([2, 2], [3, 4, 4, 5], [(1, 2)], [A, B])   # AB = tc(A x B, {(2,3)})
    np.testing.assert_allclose(orc.tc_literal(mm), A @ B, rtol=1e-13)


def test_example1_partial(orc):
    """Example 1: Y(i2, i8) = sum X1(i1) X2(i2,i3) X3(i3,i1,i6) X4(i6,i8)."""
    net = W.example1()
    X1, X2, X3, X4 = net.data
    ref = np.einsum("a,bc,cad,de->be", X1, X2, X3, X4)
    np.testing.assert_allclose(orc.tc_literal(net), ref, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("maker", [
    lambda: W.triangle(3, seed=4),
    lambda: W.ring(4, 2, seed=5),
    lambda: W.example5(n=2, seed=6),
    lambda: W.torus(L=2, D=2, seed=7, dtype=np.float64),
    lambda: W.random_network(9, 3, dtype=np.float64, bmax=3, pmax=5),
])
def test_reduced_equals_literal_definition(orc, maker):
    net = maker()
    assert orc.tc_full(net) == pytest.approx(orc.tc_literal(net), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("maker", [
    lambda: W.example5(n=3, seed=1),
    lambda: W.tt_caterpillar(cores=5, bond=3, phys=4, seed=2, dtype=np.float64),
    lambda: W.chain([3, 4, 2, 5], seed=3),
])
def test_lemma8_tree_recursion(orc, maker):
    net = maker()
    ref = orc.tc_full(net)
    for root in range(net.p):
        assert orc.tc_tree(net, root) == pytest.approx(ref, rel=1e-11, abs=1e-13)


# --------------------------------------------------------------------------
# DFT / convolution conventions
# --------------------------------------------------------------------------

@pytest.mark.parametrize("m", [1, 2, 8, 64, 1024])
def test_fft_matches_library_and_definition(orc, m):
    rng = np.random.default_rng(m)
    x = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    np.testing.assert_allclose(orc.fft(x), np.fft.fft(x), atol=1e-9 * max(1, m))
    if m <= 64:
        np.testing.assert_allclose(orc.dft(x), np.fft.fft(x), atol=1e-10 * max(1, m))
    np.testing.assert_allclose(orc.fft(orc.fft(x), inverse=True), x, atol=1e-12 * max(1, m))


def test_convolution_theorem(orc):
    """Lemma 1: F(x*y) = Fx o Fy."""
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(32), rng.standard_normal(32)
    np.testing.assert_allclose(np.fft.fft(orc.circ_conv(x, y)), np.fft.fft(x) * np.fft.fft(y),
                               atol=1e-10)


# --------------------------------------------------------------------------
# Method 1
# --------------------------------------------------------------------------

def _cs(h, s, x, m):
    out = np.zeros(m)
    np.add.at(out, h, s * x)
    return out


def test_m1_combine_routes_agree(orc):
    """Eq. (1) via the DFT equals the direct circular convolution at index 0 (Lemma 1)."""
    net = W.triangle(6, seed=2)
    for s in range(5):
        a = orc.m1_estimate(net, 32, 4, s)["estimate"]
        b = orc.m1_estimate(net, 32, 4, s, combine="dft")["estimate"]
        assert a == pytest.approx(b, rel=1e-10, abs=1e-10)


def test_m1_single_edge_is_count_sketch_inner_product(orc):
    """One contraction: the estimate is (Cx)^T (Cy) (Lemma 2's estimator), since the
    second mode gets the complement sketch (Def. 14, Lemma 5)."""
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(50), rng.standard_normal(50)
    net = W.Network([1, 1], [50, 50], [(0, 1)], [x, y])
    for m in (1, 7, 64):
        for s in range(4):
            h, sg = orc.hash_table(11, s, 0, 50, m)
            ref = _cs(h, sg, x, m) @ _cs(h, sg, y, m)
            assert orc.m1_estimate(net, m, 11, s)["estimate"] == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_m1_complement_lemma5(orc):
    """F C' x = conj(F C x): the second mode's sketch is the circular reversal."""
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal(20), rng.standard_normal(20)
    net = W.Network([1, 1], [20, 20], [(0, 1)], [x, y])
    m = 16
    sk = orc.m1_estimate(net, m, 5, 2, want_sketches=True)["sketches"]
    h, sg = orc.hash_table(5, 2, 0, 20, m)
    np.testing.assert_allclose(sk[0], _cs(h, sg, x, m), atol=1e-13)
    np.testing.assert_allclose(np.fft.fft(sk[1]), np.conj(np.fft.fft(_cs(h, sg, y, m))), atol=1e-12)


def test_m1_single_edge_exact_variance(orc):
    """Enumeration over all fully random (h, s): mean x^T y and variance
    (1/m)(|x|^2|y|^2 + (x^T y)^2 - 2 sum x_i^2 y_i^2) (count-sketch inner product,
    cf. Lemma 2), which is <= (2/m)|x|^2|y|^2."""
    x, y = np.array([1.5, -2.0, 0.5]), np.array([0.25, 1.0, -3.0])
    net = W.Network([1, 1], [3, 3], [(0, 1)], [x, y])
    for m in (2, 3):
        mean, var, cnt = orc.m1_enumerate(net, m)
        assert cnt == (2 * m) ** 3
        ref = (x @ x * (y @ y) + (x @ y) ** 2 - 2 * np.sum(x**2 * y**2)) / m
        assert mean == pytest.approx(x @ y, rel=1e-12)
        assert var == pytest.approx(ref, rel=1e-10)
        assert var <= 2 / m * (x @ x) * (y @ y)


@pytest.mark.parametrize("m", [2, 3])
def test_m1_enumeration_unbiased_cyclic(orc, m):
    """Lemma 6 on the cyclic triangle: the exact mean over all hash functions is
    tc, and the exact variance is below 3^t/m prod ||X_k||^2."""
    net = W.triangle(2, seed=8)
    mean, var, cnt = orc.m1_enumerate(net, m)
    assert cnt == (2 * m) ** 6
    assert mean == pytest.approx(orc.tc_full(net), rel=1e-12, abs=1e-12)
    assert var <= 3**3 / m * net.input_norm() ** 2


def test_m1_injective_hashes_exact(orc):
    """Collision-free buckets and +1 signs make Eq. (1) exact: with bucket i*B^e
    (B = 2n, m = B^t) the combined bucket is 0 mod m only when every contracted
    index pair agrees."""
    for net in (W.triangle(2, seed=1), W.triangle(3, seed=2), W.ring(4, 2, seed=3)):
        n = net.dims[0]
        B = 2 * n
        m = B**net.t
        tables = []
        for e in range(net.t):
            h = np.arange(n) * B**e
            tables.append(np.concatenate([h, np.ones(n, np.int64)]))
        est = orc.m1_estimate(net, m, 0, 0, tables=tables)["estimate"]
        assert est == pytest.approx(orc.tc_full(net), rel=1e-12, abs=1e-12)


def test_m1_degenerate_hashes(orc):
    """h = 0, s = +1: every tensor collapses to its entry sum, and the estimate is
    prod_k sum_i X_k(i).  m = 1: prod_k <X_k, kron of signs>."""
    net = W.triangle(4, seed=9)
    tables = [np.concatenate([np.zeros(4, np.int64), np.ones(4, np.int64)])] * 3
    for m in (1, 5, 16):
        est = orc.m1_estimate(net, m, 0, 0, tables=tables)["estimate"]
        assert est == pytest.approx(np.prod([x.sum() for x in net.data]), rel=1e-12)
    est = orc.m1_estimate(net, 1, 21, 3)["estimate"]
    sg = [orc.hash_table(21, 3, e, 4, 1)[1] for e in range(3)]
    A, B, C = net.data     # A modes (0,1) edges e2 (owner), e0 (owner); B: e0', e1; C: e1', e2'
    ref = (sg[2] @ A @ sg[0]) * (sg[0] @ B @ sg[1]) * (sg[1] @ C @ sg[2])
    assert est == pytest.approx(ref, rel=1e-12)


def test_m1_statistics_triangle(orc):
    """Lemma 6 by Monte Carlo over the hash family: mean within 5 standard errors of
    tc and the sample variance below the bound; Gaussian data give variance close
    to prod ||X||^2 / m."""
    net = W.triangle(8, seed=10)
    m, K = 64, 3000
    est = np.array([orc.m1_estimate(net, m, 17, r)["estimate"] for r in range(K)])
    tc = orc.tc_full(net)
    mu, var = orc.mean_var(est)
    bound = 3**3 / m * net.input_norm() ** 2
    assert abs(mu - tc) <= 5 * math.sqrt(bound / K)
    assert var <= bound
    assert 0.5 < var / (net.input_norm() ** 2 / m) < 2.0


def test_mean_var(orc):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(1000) * 3 + 1
    mu, var = orc.mean_var(x)
    assert mu == pytest.approx(x.mean(), rel=1e-12)
    assert var == pytest.approx(x.var(ddof=1), rel=1e-12)


def test_median_of_means_special_cases(orc):
    import statistics
    # a worked case: S = 7, G = 3 -> groups [0,2) [2,4) [4,7)
    x = [1.0, 3.0, 10.0, 20.0, -4.0, 0.0, 1.0]
    assert orc.median_of_means(x, 3) == 2.0          # means 2, 15, -1 -> median 2
    # even G: the mean of the two middle group means
    assert orc.median_of_means([5.0, 1.0, 3.0, 100.0], 4) == 4.0
    rng = np.random.default_rng(9)
    y = rng.standard_normal(101)
    assert orc.median_of_means(y, 1) == pytest.approx(float(np.mean(y)), rel=1e-14)
    assert orc.median_of_means(y, 101) == statistics.median(y.tolist())
    # the median ignores one wild group that the mean does not
    z = np.ones(90)
    z[:10] = 1e6
    assert orc.median_of_means(z, 9) == 1.0


# --------------------------------------------------------------------------
# Method 2
# --------------------------------------------------------------------------

def _tree_streams(net, root):
    """Children per tensor, in mode order, from a breadth-first orientation."""
    partner = {}
    for (u, v) in net.edges:
        partner[u], partner[v] = v, u
    parent_mode = {root: None}
    children = {}
    queue = [root]
    while queue:
        k = queue.pop(0)
        children[k] = []
        for u in net.modes(k):
            if u == parent_mode[k]:
                continue
            l = net.tensor_of(partner[u])
            parent_mode[l] = partner[u]
            children[k].append(l)
            queue.append(l)
    return children


def test_m2_injective_hashes_exact(orc):
    """With identity count sketches (h(i) = i, s = +1), collision-free tensor
    sketches (u, w) -> u + n w and padding at index 0, every recursive sketch is an
    isometric embedding, so Eq. (2) reproduces the exact contraction."""
    for net in (W.example5(n=2, seed=3), W.chain([2, 2, 2], seed=4),
                W.tt_caterpillar(cores=3, bond=2, phys=2, seed=5, dtype=np.float64)):
        n = net.dims[0]
        m = 4096
        children = _tree_streams(net, 0)
        tables = {}
        for e in range(net.t):
            tables[e] = (np.arange(n), np.ones(n, np.int64))
        ident = np.arange(m)
        for k, ch in children.items():
            c = len(ch)
            if c == 0:
                continue
            qt = 1
            while qt < c:
                qt *= 2
            # every level multiplies the span of the right operand by the width so far
            width = n
            l = qt
            while l >= 2:
                for j in range(l // 2):
                    tables[orc.stream_tsketch(k, l, j, 0)] = (ident % m, np.ones(m, np.int64))
                    tables[orc.stream_tsketch(k, l, j, 1)] = ((ident * width) % m, np.ones(m, np.int64))
                width = width * width
                l //= 2
            for j in range(c, qt):
                tables[orc.stream_pad(k, j)] = (np.zeros(1, np.int64), np.ones(1, np.int64))
        est = orc.m2_estimate(net, m, 0, 0, root=0, tables=tables)["estimate"]
        assert est == pytest.approx(orc.tc_full(net), rel=1e-11, abs=1e-12)


@pytest.mark.parametrize("maker,m,K", [
    (lambda: W.example5(n=3, seed=1), 16, 3000),
    (lambda: W.tt_caterpillar(cores=5, bond=4, phys=3, seed=2, dtype=np.float64), 64, 2000),
])
def test_m2_statistics(orc, maker, m, K):
    """Lemma 9 by Monte Carlo: mean within 5 standard errors of the Lemma 8 value and
    the sample variance below ((1 + 8/m)^{2t} - 1) prod ||X_k||^2."""
    net = maker()
    est = np.array([orc.m2_estimate(net, m, 23, r)["estimate"] for r in range(K)])
    tc = orc.tc_tree(net, 0)
    mu, var = orc.mean_var(est)
    bound = ((1 + 8 / m) ** (2 * net.t) - 1) * net.input_norm() ** 2
    assert abs(mu - tc) <= 5 * math.sqrt(var / K)
    assert var <= bound


def test_m2_leaf_sketch_and_root(orc):
    """Example 5's leaves are plain count sketches x_l = C_{k,l} X_l, and the
    estimate is the inner product x_o^T r_o (Algorithm 2)."""
    net = W.example5(n=4, seed=7)
    m = 32
    out = orc.m2_estimate(net, m, 3, 1, want_trace=True)
    # X5 hangs off X2 through edge (4, 9) = edge index 3
    h, s = orc.hash_table(3, 1, 3, 4, m)
    np.testing.assert_allclose(out["x"][4], _cs(h, s, net.data[4], m), atol=1e-13)
    assert out["estimate"] == pytest.approx(out["x"][0] @ out["r_root"], rel=1e-12, abs=1e-12)


def test_m2_single_edge_is_count_sketch_inner_product(orc):
    """Two vectors: R_o = C and x_l = C y, so the estimate is (Cx)^T(Cy)."""
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(30), rng.standard_normal(30)
    net = W.Network([1, 1], [30, 30], [(0, 1)], [x, y])
    for s in range(3):
        h, sg = orc.hash_table(2, s, 0, 30, 16)
        ref = _cs(h, sg, x, 16) @ _cs(h, sg, y, 16)
        assert orc.m2_estimate(net, 16, 2, s)["estimate"] == pytest.approx(ref, rel=1e-12)


def test_bf16_rounding_matches_torch(orc):
    """The oracle's BF16 operand rounding (ties to even, through FP32) against
    torch's CPU conversion, on random values, exact ties, and values that
    round differently from FP64 straight to BF16."""
    import torch
    rng = np.random.default_rng(3)
    xs = list(rng.standard_normal(2000) * 10.0 ** rng.integers(-20, 20, 2000))
    xs += [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 2.0 ** -130, 0.0, -0.0, 3.0e38]
    xs += [1.0 + 2.0 ** -8 + 2.0 ** -40]          # above the tie in FP64, a tie once rounded to FP32
    ref = torch.tensor(xs, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([orc.bf16_round(x) for x in xs])
    assert np.array_equal(got, ref)


def test_bf16_products_exact_on_small_integers(orc):
    """With integer entries small enough that every operand of every product
    (entries and sketch values) is a BF16 integer, the BF16-product variant of
    Method 2 equals the FP64 estimator up to the FP64 rounding of the
    latter's FFT-form tensor sketches (which the BF16 rounding removes)."""
    tree = W.example5(n=3, seed=2, dist="int")
    for r in range(4):
        a = orc.m2_estimate(tree, 16, 5, r, want_trace=True)
        b = orc.m2_estimate(tree, 16, 5, r, bf16_products=True)["estimate"]
        assert np.abs(a["r_root"]).max() <= 512 and np.allclose(a["r_root"], np.round(a["r_root"]), atol=1e-9)
        assert b == pytest.approx(a["estimate"], rel=1e-12, abs=1e-9)
        assert b == round(b)
    # and on Gaussian data it differs, by about BF16's rounding of the operands
    g = W.example5(n=4, seed=3)
    a = orc.m2_estimate(g, 64, 1, 0, want_trace=True)
    b = orc.m2_estimate(g, 64, 1, 0, want_trace=True, bf16_products=True)
    scale = np.linalg.norm(a["x"][0]) * np.linalg.norm(a["r_root"])
    assert 0 < abs(a["estimate"] - b["estimate"]) <= 2 * 2.0 ** -8 * scale
