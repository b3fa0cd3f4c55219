"""Host-only checks of the library's (eps, delta) sizing (tn_sketch_size,
tn_median_groups): the median group count against scipy's binomial tail, and
the bound-driven choice (the variance bounds of Lemmas 6 and 9, Chebyshev and
the median trick of Theorem 1's proof) against the rule restated here.  The
bound mode reads no tensor data and makes no device call."""
import math

import numpy as np
import pytest
from scipy.stats import binom

import tn_workloads as W


@pytest.fixture(scope="module")
def T():
    import paper_2603_07387_amd as T
    T.load()
    return T


@pytest.mark.parametrize("delta", [0.2, 0.05, 0.01, 1e-3, 1e-6])
@pytest.mark.parametrize("p", [0.05, 0.1, 0.25, 0.4])
def test_median_groups_is_the_least_odd_count(T, delta, p):
    G = T.tn_median_groups(delta, p)
    assert G % 2 == 1
    assert binom.sf((G - 1) // 2, G, p) <= delta * (1 + 1e-9)       # P(X >= (G+1)/2)
    if G > 1:
        assert binom.sf((G - 3) // 2, G - 2, p) > delta


def _rule(net, method, eps, delta, max_groups):
    """The choice restated: v(m) from the bound, G = 1 with p = delta, or the
    least G S over p in 0.02 .. 0.48; least work G S (q N + p m log2 m)."""
    t = len(net.edges)
    ladder = [2 ** k for k in range(6, 14 if method == "acyclic" else 15)]
    N = float(sum(np.prod(net.shape(k)) for k in range(net.p)))
    q = float(np.mean(net.orders))
    best = None
    for m in ladder:
        v = 3.0 ** t / m if method == "cyclic" else (1 + 8.0 / m) ** (2 * t) - 1
        cands = [(1, delta, math.ceil(v / (delta * eps * eps)))]
        if max_groups > 1:
            for i in range(1, 25):
                pg = 0.02 * i
                G = 1
                while binom.sf((G - 1) // 2, G, pg) > delta:
                    G += 2
                if G <= max_groups:
                    cands.append((G, pg, math.ceil(v / (pg * eps * eps))))
        G, pg, S = min(cands, key=lambda c: c[0] * c[2])
        S = max(1, S)
        if S > 2 ** 20:
            continue
        w = G * S * (q * N + net.p * m * max(math.log2(m), 1))
        if best is None or w < best["work"]:
            best = {"m": m, "samples": S, "groups": G, "work": w}
    return best


@pytest.mark.parametrize("eps,delta,G", [(0.1, 0.05, 1), (0.05, 0.01, 1), (0.05, 0.01, 101), (1e-2, 1e-4, 999)])
def test_bound_choice_follows_the_rule(T, eps, delta, G):
    import torch
    cases = [(W.triangle(16), "cyclic"), (W.ring(5, 8), "cyclic"),
             (W.tt_caterpillar(cores=8, bond=8, phys=4), "acyclic"), (W.example5(n=4), "acyclic")]
    for net, method in cases:
        spec = T.NetworkSpec.from_network(net, dtype=torch.float32)
        got = T.tn_sketch_size([spec], T.TN_CYCLIC if method == "cyclic" else T.TN_ACYCLIC, eps, delta,
                               max_groups=G, mode=T.TN_SIZE_BOUND)[0]
        ref = _rule(net, method, eps, delta, G)
        assert (got["m"], got["samples"], got["groups"]) == (ref["m"], ref["samples"], ref["groups"]), (net, got, ref)
        assert got["work"] == pytest.approx(ref["work"], rel=1e-12)


def test_median_beats_plain_mean_at_small_delta(T):
    """At delta = 1e-4 Chebyshev alone needs S = v / (delta eps^2); the median
    of G groups with a constant miss probability needs far fewer samples."""
    import torch
    spec = T.NetworkSpec.from_network(W.triangle(16), dtype=torch.float32)
    one = T.tn_sketch_size([spec], T.TN_CYCLIC, 0.05, 1e-4, max_groups=1)[0]
    med = T.tn_sketch_size([spec], T.TN_CYCLIC, 0.05, 1e-4, max_groups=999)[0]
    assert med["groups"] > 1 and med["groups"] * med["samples"] < 0.2 * one["samples"]


def test_sizing_argument_errors(T):
    import torch
    spec = T.NetworkSpec.from_network(W.triangle(4), dtype=torch.float32)
    for args in [(0.0, 0.1), (0.1, 0.0), (0.1, 1.0)]:
        with pytest.raises(T.TNError) as e:
            T.tn_sketch_size([spec], T.TN_CYCLIC, *args)
        assert e.value.code == T.TN_ERR_ARG
    with pytest.raises(T.TNError) as e:
        T.tn_median_groups(0.1, 0.5)
    assert e.value.code == T.TN_ERR_ARG
    with pytest.raises(T.TNError) as e:   # a cyclic network under the acyclic method
        T.tn_sketch_size([spec], T.TN_ACYCLIC, 0.1, 0.1)
    assert e.value.code == T.TN_ERR_CYCLIC
