"""The acyclic estimator with TN_FLAG_MFMA_F32 (SMVP products on the FP32
matrix cores, FP32 accumulation), checked per tree level against the exact
FP64 oracle.

For FP32 and BF16 data both operands of w_k = mat(X_k) G are exact in FP32 (the
data, and g, which the FP64-product path also stores in FP32), so the only new
error is the FP32 accumulation: a block sums its column range of K columns in
K / 4 matrix instructions, each rounding its running sum at 2^-24, and the
column ranges meet in FP64.  Rounding errors of random sign in a running sum
of terms of random sign give about 2^-24 sqrt(K) relative to the result; the
stored w and g add 2^-24 each.  Bar per tensor l with d_l product levels in its
subtree, K the widest contraction of the network:
  ||x_l - x_l^exact|| <= 2^-24 (8 + 2 sqrt(K)) (1 + d_l) ||x_l^exact||,
levels added linearly (a generous bound: they are uncorrelated).  Each estimate
is within bar(L) ||x_o|| ||r_o|| (Cauchy-Schwarz at the root).  That the
products really are FP32 ones shows at depth 1 of the caterpillar (K = 4096):
the error there is several times that of the FP64 products on the same inputs.
"""
import numpy as np
import pytest

import tn_workloads as W

from test_gpu_m2_bf16 import subtree_levels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    return T


def widest(net, root=0):
    """The largest number of columns K of any product mat(X_k) G: the product
    of the child-mode sizes of a tensor with children."""
    owner = np.repeat(np.arange(net.p), net.orders)
    adj = [[] for _ in range(net.p)]
    for (u, v) in net.edges:
        adj[owner[u]].append((owner[v], v))
        adj[owner[v]].append((owner[u], u))
    parent, order = {root: -1}, [root]
    for a in order:
        for b, _ in adj[a]:
            if b not in parent:
                parent[b] = a
                order.append(b)
    k_max = 1
    for a in range(net.p):
        kids = [net.dims[mode] for b, mode in adj[a] if parent.get(b) == a]
        if kids:
            k_max = max(k_max, int(np.prod(kids)))
    return k_max


def bar(d, K):
    return 2.0 ** -24 * (8.0 + 2.0 * np.sqrt(K)) * (1.0 + d)


CASES = {
    "example5": lambda: (W.example5(n=4, seed=3), 128, 6),
    "chain": lambda: (W.chain([5, 6, 7, 40, 33], seed=4), 256, 6),
    "caterpillar8": lambda: (W.tt_caterpillar(cores=8, bond=32, phys=16, seed=2), 1024, 4),
    "caterpillar32": lambda: (W.tt_caterpillar(), 4096, 3),
}


def run(T, net, dtype, m, S, seed, flags):
    import torch
    td = getattr(torch, dtype)
    ts = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda().to(td).contiguous() for x in net.data]
    view = net.with_data([t.double().cpu().numpy() for t in ts])
    spec = T.NetworkSpec.from_network(net, ts)
    plan = T.Plan([spec], T.TN_ACYCLIC, m, S, seed, root=0, flags=flags)
    smp = torch.empty(S, dtype=torch.float64, device="cuda")
    plan.estimate(samples_out=smp)
    sk = plan.sketches(0, S).cpu().numpy()
    return view, smp.cpu().numpy(), sk


@pytest.mark.parametrize("case", list(CASES))
def test_f32_products_per_level(T, orc, case):
    net, m, S = CASES[case]()
    view, got, sk = run(T, net, "float32", m, S, 9, T.TN_FLAG_MFMA_F32)
    _, got64, sk64 = run(T, net, "float32", m, S, 9, 0)
    d = subtree_levels(net)
    K = widest(net)
    L = max(d.values())
    worst = {"d1_f32": 0.0, "d1_f64": 0.0, "over_bar": 0.0, "estimate_over_bar": 0.0}
    for r in range(S):
        ex = orc.m2_estimate(view, m, 9, r, want_trace=True)
        for l in range(1, net.p):
            if d[l] == 0:
                continue
            nx = np.linalg.norm(ex["x"][l])
            e = np.linalg.norm(sk[r, l] - ex["x"][l]) / nx
            assert e <= bar(d[l], K), (case, r, l, d[l], e)
            worst["over_bar"] = max(worst["over_bar"], e / bar(d[l], K))
            if d[l] == 1:
                worst["d1_f32"] = max(worst["d1_f32"], e)
                worst["d1_f64"] = max(worst["d1_f64"], np.linalg.norm(sk64[r, l] - ex["x"][l]) / nx)
        scale = np.linalg.norm(ex["x"][0]) * np.linalg.norm(ex["r_root"])
        e_y = abs(got[r] - ex["estimate"]) / scale
        assert e_y <= bar(L, K), (case, r, e_y)
        worst["estimate_over_bar"] = max(worst["estimate_over_bar"], e_y / bar(L, K))
    print(case, "K", K, {k: f"{v:.3e}" for k, v in worst.items()})
    if K >= 4096:
        assert worst["d1_f32"] > 4.0 * worst["d1_f64"]


def test_f32_products_bf16_data(T, orc):
    """BF16 data: X is exact in FP32; the same bars against the exact oracle."""
    net = W.tt_caterpillar(cores=6, bond=16, phys=8, seed=7)
    view, got, sk = run(T, net, "bfloat16", 512, 4, 3, T.TN_FLAG_MFMA_F32)
    d = subtree_levels(net)
    K, L = widest(net), max(d.values())
    for r in range(4):
        o = orc.m2_estimate(view, 512, 3, r, root=0, want_trace=True)
        scale = np.linalg.norm(o["x"][0]) * np.linalg.norm(o["r_root"])
        assert abs(got[r] - o["estimate"]) <= bar(L, K) * scale
        for l in range(1, net.p):
            if d[l]:
                assert np.linalg.norm(sk[r, l] - o["x"][l]) <= bar(d[l], K) * np.linalg.norm(o["x"][l])


def test_f32_products_bench_shape(T, orc):
    """The caterpillar at the benchmark's launch shape (m = 4096, S = 4096,
    FP32 products): sampled estimates against the oracle within the bar."""
    import torch
    net = W.tt_caterpillar(seed=3)
    S, m = 4096, 4096
    view, got, _ = run(T, net, "float32", m, S, 0, T.TN_FLAG_MFMA_F32)
    K, L = widest(net), max(subtree_levels(net).values())
    for r in (0, 1, 2047, 4095):
        o = orc.m2_estimate(view, m, 0, r, root=0, want_trace=True)
        scale = np.linalg.norm(o["x"][0]) * np.linalg.norm(o["r_root"])
        assert abs(got[r] - o["estimate"]) <= bar(L, K) * scale, r
    torch.cuda.synchronize()


def test_f32_flag_rejections(T):
    import torch
    tri = W.triangle(8, seed=1, dtype=np.float32)
    spec = T.NetworkSpec.from_network(tri, [torch.from_numpy(x).cuda() for x in tri.data])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec], T.TN_CYCLIC, 64, 4, 1, flags=T.TN_FLAG_MFMA_F32)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
    net = W.tt_caterpillar(cores=4, bond=8, phys=4, seed=1)
    ts = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda() for x in net.data]
    spec64 = T.NetworkSpec.from_network(net, ts)
    with pytest.raises(T.TNError) as e:
        T.Plan([spec64], T.TN_ACYCLIC, 64, 4, 1, flags=T.TN_FLAG_MFMA_F32)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
    spec32 = T.NetworkSpec.from_network(net, [t.float() for t in ts])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec32], T.TN_ACYCLIC, 64, 4, 1, flags=T.TN_FLAG_MFMA_F32 | T.TN_FLAG_MFMA_BF16)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
