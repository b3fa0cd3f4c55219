"""The acyclic estimator with TN_FLAG_MFMA_BF16 (SMVP products on the BF16
matrix cores, FP32 accumulation), checked per tree level.

The hashes and combines are those of the FP64 path; the products
w_k = mat(X_k) G round both operands to BF16 (ties to even, via FP32) and
accumulate in FP32, and the root's x_o^T r_o does the same.  Two bars:

* Against the oracle's BF16-product variant (the same operand rounding, FP64
  sums): at depth 1 (a tensor whose children are leaves, one product) the only
  differences are the FP32 accumulation and a rare operand rounding that flips
  because the GPU's 32-bit fixed-point sketch differs from the oracle's FP64
  one, so ||x_l - x_l^bf16|| <= 6e-4 ||x_l||: 7-20x below the 4e-3 that the
  BF16 rounding itself moves x_l (measured: at most 1.7e-4).  A truncating
  rounding, an unrounded operand or a wrong operand fails it.  Deeper, the
  flips feed into the next level's roundings and the two drift apart at
  BF16's own rate, so deeper levels are checked against exact arithmetic.
* Against the exact FP64 oracle, per tensor l with d_l product levels in its
  subtree: ||x_l - x_l^exact|| <= 2^-8 (2 + d_l / 2) ||x_l^exact||.  Each level
  rounds two operands by at most 2^-9 relative each (2^-8 per product); the
  rounding errors of a level are uncorrelated, so levels add far more slowly
  than d 2^-8, and the constant covers one level's cancellation in its sums.
  Measured on these networks: 2.3e-3 .. 4.2e-3 at d = 1, 8.1e-3 at d = 4, 2.4e-2
  at d = 31 against bars of 9.8e-3, 1.6e-2 and 6.8e-2; a dropped level (error
  ~1) or a rounding biased by 2^-9 per operand (~d 2^-8 = 0.12 at d = 31) fails.
* Each estimate: |y - y_exact| <= 2^-8 (2 + L / 2) ||x_o|| ||r_o|| with L the
  product levels, the per-level bar carried to y = x_o^T r_o by Cauchy-Schwarz
  (loose by nature: the errors of x_o and r_o are not aligned with them).
"""
import numpy as np
import pytest

import tn_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    return T


def levels(net, root=0):
    """Number of depths at which some tensor has children (products run)."""
    owner = np.repeat(np.arange(net.p), net.orders)
    adj = [[] for _ in range(net.p)]
    for (u, v) in net.edges:
        adj[owner[u]].append(owner[v])
        adj[owner[v]].append(owner[u])
    depth = {root: 0}
    order = [root]
    for a in order:
        for b in adj[a]:
            if b not in depth:
                depth[b] = depth[a] + 1
                order.append(b)
    return len({depth[k] for k in range(net.p) if any(depth.get(b, -1) == depth[k] + 1 for b in adj[k])})


def run_bf16(T, net, dtype, m, S, seed):
    import torch
    td = getattr(torch, dtype)
    ts = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda().to(td).contiguous()
          for x in net.data]
    view = net.with_data([t.double().cpu().numpy() for t in ts])
    spec = T.NetworkSpec.from_network(net, ts)
    plan = T.Plan([spec], T.TN_ACYCLIC, m, S, seed, root=0, flags=T.TN_FLAG_MFMA_BF16)
    samples = torch.empty(S, dtype=torch.float64, device="cuda")
    plan.estimate(samples_out=samples)
    torch.cuda.synchronize()
    return view, samples.cpu().numpy()


def subtree_levels(net, root=0):
    """Per tensor: the number of product levels in its subtree (1 for a tensor
    whose children are all leaves, 0 for a leaf)."""
    owner = np.repeat(np.arange(net.p), net.orders)
    adj = [[] for _ in range(net.p)]
    for (u, v) in net.edges:
        adj[owner[u]].append(owner[v])
        adj[owner[v]].append(owner[u])
    parent, order = {root: -1}, [root]
    for a in order:
        for b in adj[a]:
            if b not in parent:
                parent[b] = a
                order.append(b)
    kids = {k: [b for b in adj[k] if parent.get(b) == k] for k in range(net.p)}
    d = {}
    for k in reversed(order):
        d[k] = (1 + max(d[c] for c in kids[k])) if kids[k] else 0
    return d


def bar(d):
    return 2.0 ** -8 * (2.0 + d / 2.0)


CASES = {
    "example5": lambda: (W.example5(n=4, seed=3), 128, 6),
    "example5_16": lambda: (W.example5(n=16, seed=5), 512, 4),
    "chain": lambda: (W.chain([5, 6, 7, 40, 33], seed=4), 256, 6),
    "caterpillar8": lambda: (W.tt_caterpillar(cores=8, bond=32, phys=16, seed=2), 1024, 4),
    "caterpillar32": lambda: (W.tt_caterpillar(), 4096, 3),
}


@pytest.mark.parametrize("case", list(CASES))
def test_bf16_products_per_level(T, orc, case):
    import torch
    net, m, S = CASES[case]()
    ts = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda().float() for x in net.data]
    view = net.with_data([t.double().cpu().numpy() for t in ts])
    spec = T.NetworkSpec.from_network(net, ts)
    plan = T.Plan([spec], T.TN_ACYCLIC, m, S, 9, root=0, flags=T.TN_FLAG_MFMA_BF16)
    smp = torch.empty(S, dtype=torch.float64, device="cuda")
    plan.estimate(samples_out=smp)
    sk = plan.sketches(0, S).cpu().numpy()
    got = smp.cpu().numpy()
    d = subtree_levels(net)
    L = max(d.values())
    worst = {"d1_bf16": 0.0, "d1_exact": 0.0, "deep_exact_over_bar": 0.0, "estimate": 0.0}
    for r in range(S):
        ex = orc.m2_estimate(view, m, 9, r, want_trace=True)
        bf = orc.m2_estimate(view, m, 9, r, want_trace=True, bf16_products=True)
        for l in range(1, net.p):
            if d[l] == 0:
                continue
            nx = np.linalg.norm(ex["x"][l])
            e_ex = np.linalg.norm(sk[r, l] - ex["x"][l]) / nx
            assert e_ex <= bar(d[l]), (case, r, l, d[l], e_ex)
            worst["deep_exact_over_bar"] = max(worst["deep_exact_over_bar"], e_ex / bar(d[l]))
            if d[l] == 1:
                e_bf = np.linalg.norm(sk[r, l] - bf["x"][l]) / nx
                assert e_bf <= 6e-4, (case, r, l, e_bf)
                worst["d1_bf16"] = max(worst["d1_bf16"], e_bf)
                worst["d1_exact"] = max(worst["d1_exact"], e_ex)
        scale = np.linalg.norm(ex["x"][0]) * np.linalg.norm(ex["r_root"])
        e_y = abs(got[r] - ex["estimate"]) / scale
        assert e_y <= bar(L), (case, r, e_y)
        worst["estimate"] = max(worst["estimate"], e_y)
    print(case, {k: f"{v:.3e}" for k, v in worst.items()})
    # the products really are BF16 ones: depth-1 sketches move by the BF16 rounding
    assert worst["d1_exact"] > 1e-3


def test_bf16_bf16_data(T, orc):
    """BF16 input data: X is exact in BF16 already, only G is rounded; the
    estimate is within the per-level bar carried to y, and at depth 1 the
    sketches match the BF16-product oracle."""
    net = W.tt_caterpillar(cores=6, bond=16, phys=8, seed=7)
    view, got = run_bf16(T, net, "bfloat16", 512, 4, 3)
    L = levels(net)
    for r in range(4):
        o = orc.m2_estimate(view, 512, 3, r, root=0, want_trace=True)
        b = orc.m2_estimate(view, 512, 3, r, root=0, bf16_products=True)
        scale = np.linalg.norm(o["x"][0]) * np.linalg.norm(o["r_root"])
        assert abs(got[r] - o["estimate"]) <= bar(L) * scale
        assert abs(got[r] - b["estimate"]) <= bar(L) * scale


def test_bf16_flag_rejected_for_cyclic(T):
    import torch
    net = W.triangle(8, seed=1, dtype=np.float32)
    spec = T.NetworkSpec.from_network(net, [torch.from_numpy(x).cuda() for x in net.data])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec], T.TN_CYCLIC, 64, 4, 1, flags=T.TN_FLAG_MFMA_BF16)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
