"""The acyclic estimator with TN_FLAG_MFMA_BF16 (SMVP products on the BF16
matrix cores, FP32 accumulation) against the exact FP64 oracle.

The hashes and combines are those of the FP64 path; the products
w_k = mat(X_k) G round their operands to BF16 (unit roundoff 2^-9), and the
sketch scatters that produce G accumulate in 32-bit fixed point (each term
rounded to 2^-(31 - lgN) of the largest product, far below the BF16 rounding
of G that follows).
To first order each tree level perturbs the vectors passed upwards by at most
about 2 * 2^-9 relative per operand pair, and the perturbations of L levels
add, so the bar for each estimate is
    |y_bf16 - y| <= L * 2^-7 * ||x_o||_2 ||r_o||_2
(the Cauchy-Schwarz scale of y = x_o^T r_o, as for the FP32 bar), with L the
number of tree levels that run a product.  The tests print the measured errors.
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


@pytest.mark.parametrize("case", ["example5", "chain", "caterpillar8", "caterpillar32"])
def test_bf16_products_error_bound(T, orc, case):
    if case == "example5":
        net, m, S, idx = W.example5(n=4, seed=3), 128, 8, range(8)
    elif case == "chain":
        net, m, S, idx = W.chain([5, 6, 7, 40, 33], seed=4), 256, 8, range(8)
    elif case == "caterpillar8":
        net, m, S, idx = W.tt_caterpillar(cores=8, bond=32, phys=16, seed=2), 1024, 6, range(6)
    else:
        net, m, S, idx = W.tt_caterpillar(), 4096, 16, [0, 7, 15]
    view, got = run_bf16(T, net, "float32", m, S, 9)
    L = max(1, levels(net))
    errs = []
    for r in idx:
        o = orc.m2_estimate(view, m, 9, r, root=0, want_trace=True)
        scale = np.linalg.norm(o["x"][0]) * np.linalg.norm(o["r_root"])
        errs.append(abs(got[r] - o["estimate"]) / scale)
    errs = np.array(errs)
    print(f"{case}: levels {L}, error / (|x_o| |r_o|): max {errs.max():.3e} median {np.median(errs):.3e}")
    assert np.all(errs <= L * 2.0 ** -7)
    # and the rounding is visible: BF16 products are not the FP64 ones
    assert errs.max() > 1e-6


def test_bf16_bf16_data(T, orc):
    """BF16 input data: X is exact in BF16 already, only G is rounded."""
    net = W.tt_caterpillar(cores=6, bond=16, phys=8, seed=7)
    view, got = run_bf16(T, net, "bfloat16", 512, 4, 3)
    L = levels(net)
    for r in range(4):
        o = orc.m2_estimate(view, 512, 3, r, root=0, want_trace=True)
        scale = np.linalg.norm(o["x"][0]) * np.linalg.norm(o["r_root"])
        assert abs(got[r] - o["estimate"]) <= L * 2.0 ** -7 * scale


def test_bf16_flag_rejected_for_cyclic(T):
    import torch
    net = W.triangle(8, seed=1, dtype=np.float32)
    spec = T.NetworkSpec.from_network(net, [torch.from_numpy(x).cuda() for x in net.data])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec], T.TN_CYCLIC, 64, 4, 1, flags=T.TN_FLAG_MFMA_BF16)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
