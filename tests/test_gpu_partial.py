"""GPU partial TNC (Corollary 1, tn_partial_plan) against the oracle.

Entry r of the output is Eq. (1) on the full TNC of the sub-tensors that fix
the free modes at r's index (tests/test_oracle_partial.py builds that
sub-network and pins it against Def. 1).  All entries of a sample share the
network's count sketches (seed, stream e for contraction e), so entry r's
sample s must equal the oracle's Method-1 estimate of entry r's sub-network
at (seed, s), within tau * A_hat as in test_gpu_m1.  Also: injected
collision-free hashes make every entry exact; over many samples every entry's
mean is within 5 standard errors of Def. 1's value, and the summed variance
respects the corollary's 3^t/m prod ||X_k||^2; the permutation of a tensor
whose free modes trail runs inside a replayed graph after an in-place data
change."""
import numpy as np
import pytest

import tn_workloads as W
from test_gpu_m1 import TAU, dev, host_view
from test_oracle_partial import entry_network, free_modes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    return T


def make(T, net, dtype, m, S, seed, flags=0):
    ts = dev(net, dtype)
    spec = T.NetworkSpec.from_network(net, ts)
    return T.PartialPlan(spec, m, S, seed, flags=flags), net.with_data(host_view(ts)), ts


def run(plan):
    import torch
    samples = torch.empty(plan.n_nets * plan.S, dtype=torch.float64, device="cuda")
    stats = plan.estimate(samples_out=samples)
    torch.cuda.synchronize()
    return stats.cpu().numpy().reshape(-1, 2), samples.cpu().numpy().reshape(plan.n_nets, plan.S)


def check(orc, net, got, m, seed, dtype, entries, samples):
    for r in entries:
        sub = entry_network(net, r)
        for s in samples:
            o = orc.m1_estimate(sub, m, seed, s, combine="conv" if m <= 2048 else "dft", want_scale=True)
            assert abs(got[r, s] - o["estimate"]) <= TAU[dtype] * o["scale"] + 1e-300, (r, s)


@pytest.mark.parametrize("dtype", ["float64", "float32", "bfloat16"])
def test_example1_per_sample(T, orc, dtype):
    """Example 1: free mode 2 leads tensor 2, free mode 8 trails tensor 4 (its
    sub-tensors need the permuted copy)."""
    net = W.example1(dtype=np.float64, dist="normal")
    plan, view, _ = make(T, net, dtype, 64, 6, 17)
    assert plan.n_nets == net.dims[1] * net.dims[7] and plan.query(13) == 2
    assert plan.out_shape == (net.dims[1], net.dims[7])
    st, got = run(plan)
    check(orc, view, got, 64, 17, dtype, range(plan.n_nets), range(6))
    assert np.allclose(st[:, 0], got.mean(axis=1), rtol=1e-12, atol=1e-12 * np.abs(got).max())


def test_cut_torus_sampled_entries(T, orc):
    """A 3 x 3 torus (bond 8, FP32) with two contractions cut: four free modes
    of size 8 on four tensors (4096 entries), m = 1024; sampled entries."""
    base = W.torus(L=3, D=8, seed=6, dist="normal")
    cut = base.edges[:2]
    net = W.Network(base.orders, base.dims, base.edges[2:], base.data)
    assert len(free_modes(net)) == 4 and len(cut) == 2
    plan, view, _ = make(T, net, "float32", 1024, 3, 5)
    assert plan.n_nets == 4096
    st, got = run(plan)
    check(orc, view, got, 1024, 5, "float32", [0, 1, 777, 2048, 4095], range(3))


def test_injective_hashes_exact(T, orc):
    """Collision-free tables (bucket i * B^e, B = 2n, m >= B^t) and signs +1:
    every entry's estimate is its exact value, Def. 1 read literally."""
    import torch
    net = W.example1(n=(3, 2, 3, 3, 3, 3, 3, 2), dtype=np.float64, dist="normal")
    B, m = 6, 256
    plan, view, _ = make(T, net, "float64", m, 2, 0)
    W_ = plan.query(0)
    tab = np.zeros((2, W_), dtype=np.int32)
    for (j, sid, nn, off) in plan.streams():
        tab[:, off:off + nn] = (np.arange(nn) * B ** sid) % m
    plan.set_hashes(torch.from_numpy(tab).cuda())
    _, got = run(plan)
    lit = orc.tc_literal(view).reshape(-1)
    assert np.allclose(got, lit[:, None], rtol=1e-12, atol=1e-12 * np.abs(lit).max())


def test_unbiased_entries_and_summed_variance(T, orc):
    """Every entry's mean over S = 20000 samples lies within 5 standard errors
    of Def. 1's value; the summed per-entry variance is below the bound of the
    corollary's proof, 3^t/m prod_k ||X_k||_F^2."""
    net = W.example1(n=(4, 3, 5, 5, 4, 6, 6, 2), dtype=np.float64, dist="normal")
    S, m = 20000, 32
    plan, view, _ = make(T, net, "float64", m, S, 3)
    st, got = run(plan)
    lit = orc.tc_literal(view).reshape(-1)
    se = np.sqrt(st[:, 1] / S)
    assert np.all(np.abs(st[:, 0] - lit) <= 5 * se + 1e-12)
    assert st[:, 1].sum() <= 3.0 ** net.t / m * view.input_norm() ** 2


def test_graph_replay_after_data_change(T, orc):
    """With TN_FLAG_GRAPH the permutation runs inside the captured graph:
    after the tensors are scaled in place, each replay matches an eager plan
    on the new data."""
    import torch
    net = W.example1(dtype=np.float64, dist="normal")
    plan, view, ts = make(T, net, "float32", 128, 4, 9, flags=T.TN_FLAG_GRAPH)
    eager, _, ts2 = make(T, net, "float32", 128, 4, 9)
    for f in (1.0, 0.5, 3.0):
        for a, b in zip(ts, ts2):
            a.mul_(f)
            b.mul_(f)
        _, g = run(plan)
        torch.ones(1000, device="cuda").sum().item()
        _, ge = run(eager)
        assert np.array_equal(g, ge)


def test_rejects_outer_factors_and_two_pass(T):
    import torch
    net = W.Network([2, 1], [3, 4, 3], [(0, 2)], [np.ones((3, 4)), np.ones(3)])
    spec = T.NetworkSpec.from_network(net, [torch.ones(3, 4, dtype=torch.float64, device="cuda"),
                                            torch.ones(3, dtype=torch.float64, device="cuda")])
    with pytest.raises(T.TNError) as e:
        T.PartialPlan(spec, 32768, 2, 0)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
    outer = W.Network([1, 1, 1], [3, 3, 2], [(0, 1)], [np.ones(3), np.ones(3), np.ones(2)])
    spec = T.NetworkSpec.from_network(outer, [torch.ones(3, dtype=torch.float64, device="cuda"),
                                              torch.ones(3, dtype=torch.float64, device="cuda"),
                                              torch.ones(2, dtype=torch.float64, device="cuda")])
    with pytest.raises(T.TNError) as e:
        T.PartialPlan(spec, 64, 2, 0)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
