"""GPU parity of the persistent fused cyclic kernel (TN_FLAG_PERSISTENT) against
the FP64 oracle, with the bars of test_gpu_m1: each per-sample estimate within
tau * A_hat (the first-order rounding scale of the FFT route), tau = 1e-5 for
FP32/BF16 data and 1e-12 for FP64."""
import numpy as np
import pytest

import tn_workloads as W
from test_gpu_m1 import TAU, make_plan, oracle_samples, run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    return T


def check(T, orc, nets, dtype, m, S, seed, idx=None):
    plan, views = make_plan(T, nets, dtype, m, S, seed, flags=T.TN_FLAG_PERSISTENT)
    stats, got = run(plan)
    tau = TAU[dtype]
    for j, net in enumerate(views):
        ii = list(range(S)) if idx is None else idx
        ref, scale = oracle_samples(orc, net, m, seed + j, ii)
        err = np.abs(got[j, ii] - ref)
        assert np.all(err <= tau * scale + 1e-300), (j, err.max(), (err / scale).max())
        assert stats[j, 0] == pytest.approx(got[j].mean(), rel=1e-12, abs=1e-12 * abs(scale).max())
    return plan, got


@pytest.mark.parametrize("dtype", ["float64", "float32", "bfloat16"])
def test_uneven_batch(T, orc, dtype):
    """Random cyclic networks of 3-12 tensors with ragged sample batches (S = 7)."""
    nets = W.random_batch(count=10, seed=4, bmax=12)
    check(T, orc, nets, dtype, 256, 7, 31)


def test_triangle_and_odd_tensor_counts(T, orc):
    """Three tensors (one unpaired in the last step), a trace (one tensor), and a
    ring of five, in one plan, m = 64 and 1024."""
    trace = W.Network([2], [9, 9], [(0, 1)], [np.random.default_rng(3).standard_normal((9, 9))])
    for m in (64, 1024):
        check(T, orc, [W.triangle(16, seed=2), trace, W.ring(5, 12, seed=4)], "float64", m, 5, 77)


def test_multi_slot_tensors(T, orc):
    """A tensor cut into several slots (50 x 40 x 60 with 2400-entry rows) feeds one
    sketch across slots, and a 4x4 torus (order-4 tensors, bond 16)."""
    big = W.Network([3, 3], [50, 40, 60, 60, 40, 50], [(0, 5), (1, 4), (2, 3)],
                    [np.random.default_rng(5).standard_normal((50, 40, 60)),
                     np.random.default_rng(6).standard_normal((60, 40, 50))])
    check(T, orc, [big], "float32", 512, 4, 5)
    check(T, orc, [W.torus()], "float32", 1024, 3, 5, idx=[0, 2])


def test_m4096_and_single_sample(T, orc):
    check(T, orc, [W.triangle(32, seed=9), W.random_network(4, 17)], "float32", 4096, 1, 2)


def test_matches_two_kernel_path_statistics(T, orc):
    """The persistent and the slot/combine paths compute the same estimator from
    the same hashes: per-sample estimates agree to rounding (both within the
    oracle bar above), and the means over 64 samples agree accordingly."""
    nets = W.random_batch(count=6, seed=4, bmax=10)
    pa, va = make_plan(T, nets, "float64", 128, 64, 3, flags=T.TN_FLAG_PERSISTENT)
    pb, _ = make_plan(T, nets, "float64", 128, 64, 3)
    sa, ga = run(pa)
    sb, gb = run(pb)
    scale = np.abs(ga).max() + np.abs(gb).max()
    assert np.all(np.abs(ga - gb) <= 1e-11 * scale)


def test_graph_replay(T, orc):
    """Captured persistent launches (queue reset by a kernel, not a memset) replay
    correctly several times with eager work in between."""
    import torch
    nets = W.random_batch(count=5, seed=4, bmax=8)
    plan, views = make_plan(T, nets, "float32", 256, 6, 8,
                            flags=T.TN_FLAG_PERSISTENT | T.TN_FLAG_GRAPH)
    eager, _ = make_plan(T, nets, "float32", 256, 6, 8, flags=T.TN_FLAG_PERSISTENT)
    ref, gref = run(eager)
    for _ in range(3):
        _, g = run(plan)
        torch.ones(1000, device="cuda").sum().item()
        assert np.array_equal(g, gref)


def test_rejects_acyclic_and_large_m(T):
    import torch
    net = W.example5(n=3, seed=1)
    spec = T.NetworkSpec.from_network(net, [torch.from_numpy(x).cuda() for x in net.data])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec], T.TN_ACYCLIC, 64, 4, 1, flags=T.TN_FLAG_PERSISTENT)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
    tri = W.triangle(8, seed=1)
    spec = T.NetworkSpec.from_network(tri, [torch.from_numpy(x).cuda() for x in tri.data])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec], T.TN_CYCLIC, 16384, 4, 1, flags=T.TN_FLAG_PERSISTENT)
    assert e.value.code == T.TN_ERR_UNSUPPORTED


def test_batched_bench_shape_persistent(T, orc):
    """The benchmark's batch in one persistent launch: all 4096 random cyclic
    networks (1.16 GB of FP32) with TN_FLAG_PERSISTENT | TN_FLAG_AUTOTUNE, m =
    1024, S = 16 (many work items, largest-first order, the sample chunking of
    the fused kernel); sampled networks and samples against the oracle, and the
    plan's statistics against its samples."""
    import torch
    nets = W.random_batch(count=4096, seed=4)
    specs, views = [], []
    for n in nets:
        ts = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float32) for x in n.data]
        specs.append(T.NetworkSpec.from_network(n, ts))
        views.append((n, ts))
    plan = T.Plan(specs, T.TN_CYCLIC, 1024, 16, 0, flags=T.TN_FLAG_PERSISTENT | T.TN_FLAG_AUTOTUNE)
    stats, got = run(plan)
    assert plan.query(11) == 1
    rng = np.random.default_rng(2)
    for j in sorted({0, 1, 2047, 4095, *rng.integers(0, 4096, 6).tolist()}):
        n, ts = views[j]
        v = n.with_data([t.double().cpu().numpy() for t in ts])
        ii = [0, 5, 15]
        ref, scale = oracle_samples(orc, v, 1024, 0 + j, ii)
        assert np.all(np.abs(got[j, ii] - ref) <= TAU["float32"] * scale), j
    assert np.all(np.isfinite(got))
    assert np.allclose(stats[:, 0], got.mean(axis=1), rtol=1e-12, atol=0)
