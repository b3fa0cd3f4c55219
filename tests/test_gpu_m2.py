"""GPU parity of the acyclic-network estimator (Eq. (2), Algorithms 2-5) against
the FP64 oracle.

Bars: hash tables bit-exact; every tensor's sketch x_l (and r_o for the root)
within tau * ||x_l||_2 of the oracle's in 2-norm; each estimate within
tau * ||x_o||_2 ||r_o||_2 (the Cauchy-Schwarz scale of the root inner product
y = x_o^T r_o).  tau = 1e-5 for FP32/BF16 data, 1e-12 for FP64.  (The
|X|-and-unit-sign propagation used for the cyclic method is no bound worth
testing here: over tens of tree levels it exceeds the estimate by many orders
of magnitude.)
"""
import math

import numpy as np
import pytest

import tn_workloads as W

pytestmark = pytest.mark.gpu

TAU = {"float64": 1e-12, "float32": 1e-5, "bfloat16": 1e-5}


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    return T


def dev(net, dtype):
    import torch
    td = getattr(torch, dtype)
    return [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda").to(td).contiguous()
            for x in net.data]


def make_plan(T, nets, dtype, m, S, seed, root=0, flags=0):
    specs, views = [], []
    for n in nets:
        ts = dev(n, dtype)
        specs.append(T.NetworkSpec.from_network(n, ts))
        views.append(n.with_data([t.double().cpu().numpy() for t in ts]))
    return T.Plan(specs, T.TN_ACYCLIC, m, S, seed, root=root, flags=flags), views


def run(plan):
    import torch
    samples = torch.empty(plan.n_nets * plan.S, dtype=torch.float64, device="cuda")
    stats = plan.estimate(samples_out=samples)
    torch.cuda.synchronize()
    return stats.cpu().numpy().reshape(-1, 2), samples.cpu().numpy().reshape(plan.n_nets, plan.S)


def check(orc, plan, views, seed, dtype, root=0, samples=None):
    stats, got = run(plan)
    tau = TAU[dtype]
    idx = list(range(plan.S)) if samples is None else samples
    for j, net in enumerate(views):
        for r in idx:
            o = orc.m2_estimate(net, plan.m, seed + j, r, root=root, want_trace=True)
            scale = np.linalg.norm(o["x"][root]) * np.linalg.norm(o["r_root"])
            assert abs(got[j, r] - o["estimate"]) <= tau * scale + 1e-300, (j, r, got[j, r], o["estimate"])
        mu = got[j].mean()
        assert stats[j, 0] == pytest.approx(mu, rel=1e-12, abs=1e-300)
    return got


def test_hashes_bit_exact(T, orc):
    nets = [W.example5(n=3), W.tt_caterpillar(cores=4, bond=5, phys=3, seed=1, dtype=np.float64)]
    plan, views = make_plan(T, nets, "float64", 64, 3, 55)
    tab = plan.hashes().cpu().numpy()
    want = set()
    for j, net in enumerate(views):
        want |= {(j, sid) for sid, _ in orc.m2_streams(net, 0)}
    got = set()
    for (j, sid, n, off) in plan.streams():
        got.add((j, sid))
        for r in range(3):
            h, s = orc.hash_table(55 + j, r, sid, n, 64)
            v = tab[r, off:off + n]
            assert np.array_equal(v & 0x7FFFFFFF, h)
            assert np.array_equal(np.where(v < 0, -1, 1), s)
    assert got == want


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_sketch_vectors(T, orc, dtype):
    """x_l = C_{k,l} mat(X_l) R_l^T r_l for every non-root tensor, r_o at the root."""
    nets = [W.example5(n=4, seed=3), W.chain([5, 6, 7, 4], seed=4)]
    m = 128
    plan, views = make_plan(T, nets, dtype, m, 4, 7)
    sk = plan.sketches(first=1, count=3).cpu().numpy()
    k0 = 0
    for j, net in enumerate(views):
        for r in range(1, 4):
            o = orc.m2_estimate(net, m, 7 + j, r, root=0, want_trace=True)
            for k in range(net.p):
                ref = o["r_root"] if k == 0 else o["x"][k]
                err = np.linalg.norm(sk[r - 1, k0 + k] - ref)
                assert err <= TAU[dtype] * np.linalg.norm(ref) + 1e-300, (j, r, k, err)
        k0 += net.p


@pytest.mark.parametrize("dtype", ["float64", "float32", "bfloat16"])
def test_example5_and_chains(T, orc, dtype):
    nets = [W.example5(n=5, seed=1), W.chain([8, 3, 9, 5, 6], seed=2),
            W.tt_caterpillar(cores=6, bond=7, phys=5, seed=3, dtype=np.float64)]
    plan, views = make_plan(T, nets, dtype, 256, 9, 3)
    check(orc, plan, views, 3, dtype)


@pytest.mark.parametrize("root", [1, 3, 6])
def test_other_roots(T, orc, root):
    net = W.example5(n=4, seed=5)
    plan, views = make_plan(T, [net], "float64", 64, 5, 11, root=root)
    check(orc, plan, views, 11, "float64", root=root)


def test_padding_three_and_five_children(T, orc):
    """Padding of the recursive sketch to the next power of two (3 -> 4, 5 -> 8)."""
    rng = np.random.default_rng(7)
    star3 = W.Network([3, 1, 1, 1], [4, 5, 6, 4, 5, 6], [(0, 3), (1, 4), (2, 5)],
                      [rng.standard_normal((4, 5, 6)), rng.standard_normal(4), rng.standard_normal(5),
                       rng.standard_normal(6)])
    dims5 = [3, 4, 2, 5, 3]
    star5 = W.Network([5] + [1] * 5, dims5 + dims5, [(i, 5 + i) for i in range(5)],
                      [rng.standard_normal(dims5)] + [rng.standard_normal(d) for d in dims5])
    plan, views = make_plan(T, [star3, star5], "float64", 512, 6, 21)
    check(orc, plan, views, 21, "float64")


@pytest.mark.parametrize("bond", [100, 300])
def test_two_child_gather_paths(T, orc, bond):
    """Tensors with two children take the register-held second child when its
    dimension is at most 256 (bond 100: 2 index rows per pass, 56 idle threads)
    and the general mixed-radix walk otherwise (bond 300)."""
    net = W.tt_caterpillar(cores=3, bond=bond, phys=3, seed=4, dtype=np.float64)
    for dtype in ("float64", "float32"):
        plan, views = make_plan(T, [net], dtype, 512, 4, 17)
        check(orc, plan, views, 17, dtype)


def test_caterpillar_full_size(T, orc):
    """Tensor-train cores (1,64,64), (64,64,64) x 30, (64,64,1) with their physical
    legs contracted against vectors, N(0, 1/64), m = 4096; sampled seeds."""
    net = W.tt_caterpillar()
    plan, views = make_plan(T, [net], "float32", 4096, 16, 0)
    check(orc, plan, views, 0, "float32", samples=[0, 5, 15])


@pytest.mark.parametrize("flags", ["fp64", "bf16"])
def test_caterpillar_bench_schedule(T, orc, flags):
    """The caterpillar at the benchmark's size and launch shape: S = 4096 samples
    in one plan (column-split products, the gathers summing the partials, four
    samples per gather block, the two-child gather kernel); sampled estimates,
    including the last sample of a block and of the plan, against the oracle
    (FP32 bar, or with BF16 products the per-level bars of test_gpu_m2_bf16:
    every sketch against exact arithmetic, depth-1 sketches against the
    BF16-product oracle)."""
    net = W.tt_caterpillar()
    if flags == "fp64":
        plan, views = make_plan(T, [net], "float32", 4096, 4096, 0)
        check(orc, plan, views, 0, "float32", samples=[0, 3, 2047, 4095])
        return
    import torch
    ts = [torch.from_numpy(np.ascontiguousarray(x)).cuda().float() for x in net.data]
    view = net.with_data([t.double().cpu().numpy() for t in ts])
    plan = T.Plan([T.NetworkSpec.from_network(net, ts)], T.TN_ACYCLIC, 4096, 4096, 0, root=0,
                  flags=T.TN_FLAG_MFMA_BF16)
    samples = torch.empty(4096, dtype=torch.float64, device="cuda")
    plan.estimate(samples_out=samples)
    torch.cuda.synchronize()
    got = samples.cpu().numpy()
    from test_gpu_m2_bf16 import bar, subtree_levels
    d = subtree_levels(net)
    for r in (0, 3, 2047, 4095):
        o = orc.m2_estimate(view, 4096, 0, r, root=0, want_trace=True)
        b = orc.m2_estimate(view, 4096, 0, r, root=0, want_trace=True, bf16_products=True)
        sk = plan.sketches(first=r, count=1).cpu().numpy()[0]
        for l in range(1, net.p):
            if d[l] == 0:
                continue
            nx = np.linalg.norm(o["x"][l])
            assert np.linalg.norm(sk[l] - o["x"][l]) <= bar(d[l]) * nx, (r, l)
            if d[l] == 1:
                assert np.linalg.norm(sk[l] - b["x"][l]) <= 6e-4 * nx, (r, l)
        scale = np.linalg.norm(o["x"][0]) * np.linalg.norm(o["r_root"])
        assert abs(got[r] - o["estimate"]) <= bar(max(d.values())) * scale, r


def test_injective_hashes_exact(T, orc):
    """Identity count sketches and collision-free tensor sketches injected through
    the test hook: Eq. (2) reproduces the exact contraction."""
    import torch
    for net in (W.example5(n=2, seed=3), W.tt_caterpillar(cores=3, bond=2, phys=2, seed=5, dtype=np.float64)):
        m = 4096
        plan, views = make_plan(T, [net], "float64", m, 2, 0)
        n = net.dims[0]
        streams = plan.streams()
        tsk = [(sid, off, nn) for (_, sid, nn, off) in streams if (1 << 62) <= sid < (1 << 63)]
        # padded order of each tensor = its largest tensor-sketch level
        qt = {}
        for sid, _, _ in tsk:
            node, level = (sid >> 32) & 0x3FFFFFFF, (sid >> 16) & 0xFFFF
            qt[node] = max(qt.get(node, 0), level)
        tab = np.zeros((2, plan.query(0)), dtype=np.int64)
        for (_, sid, nn, off) in streams:
            if sid < (1 << 62):
                tab[:, off:off + nn] = np.arange(nn)        # identity count sketches
        for sid, off, nn in tsk:
            # level l combines operands of width n^(qt/l): shift the right one past the left
            node, level, side = (sid >> 32) & 0x3FFFFFFF, (sid >> 16) & 0xFFFF, sid & 1
            width = n ** (qt[node] // level)
            tab[:, off:off + nn] = (np.arange(nn) * (width if side else 1)) % m
        # padding sketches stay at bucket 0 with sign +1
        plan.set_hashes(torch.from_numpy(tab.astype(np.int32)).cuda())
        _, got = run(plan)
        assert np.allclose(got[0], orc.tc_full(views[0]), rtol=1e-12, atol=1e-12)


def test_unbiased_on_gpu(T, orc):
    """Lemma 9 on the device: the mean of 20000 samples is within 5 standard errors
    of the Lemma 8 value, and the sample variance is below
    ((1 + 8/m)^{2t} - 1) prod ||X_k||^2."""
    net = W.example5(n=3, seed=1)
    plan, views = make_plan(T, [net], "float64", 16, 20000, 23)
    stats, got = run(plan)
    tc = orc.tc_tree(views[0], 0)
    bound = ((1 + 8 / 16) ** (2 * net.t) - 1) * views[0].input_norm() ** 2
    assert abs(stats[0, 0] - tc) <= 5 * math.sqrt(stats[0, 1] / 20000)
    assert stats[0, 1] <= bound


def test_bitwise_deterministic(T, orc):
    nets = [W.tt_caterpillar(cores=8, bond=16, phys=8, seed=2)]
    plan, _ = make_plan(T, nets, "float32", 1024, 64, 4)
    _, a = run(plan)
    _, b = run(plan)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autotuned_caterpillar(T, orc, prec):
    """TN_FLAG_AUTOTUNE on the acyclic sweep (column-split and gather block
    targets timed on the first chunk): at the benchmark's shape the tuned
    plan's estimates match the oracle (FP32 bar; FP32 products: the bar of
    test_gpu_m2_f32), differ from the default schedule's within that bar (the
    regrouping of partial sums), and repeat bit for bit."""
    import torch
    net = W.tt_caterpillar()
    extra = T.TN_FLAG_MFMA_F32 if prec == "fp32" else 0
    tuned, views = make_plan(T, [net], "float32", 4096, 4096, 0, flags=T.TN_FLAG_AUTOTUNE | extra)
    base, _ = make_plan(T, [net], "float32", 4096, 4096, 0, flags=extra)
    _, a = run(tuned)
    _, a2 = run(tuned)
    _, b = run(base)
    assert np.array_equal(a, a2)
    from test_gpu_m2_f32 import bar as bar32, widest
    from test_gpu_m2_bf16 import subtree_levels
    L = max(subtree_levels(net).values())
    tol = TAU["float32"] if prec == "fp64" else bar32(L, widest(net))
    # w and g are stored in FP32 between levels, so a regrouped FP64 sum that
    # rounds to a neighbouring FP32 value carries into the levels above
    regroup = tol
    for r in (0, 3, 2047, 4095):
        o = orc.m2_estimate(views[0], 4096, 0, r, root=0, want_trace=True)
        scale = np.linalg.norm(o["x"][0]) * np.linalg.norm(o["r_root"])
        assert abs(a[0, r] - o["estimate"]) <= tol * scale, r
        assert abs(a[0, r] - b[0, r]) <= regroup * scale, r
    torch.cuda.synchronize()
