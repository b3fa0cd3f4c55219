"""GPU parity of the cyclic-network estimator (Eq. (1)) against the FP64 oracle.

Bars: hash tables bit-exact; per-sample sketch vectors within tau * A_b where
A_b sums |X(i)| over the entries hashed to bucket b; per-sample estimates
within tau * (the oracle's first-order rounding scale
(1/m) sum_j sum_k U_k prod_{k' != k} |Y_k'[j]|, U_k = sum |X_k|).  tau = 1e-5
for FP32/BF16 data (FP32 arithmetic), 1e-12 for FP64.
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


def host_view(tensors):
    """Exactly the values the device holds, as float64 (bf16/f32 rounding included)."""
    return [t.double().cpu().numpy() for t in tensors]


def make_plan(T, nets, dtype, m, S, seed, flags=0):
    specs, views = [], []
    for n in nets:
        ts = dev(n, dtype)
        specs.append(T.NetworkSpec.from_network(n, ts))
        views.append(n.with_data(host_view(ts)))
    return T.Plan(specs, T.TN_CYCLIC, m, S, seed, flags=flags), views


def run(plan):
    import torch
    samples = torch.empty(plan.n_nets * plan.S, dtype=torch.float64, device="cuda")
    stats = plan.estimate(samples_out=samples)
    torch.cuda.synchronize()
    return stats.cpu().numpy().reshape(-1, 2), samples.cpu().numpy().reshape(plan.n_nets, plan.S)


def oracle_samples(orc, net, m, seed, samples):
    combine = "conv" if m <= 2048 else "dft"
    est, scale = [], []
    for r in samples:
        o = orc.m1_estimate(net, m, seed, r, combine=combine, want_scale=True)
        est.append(o["estimate"])
        scale.append(o["scale"])
    return np.array(est), np.array(scale)


def check_estimates(orc, plan, views, seed, dtype, samples_idx=None):
    stats, got = run(plan)
    tau = TAU[dtype]
    for j, net in enumerate(views):
        idx = list(range(plan.S)) if samples_idx is None else samples_idx
        ref, scale = oracle_samples(orc, net, plan.m, seed + j, idx)
        err = np.abs(got[j, idx] - ref)
        assert np.all(err <= tau * scale + 1e-300), (j, err.max(), (err / scale).max())
        mu, var = got[j].mean(), got[j].var(ddof=1) if plan.S > 1 else 0.0
        assert stats[j, 0] == pytest.approx(mu, rel=1e-12, abs=1e-12 * abs(scale).max())
        assert stats[j, 1] == pytest.approx(var, rel=1e-9, abs=1e-300)
    return got


def check_sketches(orc, plan, views, seed, dtype, first, count):
    """Every bucket of every tensor's sketch in samples [first, first + count)
    within tau * A_b, A_b being the same bucket of the sketch of |X| with all
    signs +1 (an entry hashed to a wrong bucket, or with a wrong sign, moves
    a bucket by about |x|, far beyond that bar)."""
    got = plan.sketches(first=first, count=count).cpu().numpy()
    k0 = 0
    for j, net in enumerate(views):
        absnet = net.with_data([np.abs(x) for x in net.data])
        for r in range(first, first + count):
            ref = orc.m1_estimate(net, plan.m, seed + j, r, want_sketches=True)["sketches"]
            tables = []
            for e in range(net.t):
                h, _ = orc.hash_table(seed + j, r, e, net.dims[net.edges[e][0]], plan.m)
                tables.append(np.concatenate([h, np.ones_like(h)]))
            A = orc.m1_estimate(absnet, plan.m, 0, 0, tables=tables, want_sketches=True)["sketches"]
            err = np.abs(got[r - first, k0:k0 + net.p] - ref)
            assert np.all(err <= TAU[dtype] * A + 1e-300), (j, r, err.max())
        k0 += net.p


@pytest.mark.parametrize("long_stream", [False, True])
def test_hashes_bit_exact(T, orc, long_stream):
    """Hash tables bit for bit against the oracle; with every stream of at most
    64 indices (one thread per stream and sample) and with a stream of 100
    (one block per stream and sample)."""
    nets = [W.triangle(8, seed=1), W.torus(L=2, D=3, seed=2), W.random_network(4, 5)]
    if long_stream:
        nets.append(W.ring(3, 100, seed=6))
    for m in (1, 64, 16384):
        plan, views = make_plan(T, nets, "float32", m, 6, 1234)
        tab = plan.hashes().cpu().numpy()
        part = plan.hashes(first=3, count=2).cpu().numpy()
        assert np.array_equal(part, tab[3:5])
        for (j, sid, n, off) in plan.streams():
            for r in range(6):
                h, s = orc.hash_table(1234 + j, r, sid, n, m)
                v = tab[r, off:off + n]
                assert np.array_equal(v & 0x7FFFFFFF, h)
                assert np.array_equal(np.where(v < 0, -1, 1), s)


@pytest.mark.parametrize("dtype", ["float64", "float32", "bfloat16"])
def test_sketch_vectors(T, orc, dtype):
    nets = [W.triangle(16, seed=3), W.Network([3, 3], [50, 40, 60, 60, 40, 50],
                                              [(0, 5), (1, 4), (2, 3)],
                                              [np.random.default_rng(5).standard_normal((50, 40, 60)),
                                               np.random.default_rng(6).standard_normal((60, 40, 50))])]
    m = 128
    plan, views = make_plan(T, nets, dtype, m, 5, 99)
    got = plan.sketches(first=1, count=4).cpu().numpy()
    k0 = 0
    for j, net in enumerate(views):
        for r in range(1, 5):
            ref = orc.m1_estimate(net, m, 99 + j, r, want_sketches=True)["sketches"]
            # A_b: the same buckets with |X| and all signs +1
            tables = []
            for e in range(net.t):
                h, _ = orc.hash_table(99 + j, r, e, net.dims[net.edges[e][0]], m)
                tables.append(np.concatenate([h, np.ones_like(h)]))
            absnet = net.with_data([np.abs(x) for x in net.data])
            A = orc.m1_estimate(absnet, m, 0, 0, tables=tables, want_sketches=True)["sketches"]
            # the complement side flips buckets, not signs, so |X| sketches bound every bucket
            err = np.abs(got[r - 1, k0:k0 + net.p] - ref)
            assert np.all(err <= TAU[dtype] * A + 1e-300), (j, r, err.max())
        k0 += net.p


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_triangle_full_size(T, orc, dtype):
    """The cyclic triangle tr(ABC) with 64 x 64 N(0,1) matrices, m = 256."""
    plan, views = make_plan(T, [W.triangle(64, seed=1)], dtype, 256, 48, 0)
    check_estimates(orc, plan, views, 0, dtype)


@pytest.mark.parametrize("m", [1024, 16384])
def test_torus_full_size(T, orc, m):
    """4 x 4 periodic lattice, bond 16, U[0,1) FP32, sampled seeds."""
    plan, views = make_plan(T, [W.torus()], "float32", m, 3, 5)
    check_estimates(orc, plan, views, 5, "float32")


def test_torus_bench_schedule(T, orc, monkeypatch):
    """The schedule the torus benchmark runs (four samples per pass, two banks,
    512-thread blocks reading their column tables once, eight loads in flight)
    on tori of the benchmark's seeds at full size, every sample against the
    oracle; then the same plan autotuned agrees to the fixed-point resolution."""
    monkeypatch.setenv("TN_SCATTER_SB", "4")
    monkeypatch.setenv("TN_SCATTER_BANKS", "2")
    nets = [W.torus(L=4, D=16, seed=2 + b) for b in range(3)]
    plan, views = make_plan(T, nets, "float32", 1024, 8, 0)
    assert plan.query(8) == 4 and plan.query(10) == 2
    got = check_estimates(orc, plan, views, 0, "float32")
    monkeypatch.delenv("TN_SCATTER_SB")
    monkeypatch.delenv("TN_SCATTER_BANKS")
    tuned, _ = make_plan(T, nets, "float32", 1024, 8, 0, flags=T.TN_FLAG_AUTOTUNE)
    _, got2 = run(tuned)
    assert np.all(np.abs(got2 - got) <= 1e-9 * np.abs(got).max())


@pytest.mark.parametrize("m", [16384, 32768, 65536])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_torus_large_m(T, orc, m, dtype):
    """m above the in-LDS FFT (two-pass combine: m = 16384 with FP64 data, all
    of 32768 and 65536) and above the in-LDS sketch (bucket-range scatter:
    32768 and 65536), the 4 x 4 torus (bond 16), sampled seeds."""
    plan, views = make_plan(T, [W.torus()], dtype, m, 2, 5)
    if m > 16384:
        assert plan.query(8) == 1 and plan.query(10) == 1  # one sample per pass, one bank
    check_estimates(orc, plan, views, 5, dtype)


def test_m8192_fp64_odd_networks_and_slots(T, orc):
    """FP64 sketches at m = 8192: the in-LDS combine at its largest FP64 size
    (1024 threads, two-level twiddles, the next pair's first slots loaded during
    the current transform), with odd tensor counts and a tensor cut into
    several slots, against the oracle per sample."""
    big = W.Network([3, 3], [50, 40, 60, 60, 40, 50], [(0, 5), (1, 4), (2, 3)],
                    [np.random.default_rng(5).standard_normal((50, 40, 60)),
                     np.random.default_rng(6).standard_normal((60, 40, 50))])
    nets = [W.triangle(24, seed=7), W.ring(5, 10, seed=8), W.random_network(7, 6, dtype=np.float64), big]
    plan, views = make_plan(T, nets, "float64", 8192, 3, 41)
    check_estimates(orc, plan, views, 41, "float64")


@pytest.mark.parametrize("m", [8192, 16384, 32768, 65536])
def test_large_m_odd_networks_fp32(T, orc, m):
    """FP32 sketches at large m with odd tensor counts (a tensor alone in its
    complex transform): the in-LDS combine with two-level twiddles and 1024
    threads (m = 8192, 16384) and the two-pass combine with tensor pairs and
    mirror-row blocks (m = 32768, 65536), against the oracle per sample."""
    nets = [W.triangle(24, seed=7), W.ring(5, 10, seed=8), W.random_network(7, 6)]
    plan, views = make_plan(T, nets, "float32", m, 3, 31)
    assert plan.query(8) == 1 or m <= 16384
    check_estimates(orc, plan, views, 31, "float32")


def test_large_m_multi_slot_and_sketches(T, orc):
    """m = 65536 with a tensor split into several slots, a triangle and a ring in
    one plan; the exported sketches match the oracle's bucket by bucket.  (The
    oracle's DFT combine: its direct convolution is O(p m^2) at this m.)"""
    big = W.Network([3, 3], [50, 40, 60, 60, 40, 50], [(0, 5), (1, 4), (2, 3)],
                    [np.random.default_rng(5).standard_normal((50, 40, 60)),
                     np.random.default_rng(6).standard_normal((60, 40, 50))])
    nets = [big, W.triangle(16, seed=3), W.ring(5, 12, seed=4)]
    m = 65536
    plan, views = make_plan(T, nets, "float64", m, 3, 21)
    check_estimates(orc, plan, views, 21, "float64")
    got = plan.sketches(first=1, count=1).cpu().numpy()
    k0 = 0
    for j, net in enumerate(views):
        ref = orc.m1_estimate(net, m, 21 + j, 1, combine="dft", want_sketches=True)["sketches"]
        # A_b: the same buckets with |X| and all signs +1 (as in test_sketch_vectors)
        tables = []
        for e in range(net.t):
            h, _ = orc.hash_table(21 + j, 1, e, net.dims[net.edges[e][0]], m)
            tables.append(np.concatenate([h, np.ones_like(h)]))
        absnet = net.with_data([np.abs(x) for x in net.data])
        A = orc.m1_estimate(absnet, m, 0, 0, tables=tables, combine="dft", want_sketches=True)["sketches"]
        # terms per bucket, and the 64-bit fixed point's rounding of each term:
        # half a quantum 2^(e + lgN - 62), max|X_k| < 2^e, lgN = max(ceil log2 N, 11)
        # for the N entries of the scatter block (at most the tensor's size)
        ones = net.with_data([np.ones_like(x) for x in net.data])
        cnt = orc.m1_estimate(ones, m, 0, 0, tables=tables, combine="dft", want_sketches=True)["sketches"]
        q = np.array([2.0 ** (np.frexp(np.abs(x).max())[1] + max(int(np.ceil(np.log2(x.size))), 11) - 62)
                      for x in net.data])
        bar = TAU["float64"] * A + cnt * (q[:, None] / 2)
        assert np.all(np.abs(got[0, k0:k0 + net.p] - ref) <= bar + 1e-300), j
        k0 += net.p


def test_m_above_65536_rejected(T):
    import torch
    net = W.triangle(8, seed=1)
    spec = T.NetworkSpec.from_network(net, [torch.from_numpy(x).cuda() for x in net.data])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec], T.TN_CYCLIC, 131072, 2, 1)
    assert e.value.code == T.TN_ERR_UNSUPPORTED


def test_batched_random_networks(T, orc):
    """Uneven random cyclic networks (3-12 tensors, bonds 2-32) in one plan."""
    nets = W.random_batch(count=12, seed=4)
    plan, views = make_plan(T, nets, "float32", 1024, 3, 11)
    check_estimates(orc, plan, views, 11, "float32")


def test_batched_bench_shape(T, orc):
    """The benchmark's batch: all 4096 random cyclic networks (29,912 tensors,
    1.16 GB of FP32) in one autotuned plan, S = 16; sampled networks and
    samples against the oracle, and the plan's statistics against its samples."""
    import torch
    nets = W.random_batch(count=4096, seed=4)
    specs, views = [], []
    for n in nets:
        ts = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float32) for x in n.data]
        specs.append(T.NetworkSpec.from_network(n, ts))
        views.append((n, ts))
    plan = T.Plan(specs, T.TN_CYCLIC, 1024, 16, 0, flags=T.TN_FLAG_AUTOTUNE)
    stats, got = run(plan)
    for j in (0, 1, 2047, 4095):
        n, ts = views[j]
        v = n.with_data([t.double().cpu().numpy() for t in ts])
        ref, scale = oracle_samples(orc, v, 1024, 0 + j, [0, 7, 15])
        assert np.all(np.abs(got[j, [0, 7, 15]] - ref) <= TAU["float32"] * scale), j
    assert np.allclose(stats[:, 0], got.mean(axis=1), rtol=1e-12, atol=0)


@pytest.mark.parametrize("sb,banks", [(1, 1), (2, 1), (4, 2), (8, 1)])
@pytest.mark.parametrize("dtype", ["float64", "float32", "bfloat16"])
def test_rows_off_the_vector_grid(T, orc, monkeypatch, dtype, sb, banks):
    """Rows of 37 entries (no whole number of 16-byte vectors) and slots that
    start 0, 1 and 2 FP32 entries into a vector (rows 0, 1771 and 3542 of a
    (40 x 100) x 37 tensor): the scatter's flat-vector path, whose vectors run
    across rows and whose first and last partial vectors are read singly, at
    several schedules, every sample against the oracle."""
    monkeypatch.setenv("TN_SCATTER_SB", str(sb))
    monkeypatch.setenv("TN_SCATTER_BANKS", str(banks))
    rng = np.random.default_rng(11)
    net = W.Network([3, 3], [40, 100, 37, 37, 100, 40], [(2, 3), (1, 4), (0, 5)],
                    [rng.standard_normal((40, 100, 37)), rng.standard_normal((37, 100, 40))])
    plan, views = make_plan(T, [net], dtype, 1024, 8, 21)
    assert plan.query(8) <= sb
    check_sketches(orc, plan, views, 21, dtype, 0, 8)
    check_estimates(orc, plan, views, 21, dtype)


@pytest.mark.parametrize("sb,banks", [(2, 1), (4, 2)])
@pytest.mark.parametrize("m", [16, 1024])
@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
def test_table_build_paths(T, orc, monkeypatch, dtype, m, sb, banks):
    """The scatter's table build and unaligned loops on one ring: A (600 x 3,
    rows of 3 entries: shorter than a 16-byte vector, which then spans several
    rows), B (111 x 37) and C (37 x 185, both rows that are no whole number of
    vectors: a vector runs into the next row and reads the wrapped column
    table), D (5 x 600).  At m = 1024 the column modes' hash words are staged
    in the accumulator LDS; at m = 16 they do not fit there (B, C and D need
    more words than the accumulators hold) and every column reads the global
    tables.  Sketches and estimates of every sample against the oracle."""
    monkeypatch.setenv("TN_SCATTER_SB", str(sb))
    monkeypatch.setenv("TN_SCATTER_BANKS", str(banks))
    rng = np.random.default_rng(13)
    shapes = [(600, 3), (3, 37, 37), (37, 37, 5), (5, 600)]
    net = W.Network([2, 3, 3, 2], [600, 3, 3, 37, 37, 37, 37, 5, 5, 600],
                    [(1, 2), (3, 5), (4, 6), (7, 8), (9, 0)], [rng.standard_normal(sh) for sh in shapes])
    plan, views = make_plan(T, [net], dtype, m, 4, 17)
    check_sketches(orc, plan, views, 17, dtype, 0, 4)
    check_estimates(orc, plan, views, 17, dtype)


@pytest.mark.parametrize("dtype", ["float64", "float32", "bfloat16"])
def test_misaligned_tensor_base(T, orc, dtype):
    """Tensors that start 1 or 3 elements past a 16-byte boundary (views at a
    storage offset): every slot takes the flat-vector path, including slots
    shorter than their unaligned head (a 2 x 1 matrix), against the oracle."""
    import torch
    rng = np.random.default_rng(12)
    shapes = [(2, 1), (1, 64), (64, 64), (64, 2)]
    net = W.Network([2, 2, 2, 2], [2, 1, 1, 64, 64, 64, 64, 2], [(1, 2), (3, 4), (5, 6), (7, 0)],
                    [rng.standard_normal(sh) for sh in shapes])
    td = getattr(torch, dtype)
    ts = []
    for k, x in enumerate(net.data):
        o = 1 + 2 * (k % 2)
        buf = torch.zeros(x.size + o, dtype=td, device="cuda")
        buf[o:] = torch.from_numpy(x.ravel()).to(td).cuda()
        ts.append(buf[o:].view(x.shape))
        assert ts[-1].data_ptr() % 16 != 0
    plan = T.Plan([T.NetworkSpec.from_network(net, ts)], T.TN_CYCLIC, 256, 6, 3)
    views = [net.with_data(host_view(ts))]
    check_sketches(orc, plan, views, 3, dtype, 0, 6)
    check_estimates(orc, plan, views, 3, dtype)


def test_bounds_follow_the_data(T, orc):
    """The per-slot fixed-point bounds are taken again on every call: one plan
    run on its tensors scaled in place (same pointers) by 2^-12, then 2^12 (a
    stale bound would overflow the accumulators), then 1, every sample against
    the oracle each time; and a call for later samples only (sketches of
    samples 5..7) against the oracle's sketches."""
    net = W.torus(L=2, D=8, seed=7)
    ts = dev(net, "float32")
    plan = T.Plan([T.NetworkSpec.from_network(net, ts)], T.TN_CYCLIC, 1024, 8, 9)
    base = [t.clone() for t in ts]
    for f in (2.0 ** -12, 2.0 ** 12, 1.0):
        for t, b in zip(ts, base):
            t.copy_(b * f)
        views = [net.with_data(host_view(ts))]
        check_estimates(orc, plan, views, 9, "float32")
    check_sketches(orc, plan, views, 9, "float32", 5, 3)


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_combine_split_over_pairs(T, orc, dtype):
    """Few (network, sample) blocks and a long product (pairs x m >= 65536):
    the in-LDS combine splits each network's tensor pairs over several blocks
    and joins their product spectra.  A ring of 33 tensors (an odd one out), a
    triangle (whose later shares are empty) and a single self-contracted
    matrix at m = 4096, S = 4, against the oracle."""
    rng = np.random.default_rng(21)
    nets = [W.ring(33, 5, seed=3), W.triangle(12, seed=4),
            W.Network([2], [9, 9], [(0, 1)], [rng.standard_normal((9, 9))])]
    plan, views = make_plan(T, nets, dtype, 4096, 4, 5)
    assert plan.query(14) > 1          # blocks per (network, sample)
    check_estimates(orc, plan, views, 5, dtype)
    short, _ = make_plan(T, nets[1:], dtype, 4096, 4, 5)   # 2 pairs x 4096 < 65536: not split
    assert short.query(14) == 1


@pytest.mark.parametrize("m,S", [(1, 3), (2, 5), (4, 7), (32, 1), (64, 17)])
def test_edge_cases(T, orc, m, S):
    rng = np.random.default_rng(m + S)
    x, y = rng.standard_normal(9), rng.standard_normal(9)
    single = W.Network([1, 1], [9, 9], [(0, 1)], [x, y])
    trace = W.Network([2], [6, 6], [(0, 1)], [rng.standard_normal((6, 6))])     # self-contraction
    odd = W.ring(3, 5, seed=S)
    plan, views = make_plan(T, [single, trace, odd], "float64", m, S, 3)
    check_estimates(orc, plan, views, 3, "float64")


def test_injective_hashes_exact(T, orc):
    """Collision-free tables injected through the test hook: Eq. (1) is exact."""
    import torch
    net = W.triangle(3, seed=2)
    n, B = 3, 6
    m = 256                             # >= B^t = 216
    plan, views = make_plan(T, [net], "float64", m, 2, 0)
    W_ = plan.query(0)
    tab = np.zeros((2, W_), dtype=np.int32)
    for (j, sid, nn, off) in plan.streams():
        tab[:, off:off + nn] = (np.arange(nn) * B**sid) % m
    plan.set_hashes(torch.from_numpy(tab).cuda())
    stats, got = run(plan)
    tc = orc.tc_full(views[0])
    assert np.allclose(got[0], tc, rtol=1e-12, atol=1e-12)
    plan.set_hashes(None)
    _, got2 = run(plan)
    assert not np.allclose(got2[0], tc)


def test_degenerate_hashes(T, orc):
    """h = 0, s = +1 injected: the estimate is prod_k sum_i X_k(i)."""
    import torch
    net = W.random_network(4, 2)
    plan, views = make_plan(T, [net], "float32", 64, 3, 0)
    plan.set_hashes(torch.zeros((3, plan.query(0)), dtype=torch.int32, device="cuda"))
    _, got = run(plan)
    ref = np.prod([x.sum() for x in views[0].data])
    scale = np.prod([np.abs(x).sum() for x in views[0].data])
    assert np.all(np.abs(got[0] - ref) <= 1e-5 * scale)


def test_unbiased_on_gpu(T, orc):
    """Lemma 6 on the device: the mean of 20000 samples is within 5 standard
    errors of tc, and the sample variance is below 3^t/m prod ||X_k||^2."""
    net = W.triangle(8, seed=10)
    plan, views = make_plan(T, [net], "float64", 64, 20000, 17)
    stats, got = run(plan)
    tc = orc.tc_full(views[0])
    bound = 3**3 / 64 * views[0].input_norm() ** 2
    assert abs(stats[0, 0] - tc) <= 5 * math.sqrt(stats[0, 1] / 20000)
    assert stats[0, 1] <= bound


def test_graph_replay(T, orc):
    import torch
    nets = [W.torus(L=2, D=8, seed=3), W.triangle(12, seed=4).astype(np.float32)]
    plan_g, views = make_plan(T, nets, "float32", 256, 9, 21, flags=T.TN_FLAG_GRAPH)
    plan_e, _ = make_plan(T, nets, "float32", 256, 9, 21)
    _, ref = run(plan_e)
    for rep in range(3):
        junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
        _, got = run(plan_g)
        for j, net in enumerate(views):
            _, scale = oracle_samples(orc, net, 256, 21 + j, range(9))
            assert np.all(np.abs(got[j] - ref[j]) <= 2e-5 * scale)
        del junk


def test_graph_replay_split_combine(T, orc):
    """A captured estimate whose combine is split over the pairs (one long
    ring, few blocks): three replays with eager work between them, each
    bitwise the eager run's estimates, and those against the oracle."""
    import torch
    nets = [W.ring(33, 5, seed=7)]
    plan_g, views = make_plan(T, nets, "float64", 4096, 3, 9, flags=T.TN_FLAG_GRAPH)
    plan_e, _ = make_plan(T, nets, "float64", 4096, 3, 9)
    _, ref = run(plan_e)
    for rep in range(3):
        junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
        _, got = run(plan_g)
        assert np.array_equal(got, ref)
        del junk
    want, scale = oracle_samples(orc, views[0], 4096, 9, range(3))
    assert np.all(np.abs(ref[0] - want) <= TAU["float64"] * scale)


def test_graph_replay_after_data_change(T, orc):
    """A replayed graph takes the slot bounds afresh: the tensors scaled in
    place by 2^12 between replays (same pointers), every sample of both
    replays against the oracle."""
    net = W.torus(L=2, D=8, seed=5)
    ts = dev(net, "float32")
    plan = T.Plan([T.NetworkSpec.from_network(net, ts)], T.TN_CYCLIC, 256, 12, 4, flags=T.TN_FLAG_GRAPH)
    base = [t.clone() for t in ts]
    for f in (1.0, 2.0 ** 12):
        for t, b in zip(ts, base):
            t.copy_(b * f)
        check_estimates(orc, plan, [net.with_data(host_view(ts))], 4, "float32")


def test_bitwise_deterministic_across_schedules(T, orc, monkeypatch):
    """Fixed-point sketch accumulation.  Every sample batch of an estimate call
    after the first starts from the slot bounds the first batch recorded, so its
    sketches are exact integer sums at one fixed scale: bit-identical run to run
    and for every samples-per-pass choice and accumulator layout.  The first
    batch keeps a running maximum; where the maximum grows after a block's first
    load round it rescales its accumulators, at points that depend on the block
    size and on which samples share the batch, so those samples agree to the
    fixed-point resolution (2^-46 of the slot's max |x| per term) only.  The
    second network holds an N(0,1) tensor of 8192 entries whose largest entry
    sits at its end (a rescale after the first round); the first is a small
    torus and a random network."""
    rng = np.random.default_rng(17)
    big = rng.standard_normal((64, 128))
    big[-1, -1] = 8.0 * np.abs(big).max()
    late_max = W.Network([2, 2], [64, 128, 128, 64], [(0, 3), (1, 2)], [big, rng.standard_normal((128, 64))])
    nets = [W.torus(L=2, D=16, seed=9), W.random_network(4, 3), late_max]
    S, first = 24, 8          # samples; the largest first batch (8 samples per pass)
    runs = {}
    for banks in ("1", "2"):
        monkeypatch.setenv("TN_SCATTER_BANKS", banks)
        for sb in ("1", "2", "4", "8"):
            monkeypatch.setenv("TN_SCATTER_SB", sb)
            p, views = make_plan(T, nets, "float32", 1024, S, 8)
            assert p.query(8) == int(sb) and p.query(10) == int(banks)
            _, g = run(p)
            _, g2 = run(p)
            assert np.array_equal(g, g2)
            runs[(sb, banks)] = g
    ref_run = runs[("1", "1")]
    for key, g in runs.items():
        assert np.array_equal(g[:, first:], ref_run[:, first:]), key
        assert np.all(np.abs(g - ref_run) <= 1e-9 * np.abs(ref_run).max(axis=1, keepdims=True)), key
    for j, net in enumerate(views):
        ref, scale = oracle_samples(orc, net, 1024, 8 + j, [0, 1, first, S - 1])
        for g in runs.values():
            assert np.all(np.abs(g[j, [0, 1, first, S - 1]] - ref) <= 1e-5 * scale)
    monkeypatch.delenv("TN_SCATTER_SB")
    monkeypatch.delenv("TN_SCATTER_BANKS")
    b, _ = make_plan(T, nets, "float32", 1024, S, 8, flags=T.TN_FLAG_AUTOTUNE)
    _, gb = run(b)
    assert b.query(8) in (1, 2, 4, 8, 16) and b.query(10) in (1, 2)
    assert np.array_equal(gb[:, 16:], ref_run[:, 16:])
    assert np.all(np.abs(gb - ref_run) <= 1e-9 * np.abs(ref_run).max(axis=1, keepdims=True))


@pytest.mark.parametrize("dtype", ["float64", "float32", "bfloat16"])
def test_two_bank_scatter_parity(T, orc, dtype, monkeypatch):
    """The two-bank accumulators (sign in the address) against the oracle: sketches
    within tau * A_b and estimates within tau * A_hat, on multi-slot tensors, a
    ragged sample batch and m = 64 / 4096."""
    monkeypatch.setenv("TN_SCATTER_BANKS", "2")
    big = W.Network([3, 3], [50, 40, 60, 60, 40, 50], [(0, 5), (1, 4), (2, 3)],
                    [np.random.default_rng(5).standard_normal((50, 40, 60)),
                     np.random.default_rng(6).standard_normal((60, 40, 50))])
    for m, S in ((64, 5), (4096, 3)):
        plan, views = make_plan(T, [W.triangle(16, seed=3), big, W.random_network(4, 11)], dtype, m, S, 21)
        assert plan.query(10) == 2
        check_estimates(orc, plan, views, 21, dtype)


def _brute_force_sized(count, limit=5e7):
    """Random cyclic networks whose brute-force oracle sum has <= limit terms."""
    out = []
    for i in range(200):
        n = W.random_network(6, i, bmax=9, pmax=7)
        terms = float(np.prod([float(n.dims[u]) for u, _ in n.edges]))
        if terms <= limit and n.nnz() >= 500:
            out.append(n)
        if len(out) == count:
            break
    return out


def test_exact_contraction(T, orc):
    for net, dtype in [(n, "float32") for n in _brute_force_sized(3)] + [(W.triangle(16, seed=1), "float64"), (W.ring(4, 6, seed=2), "float64"),
                       (W.torus(L=2, D=4, seed=3), "float32"), (W.example5(n=3), "float64"),
                       (W.random_network(4, 7, bmax=4, pmax=6), "float32"),
                       (W.random_network(4, 8, bmax=5, pmax=5), "float32"),
                       (W.Network([2], [5, 5], [(0, 1)], [np.arange(25.0).reshape(5, 5)]), "float64")]:
        ts = dev(net, dtype)
        v = net.with_data(host_view(ts))
        got = T.tn_contract_exact(T.NetworkSpec.from_network(net, ts))
        ref = orc.tc_full(v)
        scale = np.prod([np.abs(x).sum() for x in v.data])
        assert abs(got - ref) <= 1e-12 * scale + 1e-12 * abs(ref), (net.name, got, ref)


def test_profile_sketch_only(T, orc):
    """TN_FLAG_PROFILE_SKETCH records events around the sketching launches only;
    the estimates are those of an unprofiled plan; without TN_FLAG_PROFILE it
    is rejected."""
    nets = [W.triangle(16, seed=2), W.ring(5, 12, seed=4)]
    base, _ = make_plan(T, nets, "float32", 256, 6, 8)
    prof, _ = make_plan(T, nets, "float32", 256, 6, 8, flags=T.TN_FLAG_PROFILE | T.TN_FLAG_PROFILE_SKETCH)
    _, g0 = run(base)
    _, g1 = run(prof)
    assert np.array_equal(g0, g1)
    ms, n = prof.kernel_time(T.TN_KERNEL_SKETCH)
    assert n > 0 and ms > 0.0
    for k in (T.TN_KERNEL_HASH, T.TN_KERNEL_COMBINE, T.TN_KERNEL_STATS):
        assert prof.kernel_time(k) == (0.0, 0)
    with pytest.raises(T.TNError) as e:
        make_plan(T, nets, "float32", 256, 6, 8, flags=T.TN_FLAG_PROFILE_SKETCH)
    assert e.value.code == T.TN_ERR_ARG


def test_tt_ladder_full_size(T, orc):
    """The literal inner product of two tensor trains (a cyclic ladder: 64
    cores of (64, 64, 64), 94 contractions) through the cyclic estimator at
    m = 4096, sampled estimates against the oracle; the exact FP64
    contraction agrees with the oracle's on a small ladder."""
    net = W.tt_ladder()
    plan, views = make_plan(T, [net], "float32", 4096, 2, 3)
    check_estimates(orc, plan, views, 3, "float32")
    small = W.tt_ladder(cores=4, bond=3, phys=2, seed=5, dtype=np.float64)
    spec = T.NetworkSpec.from_network(small, dev(small, "float64"))
    assert T.tn_contract_exact(spec) == pytest.approx(orc.tc_full(small), rel=1e-12, abs=1e-14)


def test_tn_log_plan_and_autotune(T, orc, capfd, monkeypatch):
    """TN_LOG=2: a plan prints its layout and the autotuner each candidate and
    its choice (or the cached schedule) on stderr, acyclic plans likewise."""
    monkeypatch.setenv("TN_LOG", "2")
    nets = [W.ring(5, 24, seed=77), W.triangle(24, seed=78)]
    plan, _ = make_plan(T, nets, "float32", 512, 24, 3, flags=T.TN_FLAG_AUTOTUNE)
    run(plan)
    err = capfd.readouterr().err
    assert "[tn] plan: cyclic, 2 networks" in err, err
    assert "[tn] autotune: " in err, err
    import torch
    net = W.tt_caterpillar(cores=4, bond=8, phys=4, seed=79)
    ts = [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in net.data]
    p2 = T.Plan([T.NetworkSpec.from_network(net, ts)], T.TN_ACYCLIC, 256, 128, 1, flags=T.TN_FLAG_AUTOTUNE)
    p2.estimate()
    torch.cuda.synchronize()
    err = capfd.readouterr().err
    assert "[tn] plan: acyclic, 1 networks" in err and "[tn] autotune: split target" in err, err
