"""The cyclic method's combine with its 1024-point DFTs on the BF16 matrix
cores (TN_FLAG_DFT_BF16) against the FP64 oracle.

The sketches (and hashes) are those of the FP32 path; only the transforms
round: two stages, each multiplying BF16-rounded factors (the 32-point DFT
matrix, the sketch or the twiddled intermediate) with FP32 accumulation, so a
spectrum value Y_k[j] moves by at most about 6 2^-9 sum_b |y_k[b]| <= 6 2^-9
U_k (U_k = sum |X_k|) to first order, and an estimate by at most 8 2^-9 times
the oracle's scale (1/m) sum_j sum_k U_k prod_{k' != k} |Y_k'[j]|.  The tests
print the measured errors in that scale, and check that the matrix-core
estimates are not the FP32 ones (the rounding is there) while their spread over
samples, the estimator's own error, is unchanged to 2 %."""
import numpy as np
import pytest

import tn_workloads as W
from test_gpu_m1 import make_plan, oracle_samples, run

pytestmark = pytest.mark.gpu

BAR = 8 * 2.0 ** -9


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    return T


@pytest.mark.parametrize("dtype", ["float32", "bfloat16"])
def test_estimates_against_oracle(T, orc, dtype):
    nets = [W.triangle(32, seed=2), W.ring(5, 12, seed=4), W.random_network(4, 11), W.torus(L=2, D=8, seed=3),
            W.Network([3, 3], [50, 40, 60, 60, 40, 50], [(0, 5), (1, 4), (2, 3)],
                      [np.random.default_rng(5).standard_normal((50, 40, 60)),
                       np.random.default_rng(6).standard_normal((60, 40, 50))])]
    plan, views = make_plan(T, nets, dtype, 1024, 6, 31, flags=T.TN_FLAG_DFT_BF16)
    _, got = run(plan)
    worst = 0.0
    for j, net in enumerate(views):
        ref, scale = oracle_samples(orc, net, 1024, 31 + j, range(6))
        rel = np.abs(got[j] - ref) / scale
        assert np.all(rel <= BAR), (j, rel.max())
        worst = max(worst, rel.max())
    print(f"{dtype}: max |error| / scale = {worst:.3e} (bar {BAR:.3e})")


def test_tensor_counts(T, orc):
    """The transform loop takes the next two tensors' sketch loads in turns:
    networks of 1 (a self-contracted matrix), 2, 6 and 7 tensors (each parity
    of the unrolled loop, and one tensor split into two slots), every sample
    within the bar."""
    rng = np.random.default_rng(8)
    nets = [W.Network([2], [40, 40], [(0, 1)], [rng.standard_normal((40, 40))]),
            W.Network([1, 1], [300, 300], [(0, 1)], [rng.standard_normal(300), rng.standard_normal(300)]),
            W.ring(6, 9, seed=5), W.ring(7, 11, seed=6),
            W.Network([2, 2, 2], [300, 260, 260, 300, 300, 300], [(1, 2), (3, 4), (5, 0)],
                      [rng.standard_normal((300, 260)), rng.standard_normal((260, 300)),
                       rng.standard_normal((300, 300))])]
    plan, views = make_plan(T, nets, "float32", 1024, 5, 11, flags=T.TN_FLAG_DFT_BF16)
    _, got = run(plan)
    for j, net in enumerate(views):
        ref, scale = oracle_samples(orc, net, 1024, 11 + j, range(5))
        assert np.all(np.abs(got[j] - ref) <= BAR * scale), (j, (np.abs(got[j] - ref) / scale).max())


def test_batch_networks_and_rounding_visible(T, orc):
    """Sampled networks of the benchmark's batch: within the bar; the
    matrix-core estimates differ from the FP32 ones (BF16 rounding present);
    the standard deviation over 64 samples agrees with the FP32 path's to 2 %
    (the rounding is far below the estimator's own spread)."""
    nets = W.random_batch(count=64, seed=4)
    pb, views = make_plan(T, nets, "float32", 1024, 64, 0, flags=T.TN_FLAG_DFT_BF16)
    pf, _ = make_plan(T, nets, "float32", 1024, 64, 0)
    sb, gb = run(pb)
    sf, gf = run(pf)
    for j in (0, 17, 63):
        ref, scale = oracle_samples(orc, views[j], 1024, j, [0, 31, 63])
        assert np.all(np.abs(gb[j, [0, 31, 63]] - ref) <= BAR * scale)
    assert np.any(gb != gf)
    ratio = np.sqrt(sb[:, 1] / sf[:, 1])
    assert np.all(np.abs(ratio - 1.0) <= 0.02), ratio.min()


def test_rejects_other_sizes(T):
    import torch
    net = W.triangle(8, seed=1, dtype=np.float32)
    spec = T.NetworkSpec.from_network(net, [torch.from_numpy(x).cuda() for x in net.data])
    for m in (512, 2048):
        with pytest.raises(T.TNError) as e:
            T.Plan([spec], T.TN_CYCLIC, m, 4, 1, flags=T.TN_FLAG_DFT_BF16)
        assert e.value.code == T.TN_ERR_UNSUPPORTED
    with pytest.raises(T.TNError) as e:
        T.Plan([spec], T.TN_CYCLIC, 1024, 4, 1, flags=T.TN_FLAG_DFT_BF16 | T.TN_FLAG_PERSISTENT)
    assert e.value.code == T.TN_ERR_UNSUPPORTED


def test_batched_bench_shape(T, orc):
    """The benchmark's default configuration: all 4096 networks of the batch in
    one autotuned plan with TN_FLAG_DFT_BF16, S = 16 (two sample chunks);
    sampled networks and samples, including the last of each chunk, against
    the oracle within the bar."""
    import torch
    nets = W.random_batch(count=4096, seed=4)
    specs, views = [], []
    for n in nets:
        ts = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float32) for x in n.data]
        specs.append(T.NetworkSpec.from_network(n, ts))
        views.append((n, ts))
    plan = T.Plan(specs, T.TN_CYCLIC, 1024, 16, 0, flags=T.TN_FLAG_AUTOTUNE | T.TN_FLAG_DFT_BF16)
    stats, got = run(plan)
    worst = 0.0
    for j in (0, 1, 2047, 4095):
        n, ts = views[j]
        v = n.with_data([t.double().cpu().numpy() for t in ts])
        ref, scale = oracle_samples(orc, v, 1024, j, [0, 7, 8, 15])
        rel = np.abs(got[j, [0, 7, 8, 15]] - ref) / scale
        assert np.all(rel <= BAR), (j, rel.max())
        worst = max(worst, rel.max())
    assert np.allclose(stats[:, 0], got.mean(axis=1), rtol=1e-12, atol=0)
    print(f"bench shape: max |error| / scale = {worst:.3e} (bar {BAR:.3e})")
