"""The cyclic method's combine with its 1024-point DFTs on the FP8 matrix
cores (TN_FLAG_DFT_FP8: OCP E4M3 operands, FP32 accumulation, power-of-two
block scales undone in FP64, the data rounded stochastically, the DFT constants
as two E4M3 terms) against the FP64 oracle and the FP32 path.

E4M3 keeps 3 mantissa bits; a stochastic rounding moves a value by less than
one ulp, 2^-3 relative.  With the first-order argument of test_gpu_dft_bf16 an
estimate then moves by at most 8 2^-3 times the oracle's rounding scale
(1/m) sum_j sum_k U_k prod_{k' != k} |Y_k'[j]| (U_k = sum |X_k|).  That bar is
loose (U_k far exceeds a typical |Y_k[j]|), so the tests check what matters
for an estimator as well:
* with the same hashes, the rms difference between the FP8 and FP32 estimates
  (the rounding noise) is at most 0.3 of the spread of the FP32 estimates over
  samples, so it adds at most 4.5 % to the variance (a wrong operand layout,
  sign or scale makes it larger than the spread itself);
* on a positive triangle the mean of 2^16 estimates lies within five standard
  errors of the exact contraction.
The last check is what the two-term constants and the stochastic rounding are
for.  With both rounded to nearest, the estimates shrank: the triangle's mean
fell 0.7 % (16 standard errors) and the spread about 3 %.  With only the
constants split it rose 0.5 % (12 standard errors), because rounding errors to
nearest correlate across tensors through the shared hashes.  Measured values
are printed."""
import math

import numpy as np
import pytest

import tn_workloads as W
from test_gpu_m1 import make_plan, oracle_samples, run

pytestmark = pytest.mark.gpu

BAR = 8 * 2.0 ** -3


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
    plan, views = make_plan(T, nets, dtype, 1024, 6, 31, flags=T.TN_FLAG_DFT_FP8)
    _, got = run(plan)
    assert np.all(np.isfinite(got))
    worst = 0.0
    for j, net in enumerate(views):
        ref, scale = oracle_samples(orc, net, 1024, 31 + j, range(6))
        rel = np.abs(got[j] - ref) / scale
        assert np.all(rel <= BAR), (j, rel.max())
        worst = max(worst, rel.max())
    print(f"{dtype}: max |error| / scale = {worst:.3e} (bar {BAR:.3e})")


def test_tensor_counts(T, orc):
    """The loads of the next two tensors taken in turns, as in the BF16 kernel:
    networks of 1, 2, 6, 7 and 3 tensors (one split into two slots), every
    sample within the bar."""
    rng = np.random.default_rng(8)
    nets = [W.Network([2], [40, 40], [(0, 1)], [rng.standard_normal((40, 40))]),
            W.Network([1, 1], [300, 300], [(0, 1)], [rng.standard_normal(300), rng.standard_normal(300)]),
            W.ring(6, 9, seed=5), W.ring(7, 11, seed=6),
            W.Network([2, 2, 2], [300, 260, 260, 300, 300, 300], [(1, 2), (3, 4), (5, 0)],
                      [rng.standard_normal((300, 260)), rng.standard_normal((260, 300)),
                       rng.standard_normal((300, 300))])]
    plan, views = make_plan(T, nets, "float32", 1024, 5, 11, flags=T.TN_FLAG_DFT_FP8)
    _, got = run(plan)
    assert np.all(np.isfinite(got))
    for j, net in enumerate(views):
        ref, scale = oracle_samples(orc, net, 1024, 11 + j, range(5))
        assert np.all(np.abs(got[j] - ref) <= BAR * scale), (j, (np.abs(got[j] - ref) / scale).max())


def test_batch_noise_below_the_estimators_spread(T, orc):
    """64 networks of the benchmark's batch, 256 samples: FP8 against FP32 with
    the same hashes, and a few samples against the oracle."""
    nets = W.random_batch(count=64, seed=4)
    p8, views = make_plan(T, nets, "float32", 1024, 256, 0, flags=T.TN_FLAG_DFT_FP8)
    pf, _ = make_plan(T, nets, "float32", 1024, 256, 0)
    s8, g8 = run(p8)
    sf, gf = run(pf)
    for j in (0, 17, 63):
        ref, scale = oracle_samples(orc, views[j], 1024, j, [0, 255])
        assert np.all(np.abs(g8[j, [0, 255]] - ref) <= BAR * scale)
    spread = gf.std(axis=1, ddof=1)
    noise = np.sqrt(np.mean((g8 - gf) ** 2, axis=1))
    ratio = np.sqrt(s8[:, 1] / sf[:, 1])
    print(f"noise / spread: median {np.median(noise / spread):.3f}, max {np.max(noise / spread):.3f}; "
          f"spread ratio {ratio.min():.4f} .. {ratio.max():.4f}")
    assert np.any(g8 != gf)
    assert np.all(noise <= 0.3 * spread), np.max(noise / spread)
    # |std(a) - std(b)| <= rms(a - b): the spreads then agree within 0.3 too
    assert np.all(np.abs(ratio - 1.0) <= 0.3), (ratio.min(), ratio.max())


def test_unbiased_on_a_positive_triangle(T, orc):
    import torch
    net = W.triangle(8, seed=5, dist="uniform", dtype=np.float32)
    tc = orc.tc_full(net.with_data([np.asarray(x, dtype=np.float64) for x in net.data]))
    S = 1 << 16
    plan, _ = make_plan(T, [net], "float32", 1024, S, 21, flags=T.TN_FLAG_DFT_FP8)
    st, _ = run(plan)
    mean, se = st[0, 0], math.sqrt(st[0, 1] / S)
    print(f"triangle: mean {mean:.6g}, tc {tc:.6g}, (mean - tc) / se = {(mean - tc) / se:.2f}")
    assert abs(mean - tc) <= 5 * se
    torch.cuda.synchronize()


def test_rejections(T):
    import torch
    net = W.triangle(8, seed=1, dtype=np.float32)
    spec = T.NetworkSpec.from_network(net, [torch.from_numpy(x).cuda() for x in net.data])
    for m in (512, 2048):
        with pytest.raises(T.TNError) as e:
            T.Plan([spec], T.TN_CYCLIC, m, 4, 1, flags=T.TN_FLAG_DFT_FP8)
        assert e.value.code == T.TN_ERR_UNSUPPORTED
    for extra in (T.TN_FLAG_PERSISTENT, T.TN_FLAG_DFT_BF16):
        with pytest.raises(T.TNError) as e:
            T.Plan([spec], T.TN_CYCLIC, 1024, 4, 1, flags=T.TN_FLAG_DFT_FP8 | extra)
        assert e.value.code == T.TN_ERR_UNSUPPORTED
    net64 = W.triangle(8, seed=1)
    spec64 = T.NetworkSpec.from_network(net64, [torch.from_numpy(x).cuda() for x in net64.data])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec64], T.TN_CYCLIC, 1024, 4, 1, flags=T.TN_FLAG_DFT_FP8)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
