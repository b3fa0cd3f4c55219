"""GPU parity of the statistics entry points: tn_median_of_means (Theorem 1's
amplification) against the oracle's median_of_means, and tn_tensor_stats
(selector features) against FP64 sums of the values the device holds.

Bars: group means are FP64 sums in a different order from the oracle's, so the
median matches within 1e-13 of max |sample| (a few FP64 ulps of the partial
sums); the count of entries >= 0 is exact; the three sums match within 1e-12
relative for FP32/BF16 data (FP64 accumulation of exactly representable
values) and within 1e-12 of sum |x| for FP64.
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


@pytest.mark.parametrize("S,G", [(1, 1), (7, 3), (1000, 1), (1000, 7), (1000, 64), (1000, 1000),
                                 (4099, 1024), (65537, 9)])
def test_median_of_means_matches_oracle(T, orc, S, G):
    import torch
    rng = np.random.default_rng(S * 31 + G)
    x = rng.standard_t(2, size=(5, S)) * 10.0 + rng.standard_normal((5, 1))
    got = T.median_of_means(torch.from_numpy(x).cuda(), G).cpu().numpy()
    for j in range(5):
        ref = orc.median_of_means(x[j], G)
        assert abs(got[j] - ref) <= 1e-13 * np.abs(x[j]).max()


def test_median_of_means_on_plan_samples(T, orc):
    import torch
    net = W.triangle(16, seed=3, dtype=np.float64)
    ts = [torch.from_numpy(a).cuda() for a in net.data]
    spec = T.NetworkSpec.from_network(net, ts)
    plan = T.Plan([spec], T.TN_CYCLIC, 64, 96, 11)
    samples = torch.empty(96, dtype=torch.float64, device="cuda")
    plan.estimate(samples_out=samples)
    med = T.median_of_means(samples.view(1, 96), 8).cpu().numpy()[0]
    ref = orc.median_of_means(samples.cpu().numpy(), 8)
    assert abs(med - ref) <= 1e-13 * np.abs(samples.cpu().numpy()).max()


def test_median_of_means_nan_and_errors(T):
    import torch
    x = torch.zeros((2, 10), dtype=torch.float64, device="cuda")
    x[1, 3] = float("nan")
    out = T.median_of_means(x, 5).cpu().numpy()
    assert out[0] == 0.0 and np.isnan(out[1])
    with pytest.raises(T.TNError):
        T.median_of_means(x, 11)
    with pytest.raises(T.TNError):
        T.median_of_means(x, 0)


@pytest.mark.parametrize("dtype", ["float64", "float32", "bfloat16"])
def test_tensor_stats_matches_host(T, dtype):
    import torch
    nets = [W.torus(L=2, D=5, seed=3, dist="normal"), W.ring(4, 33, seed=4, dtype=np.float32),
            W.random_network(4, 7)]
    td = getattr(torch, dtype)
    specs, held = [], []
    for n in nets:
        ts = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda().to(td) for a in n.data]
        specs.append(T.NetworkSpec.from_network(n, ts))
        held += [t.double().cpu().numpy().ravel() for t in ts]
    got = T.tn_tensor_stats(specs)
    assert got.shape == (len(held), 4)
    for k, a in enumerate(held):
        assert got[k, 3] == float(np.count_nonzero(a >= 0))
        sa = float(np.abs(a).sum())
        assert abs(got[k, 0] - a.sum()) <= 1e-12 * sa
        assert abs(got[k, 1] - float((a * a).sum())) <= 1e-12 * float((a * a).sum())
        assert abs(got[k, 2] - sa) <= 1e-12 * sa
