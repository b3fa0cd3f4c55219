"""Host logic of the sketch-size selector: labels, features and the choice of
(m, S).  No GPU calls."""
import math

import numpy as np
import pytest

from paper_2603_07387_amd import selector as S


def _host_stats(net):
    return np.array([[float(x.astype(np.float64).sum()), float((x.astype(np.float64) ** 2).sum()),
                      float(np.abs(x.astype(np.float64)).sum()), float((x >= 0).sum())]
                     for x in net.data])


def test_envelope_labels():
    v = {64: 0.01, 128: 0.5, 256: 0.1, 512: float("nan"), 1024: 0.01}
    lab = {m: math.exp(x) for m, x in S.envelope_labels(v).items()}
    assert set(lab) == {64, 128, 256, 1024}
    assert lab[1024] == pytest.approx(0.01)
    assert lab[256] == pytest.approx(0.1)              # above 0.01 * 1024 / 256
    assert lab[128] == pytest.approx(0.5)
    assert lab[64] == pytest.approx(1.0)               # raised to 0.5 * 128 / 64
    # clipping
    lab = S.envelope_labels({64: 1e-30, 128: 1e30})
    assert lab[128] == S.LOGV_CEIL and lab[64] == S.LOGV_CEIL
    assert S.envelope_labels({64: 1e-30})[64] == S.LOGV_FLOOR


def test_features_finite_and_scale_free():
    import tn_workloads as W
    pairs = S.family_networks(40, 5) + S.batch_networks(3)
    for net, method in pairs:
        st = _host_stats(net)
        for m in S.LADDER[method]:
            f = S.features(net, st, method, m)
            assert f.shape == (S.D_IN,) and np.all(np.isfinite(f))
    # features do not change when a tensor is scaled
    net = W.torus(L=2, D=4, seed=1, dist="uniform")
    scaled = net.with_data([x * np.float32(3.0 ** k) for k, x in enumerate(net.data)])
    np.testing.assert_allclose(S.features(net, _host_stats(net), "cyclic", 256),
                               S.features(scaled, _host_stats(scaled), "cyclic", 256), rtol=1e-5, atol=1e-6)


def test_family_networks_unit_norm_and_seeded():
    a = S.family_networks(12, 3)
    b = S.family_networks(12, 3)
    for (na, ma), (nb, mb) in zip(a, b):
        assert ma == mb and na.name == nb.name
        for x, y in zip(na.data, nb.data):
            assert np.array_equal(x, y)
            assert np.linalg.norm(x.astype(np.float64)) == pytest.approx(1.0, rel=1e-5)


def test_choose_minimizes_work_under_target():
    import tn_workloads as W
    net = W.ring(3, 64, seed=0)
    # v(m) = 2 / m: S(m) = ceil(4 * 2 / (m * 1e-4)); work = S (q N + p m log2 m)
    logv = {m: math.log(2.0 / m) for m in S.LADDER["cyclic"]}
    m, Sm, w = S.choose(net, "cyclic", logv, eps=1e-2, z=2.0)
    best = min(S.LADDER["cyclic"], key=lambda k: math.ceil(8e4 / k) * S.work_per_sample(net, "cyclic", k))
    assert m == best and Sm == math.ceil(8e4 / m)
    assert w == pytest.approx(Sm * S.work_per_sample(net, "cyclic", m))
    # the chosen (m, S) meets the target
    assert 2.0 * math.sqrt(2.0 / m / Sm) <= 1e-2


def test_choose_infeasible_falls_back_to_least_variance():
    import tn_workloads as W
    net = W.ring(3, 64, seed=0)
    logv = {m: 30.0 - 0.1 * math.log2(m) for m in S.LADDER["cyclic"]}
    m, Sm, _ = S.choose(net, "cyclic", logv, max_samples=1000)
    assert m == S.LADDER["cyclic"][-1] and Sm == 1000
    # tiny variance: one sample at the cheapest size
    m, Sm, _ = S.choose(net, "cyclic", {k: -50.0 for k in S.LADDER["cyclic"]})
    assert Sm == 1 and m == S.LADDER["cyclic"][0]
