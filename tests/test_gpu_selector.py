"""The learned sketch-size selector against the pilot-sample fallback.

The selector is trained here from scratch: variance data from the library's
estimator on 6000 networks of the ring / torus / caterpillar / random families
(K = 64 samples per (network, m)), the regressor trained by the library's MLP
kernels.  Both selectors then pick (m, S) for input-relative error 1e-2 at
z = 2 on held-out networks (unseen seeds and sizes, and networks of the
batched random workload), the picks are run with fresh seeds and judged against
the library's exact contraction.  Every step is deterministic for fixed seeds
(fixed-point scatter, fixed-order reductions).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def trained():
    import torch
    import paper_2603_07387_amd as T
    from paper_2603_07387_amd import selector as S
    assert torch.cuda.is_available()
    T.load()
    measured = S.measure_variances(S.family_networks(6000, 41), K=64, seed=41)
    X, y, idx = S.dataset(measured)
    sel = S.Selector(64, seed=41)
    losses = sel.fit(X, y, groups=idx, epochs=400, lr=2e-3, seed=41)
    return sel, X, y, losses


def test_variance_data_and_fit(trained):
    from paper_2603_07387_amd import selector as S
    sel, X, y, losses = trained
    assert X.shape[1] == S.D_IN and len(y) > 40000
    assert np.all((y >= S.LOGV_FLOOR) & (y <= S.LOGV_CEIL))
    assert losses[-1] < 0.05 * losses[0]
    rmse = float(np.sqrt(np.mean((sel.predict(X, raw=True) - y) ** 2)))
    assert rmse < 0.25 * float(np.std(y))
    # the calibration margin is a small positive shift that covers most labels
    assert 0.0 < sel.margin < 3.0
    assert np.mean(sel.predict(X) >= y) > 0.8


def test_labels_follow_the_one_over_m_law(trained):
    """Lemma 6 / Lemma 2: v(m) m does not grow with m, so the fitted labels of
    one network fall by about a factor 2 per doubling of m at large m."""
    from paper_2603_07387_amd import selector as S
    import tn_workloads as W
    net = S._unit(W.ring(3, 64, seed=5, dtype=np.float32, dist="normal"))
    (light, method, stats, v), = S.measure_variances([(net, "cyclic")], K=256, seed=3)
    lab = S.envelope_labels(v)
    ms = sorted(lab)
    for a, b in zip(ms, ms[1:]):
        assert lab[b] <= lab[a] - math.log(2.0) + 1e-9 or lab[a] in (S.LOGV_FLOOR, S.LOGV_CEIL)
    # and the measured slope at large m is close to -1 in log-log
    slope = (math.log(v[16384]) - math.log(v[1024])) / math.log(16.0)
    assert -1.35 < slope < -0.65


def test_save_load_roundtrip(trained, tmp_path):
    from paper_2603_07387_amd import selector as S
    sel, X, _, _ = trained
    path = tmp_path / "sel.npz"
    sel.save(path)
    sel2 = S.Selector.load(path)
    np.testing.assert_array_equal(sel.predict(X[:500]), sel2.predict(X[:500]))


def test_learned_beats_pilot(trained):
    from paper_2603_07387_amd import selector as S
    sel = trained[0]
    batch = S.evaluate(sel, S.batch_networks(60, start=1000))
    fams = S.evaluate(sel, S.family_networks(60, 43, held_out=True))
    sb, sf, sa = S.summarize(batch), S.summarize(fams), S.summarize(batch + fams)
    print("batch", sb)
    print("families", sf)
    # on the batched workload: at least the pilot's hit rate for less work
    assert sb["networks"] >= 40
    assert sb["hit_rate_learned"] >= sb["hit_rate_pilot"]
    assert sb["hit_rate_learned"] >= 0.9
    assert sb["work_learned"] < sb["work_pilot"]
    # over everything held out: a higher hit rate
    assert sa["hit_rate_learned"] >= sa["hit_rate_pilot"]
