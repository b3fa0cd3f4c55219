"""The library's sizing on the GPU: the regressor file (tn_mlp_save /
tn_mlp_load), the learned and pilot choices of tn_sketch_size against the
Python selector's (selector.choose, selector.pilot_choose) on the same inputs,
and tn_sketch_plan with m <= 0."""
import zlib

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


def specs_of(T, nets):
    import torch
    out = []
    for n in nets:
        ts = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda() for x in n.data]
        out.append(T.NetworkSpec.from_network(n, ts))
    return out


def test_mlp_file_roundtrip_and_crc(T, tmp_path):
    import torch
    net = T.MLP(32, 64, seed=3)
    path = str(tmp_path / "reg.tnmlp")
    net.save(path, [1.5, -2.25, 0.125])
    raw = open(path, "rb").read()
    assert raw[:8] == b"TNMLP\0\0\1"
    assert int.from_bytes(raw[-4:], "little") == zlib.crc32(raw[:-4])      # the file's CRC-32
    net2, meta = T.MLP.load(path)
    assert meta == [1.5, -2.25, 0.125] and (net2.d_in, net2.hidden) == (32, 64)
    np.testing.assert_array_equal(net.params(), net2.params())
    X = torch.randn(100, 32, device="cuda")
    assert torch.equal(net.predict(X), net2.predict(X))
    bad = bytearray(raw)
    bad[40] ^= 1
    open(path, "wb").write(bytes(bad))
    with pytest.raises(T.TNError) as e:
        T.MLP.load(path)
    assert e.value.code == T.TN_ERR_ARG and "CRC" in str(e.value)
    open(path, "wb").write(raw[:-8])
    with pytest.raises(T.TNError):
        T.MLP.load(path)


def _selector(T, seed=7):
    """An untrained selector (random weights, spread-out predictions): the C
    and Python choices must agree on whatever it predicts."""
    from paper_2603_07387_amd import selector as S
    sel = S.Selector(64, seed=seed)
    sel.mu, sel.sd, sel.margin = -6.0, 3.0, 0.5
    return sel


def test_learned_choice_matches_python_selector(T):
    from paper_2603_07387_amd import selector as S
    sel = _selector(T)
    sel.register()
    pairs = S.family_networks(40, 5, held_out=True) + S.batch_networks(10, start=200)
    for eps, z in ((1e-2, 2.0), (3e-2, 1.5), (1e-3, 3.0)):
        agree = 0
        for net, method in pairs:
            spec = specs_of(T, [net])
            meth = T.TN_CYCLIC if method == "cyclic" else T.TN_ACYCLIC
            c = T.tn_sketch_size(spec, meth, eps, 1.0 / z ** 2, mode=T.TN_SIZE_LEARNED)[0]
            st = S.stats_of(spec)[0]
            m, Sn, w = sel.choose(net, st, method, eps, z)
            agree += (c["m"], c["samples"]) == (m, Sn)
            assert c["groups"] == 1
        # features are the same float32 values up to libm rounding: a choice at an
        # exact tie of two sizes may differ; nearly all must agree
        assert agree >= len(pairs) - 1, (eps, agree)
    T.tn_set_size_selector(None, 0.0, 1.0, 0.0)


def test_pilot_choice_matches_python_pilot(T):
    from paper_2603_07387_amd import selector as S
    for i, (net, method) in enumerate(S.family_networks(12, 9, held_out=True)):
        spec = specs_of(T, [net])
        meth = T.TN_CYCLIC if method == "cyclic" else T.TN_ACYCLIC
        c = T.tn_sketch_size(spec, meth, 1e-2, 0.25, mode=T.TN_SIZE_PILOT, seed=100 + i)[0]
        norm = float(np.sqrt(np.prod(S.stats_of(spec)[0][:, 1])))
        (m, Sn, w), _ = S.pilot_choose(spec, net, method, norm, 1e-2, 2.0, seed=100 + i)
        assert (c["m"], c["samples"]) == (m, Sn), (i, c, m, Sn)


def test_plan_chooses_its_size(T):
    """tn_sketch_plan with m <= 0: the pilot (and, registered, the learned) size
    of tn_sketch_size at the plan's target; with S given, the least m whose
    bound meets it."""
    import torch
    net = W.triangle(32, seed=4, dtype=np.float32)
    spec = specs_of(T, [net])
    T.tn_set_size_target(1e-2, 0.25)
    c = T.tn_sketch_size(spec, T.TN_CYCLIC, 1e-2, 0.25, mode=T.TN_SIZE_PILOT, seed=9)[0]
    plan = T.Plan(spec, T.TN_CYCLIC, 0, 0, 9, flags=T.TN_FLAG_SIZE_PILOT)
    assert (plan.query(3), plan.query(2)) == (c["m"], c["samples"])
    stats = plan.estimate()
    torch.cuda.synchronize()
    # bound with a given S: v(m) = 27 / m must meet v / S <= delta eps^2
    S = 4096
    plan2 = T.Plan(spec, T.TN_CYCLIC, 0, S, 1)
    m2 = plan2.query(3)
    assert plan2.query(2) == S and 27.0 / m2 / S <= 0.25 * 1e-4 and (m2 == 64 or 27.0 / (m2 / 2) / S > 0.25e-4)
    sel = _selector(T)
    sel.register()
    cl = T.tn_sketch_size(spec, T.TN_CYCLIC, 1e-2, 0.25, mode=T.TN_SIZE_LEARNED)[0]
    plan3 = T.Plan(spec, T.TN_CYCLIC, -1, 0, 2, flags=T.TN_FLAG_SIZE_LEARNED)
    assert (plan3.query(3), plan3.query(2)) == (cl["m"], cl["samples"])
    T.tn_set_size_selector(None, 0.0, 1.0, 0.0)
    with pytest.raises(T.TNError) as e:   # learned sizing without a regressor
        T.Plan(spec, T.TN_CYCLIC, 0, 0, 2, flags=T.TN_FLAG_SIZE_LEARNED)
    assert e.value.code == T.TN_ERR_ARG
