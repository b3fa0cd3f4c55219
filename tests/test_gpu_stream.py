"""Turnstile streaming with resident sketches (TN_FLAG_RESIDENT) and the two
applications the paper derives from it: triangle counting (Cor. 3) and join
size (Cor. 2), on seeded synthetic streams.

The sketch is linear, so after any stream of updates a resident plan's
sketches must be those of the tensors the stream describes: per sample, the
combined estimate must match the oracle's Method-1 estimate on the final
dense tensors (at the same seed and sample) within tau * A_hat, with A_hat
taken over |X_0| plus the magnitudes of every update (the terms the float
atomics summed).  Count streams (integer updates, FP32 sketches) sum exactly.
The means over samples are compared with the exact triangle count / join size
within 5 standard errors."""
import numpy as np
import pytest

import tn_workloads as W
from test_gpu_m1 import TAU

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    return T


def resident(T, net, dtype, m, S, seed, data=None):
    import torch
    td = getattr(torch, dtype)
    src = data if data is not None else [np.zeros(net.shape(k)) for k in range(net.p)]
    ts = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda").to(td) for x in src]
    spec = T.NetworkSpec.from_network(net, ts)
    return T.Plan([spec], T.TN_CYCLIC, m, S, seed, flags=T.TN_FLAG_RESIDENT), ts


def feed(T, plan, stream, batch=8192, net=0):
    import torch
    for k in range(stream.net.p):
        sel = np.nonzero(stream.tensor == k)[0]
        for b0 in range(0, len(sel), batch):
            ii = sel[b0:b0 + batch]
            plan.update(k, torch.from_numpy(stream.index[ii]).cuda(), torch.from_numpy(stream.delta[ii]).cuda(),
                        net=net)


def combined(plan):
    import torch
    samples = torch.empty(plan.n_nets * plan.S, dtype=torch.float64, device="cuda")
    st = plan.combine(samples_out=samples)
    torch.cuda.synchronize()
    return st.cpu().numpy().reshape(-1, 2), samples.cpu().numpy().reshape(plan.n_nets, plan.S)


def check_parity(orc, net_final, net_abs, got, m, seed, samples, tau):
    for r in samples:
        o = orc.m1_estimate(net_final, m, seed, r, combine="dft", want_scale=False)
        a = orc.m1_estimate(net_abs, m, seed, r, combine="dft", want_scale=True)
        assert abs(got[r] - o["estimate"]) <= tau * a["scale"] + 1e-300, (r, got[r], o["estimate"])


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_updates_after_a_scan(T, orc, dtype):
    """Scan a random network (the initial tensors), stream random real-valued
    updates into two of its tensors (repeated indices, some outside the
    tensor, which are ignored), and combine: per sample the oracle's estimate
    of the updated tensors."""
    import torch
    net = W.random_network(4, 21, dtype=np.float64)
    m, S, seed = 256, 6, 3
    plan, _ = resident(T, net, dtype, m, S, seed, data=net.data)
    plan.estimate()
    rng = np.random.default_rng(5)
    final = [np.array(x, dtype=np.float64) for x in net.data]
    absx = [np.abs(x) for x in final]
    for k in (0, net.p - 1):
        size = final[k].size
        idx = rng.integers(-3, size + 3, 500)
        dl = rng.standard_normal(500)
        plan.update(k, torch.from_numpy(idx).cuda(), torch.from_numpy(dl).cuda())
        ok = (idx >= 0) & (idx < size)
        np.add.at(final[k].reshape(-1), idx[ok], dl[ok])
        np.add.at(absx[k].reshape(-1), idx[ok], np.abs(dl[ok]))
    if dtype == "float32":   # the scan read the FP32-rounded initial tensors
        for k in range(net.p):
            final[k] = final[k] - net.data[k] + net.data[k].astype(np.float32).astype(np.float64)
    _, got = combined(plan)
    check_parity(orc, net.with_data(final), net.with_data(absx), got[0], m, seed, range(S), TAU[dtype])


def test_reset_then_stream_equals_scan_of_final(T, orc):
    """From reset (all-zero sketches), a stream whose net effect is a random
    tensor network gives the same estimates (to rounding) as scanning that
    network's tensors."""
    import torch
    net = W.random_network(4, 8, dtype=np.float64)
    m, S, seed = 512, 4, 11
    plan, _ = resident(T, net, "float64", m, S, seed)
    plan.reset()
    rng = np.random.default_rng(1)
    for k in range(net.p):
        x = net.data[k].reshape(-1)
        idx = np.concatenate([np.arange(x.size), rng.integers(0, x.size, 200)])
        dl = np.concatenate([x, np.zeros(200)])
        dl[x.size:] = rng.standard_normal(200)
        dl = np.concatenate([dl, -dl[x.size:]])          # inserted, then deleted again
        idx = np.concatenate([idx, idx[x.size:]])
        plan.update(k, torch.from_numpy(idx).cuda(), torch.from_numpy(dl).cuda())
    _, got = combined(plan)
    scan, _ = resident(T, net, "float64", m, S, seed, data=net.data)
    samples = torch.empty(S, dtype=torch.float64, device="cuda")
    scan.estimate(samples_out=samples)
    ref = samples.cpu().numpy()
    scale = np.array([orc.m1_estimate(net.with_data([np.abs(x) * 3 for x in net.data]), m, seed, r,
                                      combine="dft", want_scale=True)["scale"] for r in range(S)])
    assert np.all(np.abs(got[0] - ref) <= 1e-12 * scale)


def test_triangle_count_from_edge_stream(T, orc):
    """Cor. 3: a directed graph of 1024 nodes streamed as ~37k edge insertions
    and deletions into X_1 = X_2 = X_3 = A; per-sample parity with the oracle
    on the final adjacency matrix, and the mean of 512 samples at m = 4096
    within 5 standard errors of tr(A^3)."""
    st = W.edge_stream(n=1024, edges=32768, triangles=512, deletions=4096, seed=7)
    final = st.dense()
    A = final.data[0]
    exact = float(np.trace(A @ A @ A))
    m, S, seed = 4096, 512, 2
    plan, _ = resident(T, st.net, "float32", m, S, seed)
    plan.reset()
    feed(T, plan, st)
    stats, got = combined(plan)
    absnet = final.with_data([np.abs(x) for x in final.data])
    check_parity(orc, final, absnet, got[0], m, seed, [0, 1, 255, 511], TAU["float32"])
    se = np.sqrt(stats[0, 1] / S)
    assert abs(stats[0, 0] - exact) <= 5 * se, (stats[0, 0], exact, se)


@pytest.mark.parametrize("kind", ["chain", "cycle", "star"])
def test_join_size_from_tuple_stream(T, orc, kind):
    """Cor. 2: Zipf(1.1) relations streamed tuple by tuple; the acyclic chain
    query and the cyclic triangle query over domains of 256, and the star
    query over 128 whose attribute a joins three relations through a copy
    tensor (WLOG 1), m = 4096, S = 256: per-sample parity with the oracle on
    the frequency tensors and the mean within 5 standard errors of the exact
    join size (for the star, also the plain sum over a, b of
    f1[a] f2[a] f3[a, b] f4[b], which needs no copy tensor)."""
    n = 128 if kind == "star" else 256
    st = W.join_stream(kind, n=n, tuples=20000, s=1.1, seed=9)
    final = st.dense()
    exact = orc.tc_full(final)
    if kind == "star":
        f1, f2, f3, f4, C = final.data
        assert np.count_nonzero(C) == n and np.all(np.einsum("iii->i", C) == 1.0)
        assert exact == pytest.approx(float((f1 * f2) @ f3 @ f4), rel=1e-12)
    m, S, seed = 4096, 256, 5
    plan, _ = resident(T, st.net, "float32", m, S, seed)
    plan.reset()
    feed(T, plan, st)
    stats, got = combined(plan)
    check_parity(orc, final, final, got[0], m, seed, [0, 100, 255], TAU["float32"])
    se = np.sqrt(stats[0, 1] / S)
    assert abs(stats[0, 0] - exact) <= 5 * se, (stats[0, 0], exact, se)


def test_updates_touch_only_their_network(T, orc):
    """Two networks in one resident plan: updating network 1 leaves network
    0's estimates bitwise unchanged; a plan without TN_FLAG_RESIDENT refuses
    updates."""
    import torch
    nets = [W.triangle(8, seed=1), W.ring(4, 6, seed=2)]
    specs = []
    for n in nets:
        ts = [torch.from_numpy(np.asarray(x, dtype=np.float64)).cuda() for x in n.data]
        specs.append(T.NetworkSpec.from_network(n, ts))
    plan = T.Plan(specs, T.TN_CYCLIC, 128, 5, 0, flags=T.TN_FLAG_RESIDENT)
    plan.estimate()
    before, _ = combined(plan)
    plan.update(0, torch.tensor([0, 5], device="cuda"), torch.tensor([1.0, -2.0], dtype=torch.float64,
                                                                      device="cuda"), net=1)
    after, _ = combined(plan)
    assert before[0, 0] == after[0, 0] and before[1, 0] != after[1, 0]
    plain = T.Plan(specs, T.TN_CYCLIC, 128, 5, 0)
    with pytest.raises(T.TNError) as e:
        plain.update(0, torch.tensor([0], device="cuda"), torch.tensor([1.0], dtype=torch.float64, device="cuda"))
    assert e.value.code == T.TN_ERR_ARG
