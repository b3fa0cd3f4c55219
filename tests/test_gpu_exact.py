"""tn_contract_exact: the exact FP64 contraction (contraction tree by dynamic
programming over subsets, pairwise steps as matrix products on the FP64
matrix cores).

* Periodic lattices against the oracle's row transfer matrices (bond 2-6).
* Matrix products of ragged sizes in every operand layout, thin products
  (matrix-vector, inner products split along K), K-split tiles and permuted
  operands, against FP64 einsum on the host (the plain sum of Def. 1-3).
* The 4 x 4 torus at bond 16 (16^8-entry intermediates, 1.1e15 FLOP): rank-one
  tensors against the product of the inner products of the contracted vectors,
  and the Uniform[0,1) torus in two presentations (the lattice and its
  transpose, which contract along different trees and layouts) against each
  other.
"""
import time

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


def exact(T, net, dtype="float64"):
    import torch
    ts = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda", getattr(torch, dtype)) for x in net.data]
    view = net.with_data([t.double().cpu().numpy() for t in ts])
    return T.tn_contract_exact(T.NetworkSpec.from_network(net, ts)), view


def einsum_value(net):
    """Full contraction by numpy einsum (FP64), one letter per contraction."""
    import string
    letters = string.ascii_letters
    lab = {}
    for e, (u, v) in enumerate(net.edges):
        lab[u] = lab[v] = letters[e]
    off = np.concatenate([[0], np.cumsum(net.orders)])
    subs = ["".join(lab[u] for u in range(off[k], off[k + 1])) for k in range(net.p)]
    return float(np.einsum(",".join(subs) + "->", *[np.asarray(x, dtype=np.float64) for x in net.data],
                           optimize="greedy"))


@pytest.mark.parametrize("R,C,D,dtype,dist", [(4, 4, 4, "float64", "normal"), (3, 5, 3, "float32", "uniform"),
                                              (2, 3, 6, "float64", "normal"), (4, 1, 5, "float32", "normal"),
                                              (4, 4, 2, "bfloat16", "uniform")])
def test_torus_against_transfer_matrices(T, orc, R, C, D, dtype, dist):
    net = W.torus(L=R, D=D, cols=C, seed=3 + R + C, dtype=np.float64, dist=dist)
    got, view = exact(T, net, dtype)
    want = orc.tc_torus(view.data, R, C)
    scale = np.prod([np.abs(x).sum() for x in view.data])
    assert abs(got - want) <= 1e-13 * scale + 1e-12 * abs(want), (got, want)


def _mats(net_shapes, edges, seed):
    rng = np.random.default_rng(seed)
    data = [rng.standard_normal(s) for s in net_shapes]
    orders = [len(s) for s in net_shapes]
    dims = [n for s in net_shapes for n in s]
    return W.Network(orders, dims, edges, data, "custom")


CASES = {
    # tr(A B C), ragged tiles (200 x 150 output, K = 333)
    "tr_abc": ([(200, 333), (333, 150), (150, 200)], [(1, 2), (3, 4), (5, 0)]),
    # tr(A B): one inner product of 210000 terms, split along K
    "tr_ab": ([(300, 700), (700, 300)], [(1, 2), (3, 0)]),
    # x^T A B y: thin products (matrix-vector)
    "xaby": ([(1000,), (1000, 1500), (1500, 900), (900,)], [(0, 1), (2, 3), (4, 5)]),
    # long K with few tiles: the K split of the matrix-core product
    "long_k": ([(256, 8192), (8192, 256), (256, 256)], [(1, 2), (3, 4), (5, 0)]),
    # order-3 tensors whose contracted modes sit in the middle (permuted operands)
    "middle": ([(24, 40, 33), (33, 17, 40), (24, 17)], [(1, 5), (2, 3), (0, 6), (4, 7)]),
    # transposed operand layouts: A stored K x M against B stored N x K
    "layouts": ([(64, 150, 90), (90, 64, 150)], [(0, 4), (1, 5), (2, 3)]),
    # a tensor with a self-contraction (trace) joined to a ring
    "trace": ([(30, 30, 40), (40, 50), (50, 40, 40)], [(0, 1), (2, 3), (4, 5), (6, 7)]),
}


@pytest.mark.parametrize("case", list(CASES))
def test_products_against_einsum(T, case):
    shapes, edges = CASES[case]
    net = _mats(shapes, edges, seed=len(case))
    got, view = exact(T, net)
    want = einsum_value(view)
    scale = np.prod([np.abs(x).sum() for x in view.data])
    assert abs(got - want) <= 1e-13 * scale + 1e-12 * abs(want), (case, got, want)


def test_random_networks_against_einsum(T):
    for i in range(12):
        net = W.random_network(8, 100 + i, bmax=12, pmax=6)
        got, view = exact(T, net, "float32")
        want = einsum_value(view)
        scale = np.prod([np.abs(x).sum() for x in view.data])
        assert abs(got - want) <= 1e-13 * scale + 1e-12 * abs(want), (i, got, want)


def test_disconnected_components_multiply(T):
    a = _mats([(40, 50), (50, 40)], [(1, 2), (3, 0)], 1)
    b = _mats([(30,), (30,)], [(0, 1)], 2)
    net = W.Network(a.orders + b.orders, a.dims + b.dims,
                    a.edges + [(4, 5)], a.data + b.data, "two")
    got, view = exact(T, net)
    want = einsum_value(a) * float(b.data[0] @ b.data[1])
    assert got == pytest.approx(want, rel=1e-12)


def _free_cache():
    import torch
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_torus_d16_rank_one(T):
    """The bond-16 4 x 4 torus with rank-one tensors X = a (x) b (x) u (x) v
    (FP64): the exact value is the product of the 32 inner products."""
    _free_cache()
    R = C = 4
    D = 16
    rng = np.random.default_rng(11)
    vecs = [[rng.uniform(0.5, 1.5, D) for _ in range(4)] for _ in range(R * C)]
    net = W.torus(L=4, D=D, seed=1, dtype=np.float64)
    net = net.with_data([np.einsum("i,j,k,l->ijkl", *v) for v in vecs])
    want = 1.0
    for r in range(R):
        for c in range(C):
            a, b, u, v = vecs[r * C + c]
            want *= b @ vecs[r * C + (c + 1) % C][0]
            want *= v @ vecs[((r + 1) % R) * C + c][2]
    t0 = time.time()
    got, _ = exact(T, net)
    dt = time.time() - t0
    print(f"rank-one torus D=16: {got:.17g} vs {want:.17g}, {dt:.1f} s ({1.13e15 / dt / 1e12:.1f} TFLOP/s overall)")
    assert got == pytest.approx(want, rel=1e-12)
    _free_cache()


def test_torus_d16_uniform_two_presentations(T):
    """The benchmark torus (4 x 4, bond 16, FP32 Uniform[0,1)): its exact value
    and that of the transposed lattice (tensor (r, c) -> (c, r), modes
    (up, down, left, right)) agree; all terms are positive, so FP64 sums of
    1e15 products agree to about 1e-13."""
    _free_cache()
    net = W.torus(L=4, D=16, seed=2)
    z1, _ = exact(T, net, "float32")
    tr = [None] * 16
    for r in range(4):
        for c in range(4):
            tr[c * 4 + r] = np.ascontiguousarray(np.transpose(net.data[r * 4 + c], (2, 3, 0, 1)))
    z2, _ = exact(T, net.with_data(tr), "float32")
    print(f"torus 4x4 D=16 uniform: {z1:.17g} / {z2:.17g}")
    assert z1 > 0 and z2 == pytest.approx(z1, rel=1e-12)
    _free_cache()


def test_out_of_memory_refused_before_allocation(T):
    """The 4 x 4 torus at bond 24 needs 24^8-entry intermediates (0.9 TB in
    FP64): the dry run of the contraction tree finds the peak above the free
    device memory and the call returns TN_ERR_OOM before allocating any of it.
    A plan whose per-sample estimates would take 512 GB is refused with
    TN_ERR_OOM too (the failed allocation is returned, the rest released)."""
    import torch
    _free_cache()
    net = W.torus(L=4, D=24, seed=4)
    ts = [torch.from_numpy(x).cuda() for x in net.data]
    with pytest.raises(T.TNError) as e:
        T.tn_contract_exact(T.NetworkSpec.from_network(net, ts))
    assert e.value.code == T.TN_ERR_OOM and "GB of device memory" in str(e.value), str(e.value)
    tri = W.triangle(8, seed=1, dtype=np.float32)
    spec = T.NetworkSpec.from_network(tri, [torch.from_numpy(x).cuda() for x in tri.data])
    with pytest.raises(T.TNError) as e:
        T.Plan([spec], T.TN_CYCLIC, 64, 1 << 36, 1)
    assert e.value.code == T.TN_ERR_OOM, str(e.value)
    # the device is still usable
    plan = T.Plan([spec], T.TN_CYCLIC, 64, 16, 1)
    plan.estimate()
    torch.cuda.synchronize()
