"""Pins of the oracle's transfer-matrix contraction of periodic lattices
(Def. 1-3 on the torus): brute force over every index assignment on tiny
lattices, the all-ones closed form, and rank-one tensors, whose contraction
factors into one inner product per contraction."""
import numpy as np
import pytest

import tn_workloads as W


@pytest.mark.parametrize("R,C,D", [(2, 2, 2), (2, 3, 2), (3, 2, 3), (3, 3, 2), (1, 3, 3), (3, 1, 2)])
def test_torus_equals_brute_force(orc, R, C, D):
    net = W.torus(L=R, D=D, cols=C, seed=R * 10 + C, dtype=np.float64, dist="normal")
    assert orc.tc_torus(net.data, R, C) == pytest.approx(orc.tc_full(net), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("R,C,D", [(4, 4, 2), (3, 4, 3), (2, 5, 2)])
def test_torus_all_ones(orc, R, C, D):
    """Every index assignment of the 2 R C contractions contributes 1."""
    ones = [np.ones((D, D, D, D)) for _ in range(R * C)]
    assert orc.tc_torus(ones, R, C) == pytest.approx(float(D) ** (2 * R * C), rel=1e-13)


@pytest.mark.parametrize("R,C,D", [(4, 4, 4), (3, 5, 3), (2, 3, 5), (4, 1, 3)])
def test_torus_rank_one(orc, R, C, D):
    """X_(r,c) = a (x) b (x) u (x) v: the sum over all indices factors into
    prod over horizontal contractions <b_(r,c), a_(r,c+1)> times prod over
    vertical ones <v_(r,c), u_(r+1,c)>."""
    rng = np.random.default_rng(R * 100 + C * 10 + D)
    vecs = [[rng.standard_normal(D) for _ in range(4)] for _ in range(R * C)]
    tens = [np.einsum("i,j,k,l->ijkl", *v) for v in vecs]
    want = 1.0
    for r in range(R):
        for c in range(C):
            a, b, u, v = vecs[r * C + c]
            want *= b @ vecs[r * C + (c + 1) % C][0]
            want *= v @ vecs[((r + 1) % R) * C + c][2]
    assert orc.tc_torus(tens, R, C) == pytest.approx(want, rel=1e-11)


def test_torus_orientation(orc):
    """A lattice and its transpose (rows <-> columns, modes permuted to
    (up, down, left, right)) have the same contraction; a tensor with its
    left and right modes swapped (a plausible index mistake) does not."""
    R, C, D = 3, 2, 3
    net = W.torus(L=R, D=D, cols=C, seed=7, dtype=np.float64, dist="normal")
    z = orc.tc_torus(net.data, R, C)
    tr = [None] * (R * C)
    for r in range(R):
        for c in range(C):
            tr[c * R + r] = np.transpose(net.data[r * C + c], (2, 3, 0, 1))
    assert orc.tc_torus(tr, C, R) == pytest.approx(z, rel=1e-12)
    bad = list(net.data)
    bad[1] = np.transpose(bad[1], (1, 0, 2, 3))
    assert abs(orc.tc_torus(bad, R, C) - z) > 1e-6 * abs(z)
