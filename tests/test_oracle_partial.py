"""CPU pins for the partial-TNC checks (Corollary 1).

The GPU's partial plan estimates entry r of the output tensor by Eq. (1) on
the full TNC of the sub-tensors X_k(s_k) that fix every free mode at r's
index (the corollary's proof).  The tests build that sub-network with plain
numpy indexing (`entry_network`) and run the oracle's Method 1 on it.  Pinned
here: for every entry, the exact contraction of the sub-network equals Def. 1
read literally on the whole partial network (Example 1's network, whose
printed formula test_oracle.py already pins), and the entry order is
row-major over the free modes in increasing mode order.
"""
import itertools

import numpy as np
import pytest

import tn_workloads as W


def free_modes(net):
    used = {u for e in net.edges for u in e}
    return [u for u in range(net.q) if u not in used]


def entry_network(net, r):
    """The full network of entry r (row-major over the free modes in
    increasing mode order): each tensor with its free modes fixed at r's
    indices; contractions kept in their order and orientation, modes
    renumbered."""
    fm = free_modes(net)
    idx = dict(zip(fm, np.unravel_index(r, [net.dims[u] for u in fm]))) if fm else {}
    orders, dims, data, newid = [], [], [], {}
    for k in range(net.p):
        x = np.asarray(net.data[k])
        sel = tuple(int(idx[u]) if u in idx else slice(None) for u in net.modes(k))
        x = np.ascontiguousarray(x[sel])
        kept = [u for u in net.modes(k) if u not in idx]
        for u in kept:
            newid[u] = len(dims)
            dims.append(net.dims[u])
        orders.append(len(kept))
        data.append(x)
    edges = [(newid[u], newid[v]) for (u, v) in net.edges]
    return W.Network(orders, dims, edges, data)


def test_entry_networks_reproduce_def1(orc):
    net = W.example1()
    fm = free_modes(net)
    assert fm == [1, 7]
    lit = orc.tc_literal(net)                        # shape (n2, n8)
    assert lit.shape == (net.dims[1], net.dims[7])
    for r, (i2, i8) in enumerate(itertools.product(range(net.dims[1]), range(net.dims[7]))):
        sub = entry_network(net, r)
        assert sub.p == 4 and sub.t == 3 and sub.orders == [1, 1, 3, 1]
        assert orc.tc_full(sub) == pytest.approx(lit[i2, i8], rel=1e-12, abs=1e-12)


def test_entry_order_with_three_free_modes(orc):
    rng = np.random.default_rng(2)
    net = W.Network([3, 2], [2, 3, 4, 3, 5], [(1, 3)],
                    [rng.standard_normal((2, 3, 4)), rng.standard_normal((3, 5))])
    lit = orc.tc_literal(net)                        # free modes 0, 2, 4
    assert lit.shape == (2, 4, 5)
    flat = lit.reshape(-1)
    for r in range(flat.size):
        assert orc.tc_full(entry_network(net, r)) == pytest.approx(flat[r], rel=1e-12, abs=1e-12)
