"""Seeded synthetic tensor networks, shared by the FP64 oracle and the HIP path.

This module holds network *structure* and *data* only: which tensors exist,
their mode sizes, which mode pairs are contracted, and seeded entries.  It
contains none of the estimator's arithmetic (no hashing, sketching, DFT or
contraction), so the oracle and the GPU path can both take their inputs from
here without sharing any method code.

Conventions (paper, Preliminaries and Def. 1-3):
  * a network is ``tc(X_1 x ... x X_p, E)``: tensor ``k`` has order ``q_k``
    and owns the consecutive global modes ``off_k .. off_k + q_k - 1``;
  * ``dims[u]`` is the size ``n_u`` of global mode ``u``;
  * ``edges`` lists contracted pairs ``(u, v)`` of 0-based global modes
    (the paper numbers modes from 1); the first element of a pair is the mode
    that receives the count sketch ``C_u`` in the cyclic method, the second
    gets its complement;
  * tensor data are row-major arrays (``vec`` is lexicographic order).

Random entries come from numpy's PCG64 generator, seeded per workload (and per
network for batches), so any subset can be regenerated on its own.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Network", "triangle", "torus", "tt_caterpillar", "tt_ladder", "ring",
    "chain", "example1", "example5", "random_network", "random_batch",
    "batch_stats", "fill",
]


class Network:
    """A tensor network ``tc(X_1 x ... x X_p, E)`` with its data."""

    def __init__(self, orders, dims, edges, data=None, name=""):
        self.orders = [int(q) for q in orders]
        self.dims = [int(n) for n in dims]
        self.edges = [(int(u), int(v)) for (u, v) in edges]
        self.name = name
        if sum(self.orders) != len(self.dims):
            raise ValueError("sum of orders must equal the number of modes")
        self.offsets = np.concatenate([[0], np.cumsum(self.orders)]).astype(int).tolist()
        self.data = list(data) if data is not None else None
        if self.data is not None:
            if len(self.data) != self.p:
                raise ValueError("one array per tensor is required")
            for k, x in enumerate(self.data):
                if tuple(x.shape) != self.shape(k):
                    raise ValueError(f"tensor {k}: shape {x.shape} != {self.shape(k)}")

    @property
    def p(self):
        return len(self.orders)

    @property
    def t(self):
        return len(self.edges)

    @property
    def q(self):
        return len(self.dims)

    def modes(self, k):
        return list(range(self.offsets[k], self.offsets[k + 1]))

    def shape(self, k):
        return tuple(self.dims[u] for u in self.modes(k))

    def tensor_of(self, u):
        for k in range(self.p):
            if self.offsets[k] <= u < self.offsets[k + 1]:
                return k
        raise IndexError(u)

    def nnz(self):
        return int(sum(int(np.prod(self.shape(k))) for k in range(self.p)))

    def astype(self, dtype):
        return Network(self.orders, self.dims, self.edges,
                       [np.ascontiguousarray(x, dtype=dtype) for x in self.data], self.name)

    def with_data(self, data):
        return Network(self.orders, self.dims, self.edges, data, self.name)

    def fro_norms(self):
        return [float(np.sqrt(np.sum(np.asarray(x, dtype=np.float64) ** 2))) for x in self.data]

    def input_norm(self):
        """prod_k ||X_k||_F, the scale of the (eps, delta) guarantee (Def. 4)."""
        return float(np.prod(self.fro_norms()))

    def __repr__(self):
        return f"Network({self.name!r}, p={self.p}, t={self.t}, nnz={self.nnz()})"


def fill(shape, rng, dist="normal", dtype=np.float32, scale=1.0):
    """Seeded entries: 'normal' N(0, scale^2), 'uniform' U[0,1), 'ones', 'lowrank'
    (a sum of two outer products of positive vectors), 'int' small integers."""
    shape = tuple(shape)
    if dist == "normal":
        x = rng.standard_normal(shape) * scale
    elif dist == "uniform":
        x = rng.random(shape)
    elif dist == "ones":
        x = np.ones(shape)
    elif dist == "int":
        x = rng.integers(-3, 4, size=shape).astype(np.float64)
    elif dist == "lowrank":
        x = np.zeros(shape)
        for _ in range(2):
            term = np.ones(())
            for n in shape:
                term = np.multiply.outer(term, rng.random(n) + 0.5)
            x = x + term
    else:
        raise ValueError(dist)
    return np.ascontiguousarray(x, dtype=dtype)


def _mk(shapes, edges, rng, dist, dtype, name, scale=1.0):
    orders = [len(s) for s in shapes]
    dims = [n for s in shapes for n in s]
    data = [fill(s, rng, dist, dtype, scale) for s in shapes]
    return Network(orders, dims, edges, data, name)


def triangle(n=64, seed=1, dtype=np.float64, dist="normal"):
    """Cyclic triangle tr(ABC): A, B, C in R^{n x n}; edges are the 0-based form of
    the paper's {(2,3),(4,5),(1,6)} (Example 4, and Cor. 3's triangle count)."""
    rng = np.random.default_rng(seed)
    return _mk([(n, n)] * 3, [(1, 2), (3, 4), (0, 5)], rng, dist, dtype, f"triangle{n}")


def ring(p, n, seed=0, dtype=np.float64, dist="normal"):
    """Cycle of p matrices: tr(X_1 X_2 ... X_p)."""
    rng = np.random.default_rng(seed)
    edges = [(2 * k + 1, 2 * ((k + 1) % p)) for k in range(p)]
    return _mk([(n, n)] * p, edges, rng, dist, dtype, f"ring{p}x{n}")


def chain(lengths, seed=0, dtype=np.float64, dist="normal"):
    """Acyclic chain v_0 - M_1 - ... - M_{L} - v_{L+1}: a vector, matrices, a vector.
    ``lengths`` gives the bond sizes n_0..n_L."""
    rng = np.random.default_rng(seed)
    shapes = [(lengths[0],)] + [(lengths[i], lengths[i + 1]) for i in range(len(lengths) - 1)] + [(lengths[-1],)]
    edges = []
    mode = 0
    for k in range(len(shapes) - 1):
        last = mode + len(shapes[k]) - 1
        edges.append((last, last + 1))
        mode += len(shapes[k])
    return _mk(shapes, edges, rng, dist, dtype, f"chain{len(shapes)}")


def torus(L=4, D=16, seed=2, dtype=np.float32, dist="uniform", cols=None):
    """L x cols (default L x L) periodic lattice of order-4 tensors (modes: left,
    right, up, down), bond dimension D, tensor (r, c) at index r cols + c;
    right(r,c)-left(r,c+1) and down(r,c)-up(r+1,c) are contracted."""
    C = L if cols is None else cols
    rng = np.random.default_rng(seed)
    shapes, edges = [], []
    idx = lambda r, c: (r % L) * C + (c % C)
    for r in range(L):
        for c in range(C):
            shapes.append((D, D, D, D))
    for r in range(L):
        for c in range(C):
            k = idx(r, c)
            edges.append((4 * k + 1, 4 * idx(r, c + 1) + 0))
            edges.append((4 * k + 3, 4 * idx(r + 1, c) + 2))
    return _mk(shapes, edges, rng, dist, dtype, f"torus{L}x{C}D{D}")


def tt_caterpillar(cores=32, bond=64, phys=64, seed=3, dtype=np.float32):
    """Acyclic reading of the two-tensor-train inner product: one TT of ``cores``
    cores (phys,bond), (bond,phys,bond)..., (bond,phys) whose physical legs are
    contracted with vectors v_k (a bond-1 tensor train).  Entries N(0, 1/64).
    Tensors 0..cores-1 are the cores, cores..2*cores-1 the vectors."""
    rng = np.random.default_rng(seed)
    sd = 1.0 / 8.0
    shapes = [(phys, bond)] + [(bond, phys, bond)] * (cores - 2) + [(bond, phys)]
    shapes += [(phys,)] * cores
    offs = np.concatenate([[0], np.cumsum([len(s) for s in shapes])]).astype(int)
    edges = []
    # bonds between consecutive cores
    edges.append((offs[0] + 1, offs[1] + 0))
    for k in range(1, cores - 1):
        edges.append((offs[k] + 2, offs[k + 1] + 0))
    # physical legs with the vectors
    edges.append((offs[0] + 0, offs[cores] + 0))
    for k in range(1, cores - 1):
        edges.append((offs[k] + 1, offs[cores + k] + 0))
    edges.append((offs[cores - 1] + 1, offs[2 * cores - 1] + 0))
    data = [fill(s, rng, "normal", dtype, sd) for s in shapes]
    orders = [len(s) for s in shapes]
    dims = [n for s in shapes for n in s]
    return Network(orders, dims, edges, data, f"ttcat{cores}b{bond}p{phys}")


def tt_ladder(cores=32, bond=64, phys=64, seed=3, dtype=np.float32):
    """Literal inner product of two tensor trains (a cyclic ladder): cores
    A_k, B_k with boundary bonds 1 dropped; A_k.phys-B_k.phys and the bond
    chains are contracted.  Entries N(0, 1/64)."""
    rng = np.random.default_rng(seed)
    sd = 1.0 / 8.0
    one = [(phys, bond)] + [(bond, phys, bond)] * (cores - 2) + [(bond, phys)]
    shapes = one + one
    offs = np.concatenate([[0], np.cumsum([len(s) for s in shapes])]).astype(int)
    edges = []
    for base in (0, cores):
        edges.append((offs[base] + 1, offs[base + 1] + 0))
        for k in range(1, cores - 1):
            edges.append((offs[base + k] + 2, offs[base + k + 1] + 0))
    pm = lambda k: 0 if k == 0 else 1
    for k in range(cores):
        edges.append((offs[k] + pm(k), offs[cores + k] + pm(k)))
    data = [fill(s, rng, "normal", dtype, sd) for s in shapes]
    orders = [len(s) for s in shapes]
    dims = [n for s in shapes for n in s]
    return Network(orders, dims, edges, data, f"ttladder{cores}b{bond}p{phys}")


def example1(n=(2, 3, 4, 4, 2, 3, 3, 2), seed=11, dtype=np.float64, dist="int"):
    """The partial TNC of Example 1 / Fig. 1: X1(n1), X2(n2,n3), X3(n4,n5,n6),
    X4(n7,n8), E = {(1,5),(3,4),(6,7)} (1-based) -> free modes 2 and 8."""
    rng = np.random.default_rng(seed)
    shapes = [(n[0],), (n[1], n[2]), (n[3], n[4], n[5]), (n[6], n[7])]
    return _mk(shapes, [(0, 4), (2, 3), (5, 6)], rng, dist, dtype, "example1")


def example5(n=4, seed=12, dtype=np.float64, dist="normal"):
    """The acyclic network of Example 5 / Fig. 3: X1, X2 in R^{n x n x n},
    X4 in R^{n x n}, X3, X5, X6, X7 in R^n, E = {(1,4),(2,7),(3,8),(5,10),(6,11),(9,12)}."""
    rng = np.random.default_rng(seed)
    shapes = [(n, n, n), (n, n, n), (n,), (n, n), (n,), (n,), (n,)]
    edges = [(0, 3), (1, 6), (2, 7), (4, 9), (5, 10), (8, 11)]
    return _mk(shapes, edges, rng, dist, dtype, "example5")


def _random_structure(rng, pmin=3, pmax=12, bmin=2, bmax=32, maxdeg=4, max_entries=1 << 18):
    """Random connected network with at least one cycle: a random recursive
    spanning tree plus U{1..floor(p/2)} extra non-parallel edges, degree <= maxdeg,
    bond sizes U{bmin..bmax}; resampled until every tensor has <= max_entries."""
    while True:
        p = int(rng.integers(pmin, pmax + 1))
        adj = []          # (a, b) tensor pairs
        deg = [0] * p
        for i in range(1, p):
            cands = [j for j in range(i) if deg[j] < maxdeg]
            j = int(cands[int(rng.integers(len(cands)))])
            adj.append((j, i))
            deg[i] += 1
            deg[j] += 1
        extra = int(rng.integers(1, p // 2 + 1))
        pairs = set((min(a, b), max(a, b)) for a, b in adj)
        tries = 0
        while extra > 0 and tries < 200:
            tries += 1
            a, b = int(rng.integers(p)), int(rng.integers(p))
            if a == b or deg[a] >= maxdeg or deg[b] >= maxdeg:
                continue
            key = (min(a, b), max(a, b))
            if key in pairs:
                continue
            pairs.add(key)
            adj.append((a, b))
            deg[a] += 1
            deg[b] += 1
            extra -= 1
        if extra > 0:
            continue
        bonds = [int(rng.integers(bmin, bmax + 1)) for _ in adj]
        tmodes = [[] for _ in range(p)]   # per tensor: list of (edge idx, side)
        for e, (a, b) in enumerate(adj):
            tmodes[a].append((e, 0))
            tmodes[b].append((e, 1))
        sizes = [int(np.prod([bonds[e] for e, _ in tm])) for tm in tmodes]
        if max(sizes) > max_entries:
            continue
        return p, adj, bonds, tmodes


def random_network(seed, index=0, dtype=np.float32, dist="normal", **kw):
    """Network ``index`` of the batched workload: structure and data drawn from a
    generator seeded with (seed, index), so any subset can be rebuilt alone."""
    rng = np.random.default_rng([int(seed), int(index)])
    p, adj, bonds, tmodes = _random_structure(rng, **kw)
    orders = [len(tm) for tm in tmodes]
    offs = np.concatenate([[0], np.cumsum(orders)]).astype(int)
    dims = []
    where = {}
    for k, tm in enumerate(tmodes):
        for j, (e, side) in enumerate(tm):
            dims.append(bonds[e])
            where[(e, side)] = offs[k] + j
    edges = [(where[(e, 0)], where[(e, 1)]) for e in range(len(adj))]
    shapes = [tuple(bonds[e] for e, _ in tm) for tm in tmodes]
    data = [fill(s, rng, dist, dtype) for s in shapes]
    return Network(orders, dims, edges, data, f"rand{seed}_{index}")


def random_batch(count=4096, seed=4, dtype=np.float32, dist="normal", start=0, **kw):
    """The batched workload: ``count`` random connected cyclic networks."""
    return [random_network(seed, i, dtype, dist, **kw) for i in range(start, start + count)]


def batch_stats(nets):
    return {
        "networks": len(nets),
        "tensors": int(sum(n.p for n in nets)),
        "entries": int(sum(n.nnz() for n in nets)),
        "mean_p": float(np.mean([n.p for n in nets])),
        "mean_t": float(np.mean([n.t for n in nets])),
    }


# ----------------------------------------------------------------------------
# Streams for the turnstile setting and the two applications (join size,
# triangle counting).  Seeded and synthetic; they hold no estimator arithmetic.
# ----------------------------------------------------------------------------

class Stream:
    """A turnstile stream over a network's tensors: update u adds delta[u] to
    entry index[u] (row-major) of tensor tensor[u].  dense() applies it to
    zero tensors (the tensors the stream describes)."""

    def __init__(self, net, tensor, index, delta, name=""):
        self.net = net                      # structure (data unused)
        self.tensor = np.asarray(tensor, dtype=np.int32)
        self.index = np.asarray(index, dtype=np.int64)
        self.delta = np.asarray(delta, dtype=np.float64)
        self.name = name

    def __len__(self):
        return len(self.index)

    def dense(self):
        data = []
        for k in range(self.net.p):
            x = np.zeros(int(np.prod(self.net.shape(k))), dtype=np.float64)
            sel = self.tensor == k
            np.add.at(x, self.index[sel], self.delta[sel])
            data.append(x.reshape(self.net.shape(k)))
        return self.net.with_data(data)


def _zipf_keys(rng, n, count, s):
    """count keys in [0, n) with P(key = i) proportional to (i + 1)^-s,
    shuffled so popularity does not follow the index."""
    w = 1.0 / np.arange(1, n + 1, dtype=np.float64) ** s
    perm = rng.permutation(n)
    return perm[rng.choice(n, size=count, p=w / w.sum())]


def edge_stream(n=1024, edges=32768, triangles=512, deletions=4096, seed=7):
    """A directed graph as a stream of edge insertions and deletions, fed to
    the triangle network tr(A A A) (Cor. 3: X_1 = X_2 = X_3 = A, contractions
    the 0-based form of {(1,6),(2,3),(4,5)}): random edges with Zipf(0.8)
    endpoints, `triangles` planted directed 3-cycles, then `deletions` of
    inserted edges (turnstile).  Each edge update is sent to all three tensors.
    Returns a Stream."""
    rng = np.random.default_rng([seed, 31])
    src = _zipf_keys(rng, n, edges, 0.8)
    dst = _zipf_keys(rng, n, edges, 0.8)
    keep = src != dst
    src, dst = list(src[keep]), list(dst[keep])
    for _ in range(triangles):
        a, b, c = rng.choice(n, size=3, replace=False)
        src += [a, b, c]
        dst += [b, c, a]
    src, dst = np.array(src, dtype=np.int64), np.array(dst, dtype=np.int64)
    sign = np.ones(len(src))
    gone = rng.choice(len(src), size=min(deletions, len(src)), replace=False)
    src = np.concatenate([src, src[gone]])
    dst = np.concatenate([dst, dst[gone]])
    sign = np.concatenate([sign, -np.ones(len(gone))])
    net = Network([2, 2, 2], [n] * 6, [(0, 5), (1, 2), (3, 4)], name=f"graph{n}")
    lin = src * n + dst
    T = len(lin)
    return Stream(net, np.repeat(np.arange(3), T), np.tile(lin, 3), np.tile(sign, 3), f"edges{n}")


def join_stream(kind="chain", n=256, tuples=20000, s=1.1, seed=9):
    """Relations as a tuple stream for join-size estimation (Cor. 2): each
    relation is a frequency tensor over its join attributes, and each tuple an
    update +1 of its entry.  kind 'chain': R1(a) R2(a,b) R3(b,c) R4(c) joined
    on a, b, c (acyclic); 'cycle': R1(a,b) R2(b,c) R3(c,a) (cyclic); 'star':
    R1(a) R2(a) R3(a,b) R4(b), where attribute a joins three relations (a
    hyperedge): by WLOG 1 a copy tensor C[a, a', a''] = [a = a' = a''] of order
    3 takes the place of the hyperedge, its three modes contracted with the
    three a modes; its n diagonal ones lead the stream (tensor 4).  Join keys
    are Zipf(s) over domains of size n.  Returns a Stream."""
    rng = np.random.default_rng([seed, 41])
    tensor, index, delta = [], [], []
    if kind == "chain":
        net = Network([1, 2, 2, 1], [n] * 6, [(0, 1), (2, 3), (4, 5)], name=f"join_chain{n}")
        arities = [1, 2, 2, 1]
    elif kind == "cycle":
        net = Network([2, 2, 2], [n] * 6, [(1, 2), (3, 4), (5, 0)], name=f"join_cycle{n}")
        arities = [2, 2, 2]
    elif kind == "star":
        # modes: R1 0; R2 1; R3 2 (a), 3 (b); R4 4; C 5, 6, 7
        net = Network([1, 1, 2, 1, 3], [n] * 8, [(0, 5), (1, 6), (2, 7), (3, 4)], name=f"join_star{n}")
        arities = [1, 1, 2, 1]
        diag = np.arange(n, dtype=np.int64)
        tensor.append(np.full(n, 4))
        index.append(diag * n * n + diag * n + diag)
        delta.append(np.ones(n))
    else:
        raise ValueError(kind)
    for k, a in enumerate(arities):
        cols = [_zipf_keys(rng, n, tuples, s) for _ in range(a)]
        lin = cols[0] if a == 1 else cols[0] * n + cols[1]
        tensor.append(np.full(tuples, k))
        index.append(lin)
        delta.append(np.ones(tuples))
    return Stream(net, np.concatenate(tensor), np.concatenate(index), np.concatenate(delta), f"{kind}{n}")
