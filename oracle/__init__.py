"""FP64 CPU oracle for the sketching estimators (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it.  The arithmetic lives in ``tn_oracle.c`` (plain C,
FP64); this module builds it with gcc and marshals numpy arrays through ctypes.

Functions (each cites the passage of arXiv 2603.07387 it follows):
  * ``hash_table``    -- the count-sketch hash family (Def. 10-11; construction
                         stated in tn_oracle.c)
  * ``tc_literal``    -- Def. 1 read literally (Iverson brackets over all modes)
  * ``tc_full``       -- Def. 1-3 with one summation index per contraction
  * ``tc_tree``       -- Lemma 8 recursion for acyclic networks
  * ``m1_estimate``   -- Method 1, Eq. (1) / Algorithm 1, per sample
  * ``m1_enumerate``  -- exact mean/variance of Method 1 over all hash functions
  * ``m2_estimate``   -- Method 2, Eq. (2) / Algorithms 2-5, per sample
  * ``xcorr_estimate``/``xcorr_enumerate`` -- the earlier cross-correlation
                         estimator of Examples 2-3 (one count sketch per
                         contraction on both modes, a chain of Def. 9
                         cross-correlations), per sample and exactly
  * ``circ_xcorr``    -- Def. 9
  * ``dft``/``fft``/``circ_conv`` -- Def. 8 and the DFT convention of Lemma 5's proof
  * ``mean_var``      -- Welford sample mean / unbiased variance
  * ``median_of_means`` -- the median amplification of Theorem 1
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tn_oracle.c")
# TN_ORACLE_SANITIZE=1: build and load an AddressSanitizer + UndefinedBehavior-
# Sanitizer copy instead (the process must preload gcc's libasan).
_SAN = os.environ.get("TN_ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libtn_oracle_san.so" if _SAN else "libtn_oracle.so")
_lib = None

STREAM_TSKETCH = 1 << 62
STREAM_PAD = 1 << 63


def build(force=False):
    """Compile tn_oracle.c with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        san = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined"] if _SAN else []
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", *san,
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        dpp = ctypes.POINTER(dp)
        L.orc_mix.restype = ctypes.c_uint64
        L.orc_mix.argtypes = [ctypes.c_uint64]
        L.orc_hash_coeffs.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_uint64)]
        L.orc_count_sketch.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_int64, ctypes.c_int64, i64p,
                                       ctypes.POINTER(ctypes.c_int32)]
        L.orc_stream_tsketch.restype = ctypes.c_uint64
        L.orc_stream_tsketch.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
        L.orc_stream_pad.restype = ctypes.c_uint64
        L.orc_stream_pad.argtypes = [ctypes.c_int64, ctypes.c_int64]
        net = [ctypes.c_int, ip, i64p, dpp, ctypes.c_int, ip]
        L.orc_tc_literal.argtypes = net + [dp]
        L.orc_tc_full.argtypes = net + [dp]
        L.orc_tc_tree.argtypes = net + [ctypes.c_int, dp]
        L.orc_tc_torus.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.POINTER(ctypes.c_double)), dp]
        L.orc_m1_estimate.argtypes = net + [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                                            i64p, ctypes.c_int, dp, dp, dp]
        L.orc_m1_enumerate.argtypes = net + [ctypes.c_int64, dp, dp, i64p]
        L.orc_m2_estimate.argtypes = net + [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                                            ctypes.c_int, ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_uint64), i64p, i64p,
                                            ctypes.c_int, dp, dp, dp]
        L.orc_bf16_round.restype = ctypes.c_double
        L.orc_bf16_round.argtypes = [ctypes.c_double]
        L.orc_dft.argtypes = [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_int]
        L.orc_fft.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int]
        L.orc_circ_conv.argtypes = [ctypes.c_int64, dp, dp, dp]
        L.orc_circ_xcorr.argtypes = [ctypes.c_int64, dp, dp, dp]
        L.orc_xcorr_estimate.argtypes = net + [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64,
                                               i64p, dp, dp, dp]
        L.orc_xcorr_enumerate.argtypes = net + [ctypes.c_int64, dp, dp, i64p]
        L.orc_mean_var.argtypes = [ctypes.c_int64, dp, dp, dp]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Net:
    """ctypes view of a tn_workloads.Network (data promoted to float64)."""

    def __init__(self, net):
        self.p = net.p
        self.t = net.t
        self.order = (ctypes.c_int * max(1, net.p))(*net.orders)
        self.dims = (ctypes.c_int64 * max(1, net.q))(*net.dims)
        self.arrays = [np.ascontiguousarray(np.asarray(x), dtype=np.float64) for x in net.data]
        DP = ctypes.POINTER(ctypes.c_double)
        self.data = (DP * max(1, net.p))(*[_dptr(a) for a in self.arrays])
        flat = [m for e in net.edges for m in e]
        self.edges = (ctypes.c_int * max(1, len(flat)))(*flat)

    def args(self):
        return [self.p, self.order, self.dims, self.data, self.t, self.edges]


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def mix(x):
    return int(lib().orc_mix(ctypes.c_uint64(x & (2**64 - 1))))


def hash_coeffs(seed, sample, stream):
    c = (ctypes.c_uint64 * 6)()
    lib().orc_hash_coeffs(seed, sample, stream, c)
    return [int(v) for v in c]


def hash_table(seed, sample, stream, n, m):
    """Count sketch of one stream: buckets h in [0, m) and signs s in {-1, +1}."""
    h = np.zeros(n, dtype=np.int64)
    s = np.zeros(n, dtype=np.int32)
    lib().orc_count_sketch(seed, sample, stream, n, m,
                           h.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return h, s


def stream_tsketch(node, level, j, side):
    return int(lib().orc_stream_tsketch(node, level, j, side))


def stream_pad(node, slot):
    return int(lib().orc_stream_pad(node, slot))


def tc_literal(net):
    """Def. 1 literally; returns an array over the free modes (scalar if none)."""
    n = _Net(net)
    used = set(m for e in net.edges for m in e)
    free = [u for u in range(net.q) if u not in used]
    shape = tuple(net.dims[u] for u in free)
    out = np.zeros(int(np.prod(shape)) if shape else 1)
    _check(lib().orc_tc_literal(*n.args(), _dptr(out)), "tc_literal")
    return out.reshape(shape) if shape else float(out[0])


def tc_full(net):
    n = _Net(net)
    out = np.zeros(1)
    _check(lib().orc_tc_full(*n.args(), _dptr(out)), "tc_full")
    return float(out[0])


def tc_torus(tensors, R, C):
    """Periodic R x C lattice contracted through its row transfer matrices;
    tensors[r * C + c] has modes (left, right, up, down), each of size D."""
    D = int(np.asarray(tensors[0]).shape[0])
    arrs = [np.ascontiguousarray(np.asarray(x, dtype=np.float64)) for x in tensors]
    assert len(arrs) == R * C and all(a.shape == (D, D, D, D) for a in arrs)
    ptrs = (ctypes.POINTER(ctypes.c_double) * (R * C))(*[_dptr(a) for a in arrs])
    out = np.zeros(1)
    _check(lib().orc_tc_torus(R, C, D, ptrs, _dptr(out)), "tc_torus")
    return float(out[0])


def tc_tree(net, root=0):
    n = _Net(net)
    out = np.zeros(1)
    _check(lib().orc_tc_tree(*n.args(), root, _dptr(out)), "tc_tree")
    return float(out[0])


def m1_estimate(net, m, seed, sample, tables=None, combine="conv", want_sketches=False,
                want_scale=False):
    """One Method-1 estimate.  ``tables``: optional per-edge [h..., s...] int arrays
    (concatenated in edge order) replacing the hash family."""
    n = _Net(net)
    est = np.zeros(1)
    sk = np.zeros(net.p * m) if want_sketches else None
    sc = np.zeros(1) if want_scale else None
    tab = None
    if tables is not None:
        tab = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.int64) for t in tables]))
    rc = lib().orc_m1_estimate(
        *n.args(), m, seed, sample,
        tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if tab is not None else None,
        {"conv": 0, "dft": 1}[combine], _dptr(est),
        _dptr(sk) if sk is not None else None, _dptr(sc) if sc is not None else None)
    _check(rc, "m1_estimate")
    out = {"estimate": float(est[0])}
    if sk is not None:
        out["sketches"] = sk.reshape(net.p, m)
    if sc is not None:
        out["scale"] = float(sc[0])
    return out


def m1_enumerate(net, m):
    """Exact (mean, variance, count) of Method 1 over every fully random hash assignment."""
    n = _Net(net)
    mean = np.zeros(1)
    var = np.zeros(1)
    cnt = ctypes.c_int64(0)
    _check(lib().orc_m1_enumerate(*n.args(), m, _dptr(mean), _dptr(var), ctypes.byref(cnt)),
           "m1_enumerate")
    return float(mean[0]), float(var[0]), int(cnt.value)


def xcorr_estimate(net, m, seed, sample, tables=None, want_sketches=False, want_scale=False):
    """One estimate of the earlier cross-correlation method (Examples 2-3): the
    same count sketch C_e on both modes of contraction e, tensor sketches, and
    e_1^T (y_1 star ... star y_p) with Def. 9 applied left to right."""
    n = _Net(net)
    est = np.zeros(1)
    sk = np.zeros(net.p * m) if want_sketches else None
    sc = np.zeros(1) if want_scale else None
    tab = None
    if tables is not None:
        tab = np.ascontiguousarray(np.concatenate([np.asarray(t, dtype=np.int64) for t in tables]))
    rc = lib().orc_xcorr_estimate(
        *n.args(), m, seed, sample,
        tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if tab is not None else None,
        _dptr(est), _dptr(sk) if sk is not None else None, _dptr(sc) if sc is not None else None)
    _check(rc, "xcorr_estimate")
    out = {"estimate": float(est[0])}
    if sk is not None:
        out["sketches"] = sk.reshape(net.p, m)
    if sc is not None:
        out["scale"] = float(sc[0])
    return out


def xcorr_enumerate(net, m):
    """Exact (mean, variance, count) of the cross-correlation estimator over
    every fully random hash assignment."""
    n = _Net(net)
    mean = np.zeros(1)
    var = np.zeros(1)
    cnt = ctypes.c_int64(0)
    _check(lib().orc_xcorr_enumerate(*n.args(), m, _dptr(mean), _dptr(var), ctypes.byref(cnt)),
           "xcorr_enumerate")
    return float(mean[0]), float(var[0]), int(cnt.value)


def m2_estimate(net, m, seed, sample, root=0, want_trace=False, tables=None, bf16_products=False):
    """One Method-2 estimate (Algorithm 2).  With want_trace, also the sketch
    x_l of every tensor (x_o for the root) and r_o.  ``tables`` maps stream id ->
    (h, s) arrays that replace the hash family for that stream.  bf16_products:
    the BF16-product variant (both factors of every SMVP product and of the
    root's dot product rounded to BF16, ties to even, via FP32; sums in FP64)."""
    n = _Net(net)
    est = np.zeros(1)
    tr = np.zeros(net.p * m) if want_trace else None
    ro = np.zeros(m) if want_trace else None
    tables = tables or {}
    ids = (ctypes.c_uint64 * max(1, len(tables)))(*[int(k) for k in tables])
    lens = np.array([len(h) for (h, s) in tables.values()] or [0], dtype=np.int64)
    tab = np.concatenate([np.concatenate([np.asarray(h, np.int64), np.asarray(s, np.int64)])
                          for (h, s) in tables.values()] or [np.zeros(1, np.int64)])
    tab = np.ascontiguousarray(tab, dtype=np.int64)
    rc = lib().orc_m2_estimate(*n.args(), m, seed, sample, root, len(tables), ids,
                               lens.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                               tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(bf16_products), _dptr(est),
                               _dptr(tr) if tr is not None else None,
                               _dptr(ro) if ro is not None else None)
    _check(rc, "m2_estimate")
    out = {"estimate": float(est[0])}
    if want_trace:
        out["x"] = tr.reshape(net.p, m)
        out["r_root"] = ro
    return out


def m2_streams(net, root=0):
    """Hash streams Method 2 draws for a tree rooted at `root`: (stream id, domain).
    Contractions e over [n_e]; per tensor with c >= 1 children, padded order
    qt = next power of two, the tensor sketches T_{l,j} (two count sketches over
    [m] each, marked by domain None) and the qt - c padding sketches over [1]."""
    partner = {}
    for (u, v) in net.edges:
        partner[u], partner[v] = v, u
    parent_mode = {root: None}
    nchild = {}
    queue = [root]
    while queue:
        k = queue.pop(0)
        nchild[k] = 0
        for u in net.modes(k):
            if u == parent_mode[k]:
                continue
            l = net.tensor_of(partner[u])
            parent_mode[l] = partner[u]
            nchild[k] += 1
            queue.append(l)
    out = [(e, net.dims[u]) for e, (u, _) in enumerate(net.edges)]
    for k in sorted(nchild):
        c = nchild[k]
        if c == 0:
            continue
        qt = 1
        while qt < c:
            qt *= 2
        l = qt
        while l >= 2:
            for j in range(l // 2):
                out.append((stream_tsketch(k, l, j, 0), None))
                out.append((stream_tsketch(k, l, j, 1), None))
            l //= 2
        for j in range(c, qt):
            out.append((stream_pad(k, j), 1))
    return out


def m2_scale(net, m, seed, sample, root=0, want_trace=False):
    """Rounding-error scale for Method 2: the same estimate with every entry
    replaced by |X| and every sign by +1 (same buckets), which bounds the
    magnitude of every partial sum the estimator forms.  With want_trace, the
    per-tensor sketch bounds as well."""
    absnet = net.with_data([np.abs(np.asarray(x, dtype=np.float64)) for x in net.data])
    tables = {}
    for sid, n in m2_streams(net, root):
        h, _ = hash_table(seed, sample, sid, m if n is None else n, m)
        tables[sid] = (h, np.ones_like(h))
    out = m2_estimate(absnet, m, seed, sample, root, want_trace=want_trace, tables=tables)
    return out if want_trace else abs(out["estimate"])


def dft(x, inverse=False):
    x = np.asarray(x, dtype=np.complex128)
    m = len(x)
    re, im = np.ascontiguousarray(x.real), np.ascontiguousarray(x.imag)
    ore, oim = np.zeros(m), np.zeros(m)
    lib().orc_dft(m, _dptr(re), _dptr(im), _dptr(ore), _dptr(oim), int(inverse))
    return ore + 1j * oim


def fft(x, inverse=False):
    x = np.asarray(x, dtype=np.complex128)
    m = len(x)
    re, im = np.ascontiguousarray(x.real).copy(), np.ascontiguousarray(x.imag).copy()
    lib().orc_fft(m, _dptr(re), _dptr(im), int(inverse))
    return re + 1j * im


def circ_conv(x, y):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(len(x))
    lib().orc_circ_conv(len(x), _dptr(x), _dptr(y), _dptr(out))
    return out


def bf16_round(x):
    """Nearest BF16 value of x (ties to even), through FP32."""
    return float(lib().orc_bf16_round(float(x)))


def circ_xcorr(x, y):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(len(x))
    lib().orc_circ_xcorr(len(x), _dptr(x), _dptr(y), _dptr(out))
    return out


def median_of_means(x, groups):
    """Median of the means of `groups` consecutive groups of x, group g holding
    x[floor(g S / G) : floor((g + 1) S / G)] (the amplification of Theorem 1)."""
    x = np.asarray(x, dtype=np.float64)
    S = len(x)
    means = [float(np.mean(x[g * S // groups:(g + 1) * S // groups])) for g in range(groups)]
    return float(np.median(means))


def mean_var(x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    mu, var = np.zeros(1), np.zeros(1)
    lib().orc_mean_var(len(x), _dptr(x), _dptr(mu), _dptr(var))
    return float(mu[0]), float(var[0])
