"""ctypes binding of libtnsketch.so: argument marshalling only.

Functions carry the C names of include/tn_sketch.h.  Tensors are torch tensors
on the current HIP device; streams default to torch's current stream.  Every
non-zero return code raises TNError with the library's message.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first: the library then shares torch's HIP runtime

TN_OK = 0
TN_ERR_ARG = -1
TN_ERR_DIMS = -2
TN_ERR_HYPEREDGE = -3
TN_ERR_SELFLOOP = -4
TN_ERR_CYCLIC = -5
TN_ERR_PARTIAL = -6
TN_ERR_OOM = -7
TN_ERR_HIP = -8
TN_ERR_UNSUPPORTED = -9
TN_F64, TN_F32, TN_BF16 = 0, 1, 2
TN_CYCLIC, TN_ACYCLIC = 1, 2
TN_FLAG_GRAPH = 0x1
TN_FLAG_PROFILE = 0x2
TN_FLAG_AUTOTUNE = 0x4
TN_FLAG_MFMA_BF16 = 0x8
TN_FLAG_PERSISTENT = 0x10
TN_FLAG_PROFILE_SKETCH = 0x20
TN_FLAG_PRIOR_XCORR = 0x40
TN_FLAG_RESIDENT = 0x80
TN_FLAG_SIZE_PILOT = 0x100
TN_FLAG_SIZE_LEARNED = 0x200
TN_FLAG_DFT_BF16 = 0x400
TN_FLAG_MFMA_F32 = 0x800
TN_FLAG_DFT_FP8 = 0x1000
TN_SIZE_BOUND, TN_SIZE_PILOT, TN_SIZE_LEARNED = 0, 1, 2
TN_KERNEL_HASH, TN_KERNEL_SKETCH, TN_KERNEL_COMBINE, TN_KERNEL_STATS = 0, 1, 2, 3

_DTYPES = {torch.float64: TN_F64, torch.float32: TN_F32, torch.bfloat16: TN_BF16}

_HERE = os.path.dirname(os.path.abspath(__file__))
# TN_SKETCH_LIB names another build of the same library (the host-side
# sanitizer build of build_sanitize.py); by default the in-tree build.
_LIBPATH = os.environ.get("TN_SKETCH_LIB") or os.path.join(_HERE, "libtnsketch.so")
_lib = None


class TNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class tn_size_choice(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("samples", ctypes.c_int64),
        ("groups", ctypes.c_int32),
        ("p_group", ctypes.c_double),
        ("v", ctypes.c_double),
        ("work", ctypes.c_double),
    ]


class tn_network(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int32),
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("dims", ctypes.POINTER(ctypes.c_int64)),
        ("data", ctypes.POINTER(ctypes.c_void_p)),
        ("dtype", ctypes.c_int32),
        ("t", ctypes.c_int32),
        ("edges", ctypes.POINTER(ctypes.c_int32)),
    ]


def lib_path():
    return _LIBPATH


def load():
    """Load the built library (no fallback: raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        raise RuntimeError(f"{_LIBPATH} is not built; run `python -m paper_2603_07387_amd.build`")
    L = ctypes.CDLL(_LIBPATH)
    P = ctypes.POINTER
    vp, i32, i64, u64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
    net_p = P(tn_network)
    L.tn_sketch_plan.argtypes = [net_p, i32, i32, i64, i64, u64, i32, u32, P(vp)]
    L.tn_sketch_plan.restype = ctypes.c_int
    L.tn_sketch_estimate.argtypes = [vp, net_p, vp, vp, vp]
    L.tn_sketch_estimate.restype = ctypes.c_int
    L.tn_contract_exact.argtypes = [net_p, vp, P(ctypes.c_double)]
    L.tn_contract_exact.restype = ctypes.c_int
    L.tn_plan_destroy.argtypes = [vp]
    L.tn_plan_destroy.restype = None
    L.tn_last_error.argtypes = []
    L.tn_last_error.restype = ctypes.c_char_p
    L.tn_plan_query.argtypes = [vp, i32]
    L.tn_plan_query.restype = ctypes.c_int64
    L.tn_plan_stream.argtypes = [vp, i64, P(i32), P(u64), P(i64), P(i64)]
    L.tn_plan_stream.restype = ctypes.c_int
    L.tn_plan_get_hashes.argtypes = [vp, i64, i64, vp, vp]
    L.tn_plan_get_hashes.restype = ctypes.c_int
    L.tn_plan_set_hashes.argtypes = [vp, vp, vp]
    L.tn_plan_set_hashes.restype = ctypes.c_int
    L.tn_plan_get_sketches.argtypes = [vp, net_p, i64, i64, vp, vp]
    L.tn_plan_get_sketches.restype = ctypes.c_int
    L.tn_plan_kernel_time.argtypes = [vp, i32, P(ctypes.c_double), P(i64)]
    L.tn_plan_kernel_time.restype = ctypes.c_int
    L.tn_median_of_means.argtypes = [vp, i64, i64, i32, vp, vp]
    L.tn_median_of_means.restype = ctypes.c_int
    L.tn_partial_plan.argtypes = [net_p, i64, i64, u64, u32, P(vp)]
    L.tn_partial_plan.restype = ctypes.c_int
    L.tn_sketch_update.argtypes = [vp, i32, i32, i64, vp, vp, vp]
    L.tn_sketch_update.restype = ctypes.c_int
    L.tn_sketch_combine.argtypes = [vp, vp, vp, vp]
    L.tn_sketch_combine.restype = ctypes.c_int
    L.tn_sketch_reset.argtypes = [vp, vp]
    L.tn_sketch_reset.restype = ctypes.c_int
    L.tn_sketch_size.argtypes = [net_p, i32, i32, ctypes.c_double, ctypes.c_double, i32, i32, u64, vp,
                                 P(tn_size_choice)]
    L.tn_sketch_size.restype = ctypes.c_int
    L.tn_median_groups.argtypes = [ctypes.c_double, ctypes.c_double, P(i32)]
    L.tn_median_groups.restype = ctypes.c_int
    L.tn_set_size_target.argtypes = [ctypes.c_double, ctypes.c_double]
    L.tn_set_size_target.restype = ctypes.c_int
    L.tn_set_size_selector.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.tn_set_size_selector.restype = ctypes.c_int
    L.tn_mlp_save.argtypes = [vp, ctypes.c_char_p, P(ctypes.c_double), i32]
    L.tn_mlp_save.restype = ctypes.c_int
    L.tn_mlp_load.argtypes = [ctypes.c_char_p, P(vp), P(ctypes.c_double), i32, P(i32)]
    L.tn_mlp_load.restype = ctypes.c_int
    _lib = L
    return L


def tn_last_error():
    return load().tn_last_error().decode(errors="replace")


def _check(rc):
    if rc < 0:
        raise TNError(int(rc), tn_last_error())
    return rc


def _stream(stream):
    if stream is None:
        if not torch.cuda.is_initialized():
            return ctypes.c_void_p(0)      # default stream; nothing queued by torch yet
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _on_current_device(t, what):
    """Raise ValueError unless tensor t lives on the current HIP device (the
    library reads and writes device memory only)."""
    if not t.is_cuda:
        raise ValueError(f"{what}: must be a device tensor, got {t.device}")
    if torch.cuda.is_initialized() and t.device.index != torch.cuda.current_device():
        raise ValueError(f"{what}: on {t.device}, the current device is cuda:{torch.cuda.current_device()}")


def _device_buffer(t, dtype, count, what):
    """Check an output or input buffer: a contiguous device tensor of `dtype`
    holding at least `count` elements."""
    if t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, expected {dtype}")
    if t.numel() < count:
        raise ValueError(f"{what}: {t.numel()} elements, at least {count} needed")
    if not t.is_contiguous():
        raise ValueError(f"{what}: not contiguous")
    _on_current_device(t, what)


class NetworkSpec:
    """A tn_network: structure from (orders, dims, edges) and device tensors."""

    def __init__(self, orders, dims, edges, tensors=None, dtype=None):
        self.orders = list(orders)
        self.dims = list(dims)
        self.edges = [int(m) for e in edges for m in e]
        self.p = len(self.orders)
        self._order = (ctypes.c_int32 * max(1, self.p))(*self.orders)
        self._dims = (ctypes.c_int64 * max(1, len(self.dims)))(*self.dims)
        self._edges = (ctypes.c_int32 * max(1, len(self.edges)))(*self.edges)
        self._data = (ctypes.c_void_p * max(1, self.p))()
        self.tensors = None
        if dtype is None:
            dtype = tensors[0].dtype if tensors else torch.float32
        self.dtype = _DTYPES[dtype]
        if tensors is not None:
            self.bind(tensors)

    @classmethod
    def from_network(cls, net, tensors=None, dtype=None):
        return cls(net.orders, net.dims, net.edges, tensors, dtype)

    def sizes(self):
        """Entries of each tensor: the product of its mode sizes."""
        out, u = [], 0
        for q in self.orders:
            n = 1
            for d in self.dims[u:u + q]:
                n *= int(d)
            out.append(n)
            u += q
        return out

    def bind(self, tensors):
        """Bind device tensors.  The C ABI trusts the pointers it is given, so
        every property it relies on is checked here first: one contiguous
        tensor per network tensor, of the network dtype, holding exactly the
        product of its mode sizes, on the current HIP device."""
        if len(tensors) != self.p:
            raise ValueError("one tensor per network tensor is required")
        sizes = self.sizes()
        for k, t in enumerate(tensors):
            if t.dtype not in _DTYPES or _DTYPES[t.dtype] != self.dtype:
                raise ValueError(f"tensor {k}: dtype {t.dtype} differs from the network dtype")
            if t.numel() != sizes[k]:
                raise ValueError(f"tensor {k}: {t.numel()} entries, its modes need {sizes[k]}")
            if not t.is_contiguous():
                raise ValueError(f"tensor {k}: not contiguous (row-major is required)")
        for k, t in enumerate(tensors):
            _on_current_device(t, f"tensor {k}")
        self.tensors = list(tensors)
        for k, t in enumerate(tensors):
            self._data[k] = t.data_ptr()
        return self

    def struct(self):
        return tn_network(self.p, self._order, self._dims, self._data, self.dtype,
                          len(self.edges) // 2, self._edges)


def _array(specs):
    arr = (tn_network * len(specs))(*[s.struct() for s in specs])
    return arr


def tn_sketch_plan(specs, method, m, samples, seed, root=-1, flags=0):
    arr = specs if isinstance(specs, ctypes.Array) else _array(specs)
    handle = ctypes.c_void_p()
    _check(load().tn_sketch_plan(arr, len(arr), method, m, samples, seed, root, flags, ctypes.byref(handle)))
    return handle


def tn_partial_plan(spec, m, samples, seed, flags=0):
    """Plan for a partial TNC (Corollary 1): one network with free modes."""
    arr = spec if isinstance(spec, ctypes.Array) else _array([spec])
    handle = ctypes.c_void_p()
    _check(load().tn_partial_plan(arr, m, samples, seed, flags, ctypes.byref(handle)))
    return handle


def tn_sketch_estimate(plan, specs, stream, stats, samples_out=None):
    """`specs` is a list of NetworkSpec or an array built by _array() (reused
    across calls: its structs point at each spec's data-pointer array, which
    NetworkSpec.bind updates in place)."""
    arr = specs if isinstance(specs, ctypes.Array) else _array(specs)
    return _check(load().tn_sketch_estimate(plan, arr, _stream(stream), _ptr(stats), _ptr(samples_out)))


def tn_contract_exact(spec, stream=None):
    out = ctypes.c_double(0.0)
    _check(load().tn_contract_exact(_array([spec]), _stream(stream), ctypes.byref(out)))
    return out.value


def tn_plan_destroy(plan):
    load().tn_plan_destroy(plan)


def tn_plan_query(plan, key):
    return int(_check(load().tn_plan_query(plan, key)))


def tn_plan_stream(plan, i):
    net, sid, n, off = ctypes.c_int32(), ctypes.c_uint64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().tn_plan_stream(plan, i, ctypes.byref(net), ctypes.byref(sid), ctypes.byref(n),
                                 ctypes.byref(off)))
    return net.value, sid.value, n.value, off.value


def tn_plan_get_hashes(plan, first, count, stream, out):
    return _check(load().tn_plan_get_hashes(plan, first, count, _stream(stream), _ptr(out)))


def tn_plan_set_hashes(plan, tables, stream=None):
    return _check(load().tn_plan_set_hashes(plan, _ptr(tables), _stream(stream)))


def tn_plan_get_sketches(plan, specs, first, count, stream, out):
    return _check(load().tn_plan_get_sketches(plan, _array(specs), first, count, _stream(stream),
                                              _ptr(out)))


def tn_plan_kernel_time(plan, kind):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(load().tn_plan_kernel_time(plan, kind, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def tn_tensor_stats(specs, stream=None):
    """Per tensor [sum x, sum x^2, sum |x|, #(x >= 0)] as a numpy (tensors, 4) array."""
    import numpy as np
    L = load()
    L.tn_tensor_stats.argtypes = [ctypes.POINTER(tn_network), ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_double)]
    nt = sum(s.p for s in specs)
    out = np.zeros(nt * 4, dtype=np.float64)
    _check(L.tn_tensor_stats(_array(specs), len(specs), _stream(stream),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(nt, 4)


def tn_tensor_stats_noalloc(specs, stream=None):
    """tn_tensor_stats through the allocation-free entry point (fixed device
    scratch of the library; at most 32768 tensors)."""
    import numpy as np
    L = load()
    L.tn_tensor_stats_noalloc.argtypes = [ctypes.POINTER(tn_network), ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double)]
    nt = sum(s.p for s in specs)
    out = np.zeros(nt * 4, dtype=np.float64)
    _check(L.tn_tensor_stats_noalloc(_array(specs), len(specs), _stream(stream),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out.reshape(nt, 4)


def tn_sketch_size(specs, method, eps, delta, max_groups=1, mode=TN_SIZE_BOUND, seed=0, stream=None):
    """Per network a dict(m, samples, groups, p_group, v, work) (tn_sketch_size)."""
    arr = specs if isinstance(specs, ctypes.Array) else _array(specs)
    out = (tn_size_choice * len(arr))()
    _check(load().tn_sketch_size(arr, len(arr), method, eps, delta, max_groups, mode, seed, _stream(stream), out))
    return [{k: getattr(c, k) for k, _ in tn_size_choice._fields_} for c in out]


def tn_median_groups(delta, p_group):
    g = ctypes.c_int32()
    _check(load().tn_median_groups(delta, p_group, ctypes.byref(g)))
    return g.value


def tn_set_size_target(eps, delta):
    _check(load().tn_set_size_target(eps, delta))


def tn_set_size_selector(mlp_handle, mu, sd, margin):
    _check(load().tn_set_size_selector(mlp_handle, mu, sd, margin))


def tn_mlp_save(net, path, meta=()):
    m = (ctypes.c_double * max(1, len(meta)))(*meta)
    _check(load().tn_mlp_save(net, os.fsencode(path), m, len(meta)))


def tn_mlp_load(path, max_meta=64):
    h = ctypes.c_void_p()
    m = (ctypes.c_double * max_meta)()
    n = ctypes.c_int32()
    _check(load().tn_mlp_load(os.fsencode(path), ctypes.byref(h), m, max_meta, ctypes.byref(n)))
    return h, list(m[:n.value])


def tn_median_of_means(samples, n_nets, S, groups, stream, out):
    return _check(load().tn_median_of_means(_ptr(samples), n_nets, S, groups, _stream(stream), _ptr(out)))


def median_of_means(samples, groups, stream=None):
    """Median of `groups` group means per row of a (n_nets, S) float64 device tensor."""
    if samples.dim() != 2 or samples.dtype != torch.float64 or not samples.is_contiguous():
        raise ValueError("samples must be a contiguous (n_nets, S) float64 tensor")
    _on_current_device(samples, "samples")
    out = torch.empty(samples.shape[0], dtype=torch.float64, device=samples.device)
    tn_median_of_means(samples, samples.shape[0], samples.shape[1], groups, stream, out)
    return out


def _mlp_lib():
    L = load()
    if getattr(L, "_mlp_ready", False):
        return L
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.tn_mlp_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, P(vp)]
    L.tn_mlp_num_params.argtypes = [vp]
    L.tn_mlp_num_params.restype = ctypes.c_int64
    L.tn_mlp_get_params.argtypes = [vp, P(ctypes.c_float)]
    L.tn_mlp_set_params.argtypes = [vp, P(ctypes.c_float)]
    L.tn_mlp_predict.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    L.tn_mlp_grad.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, P(ctypes.c_double)]
    L.tn_mlp_step.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_float, vp]
    L.tn_mlp_train.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_float, vp, P(ctypes.c_double)]
    L.tn_mlp_destroy.argtypes = [vp]
    L.tn_mlp_destroy.restype = None
    L.tn_mlp_shape.argtypes = [vp, P(ctypes.c_int32), P(ctypes.c_int32)]
    L._mlp_ready = True
    return L


def tn_mlp_create(d_in, hidden, seed):
    h = ctypes.c_void_p()
    _check(_mlp_lib().tn_mlp_create(d_in, hidden, seed, ctypes.byref(h)))
    return h


def tn_mlp_num_params(net):
    return int(_check(_mlp_lib().tn_mlp_num_params(net)))


def tn_mlp_get_params(net):
    import numpy as np
    out = np.zeros(tn_mlp_num_params(net), dtype=np.float32)
    _check(_mlp_lib().tn_mlp_get_params(net, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return out


def tn_mlp_set_params(net, params):
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(_mlp_lib().tn_mlp_set_params(net, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))


def tn_mlp_predict(net, X, stream, out):
    return _check(_mlp_lib().tn_mlp_predict(net, _ptr(X), X.shape[0], _stream(stream), _ptr(out)))


def tn_mlp_grad(net, X, y, stream, grad):
    loss = ctypes.c_double()
    _check(_mlp_lib().tn_mlp_grad(net, _ptr(X), _ptr(y), X.shape[0], _stream(stream), _ptr(grad),
                                  ctypes.byref(loss)))
    return loss.value


def tn_mlp_step(net, X, y, lr, stream=None):
    return _check(_mlp_lib().tn_mlp_step(net, _ptr(X), _ptr(y), X.shape[0], lr, _stream(stream)))


def tn_mlp_train(net, X, y, batch, epochs, lr, stream=None, want_losses=True):
    import numpy as np
    losses = np.zeros(max(1, epochs), dtype=np.float64) if want_losses else None
    _check(_mlp_lib().tn_mlp_train(
        net, _ptr(X), _ptr(y), X.shape[0], batch, epochs, lr, _stream(stream),
        losses.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if losses is not None else None))
    return losses[:epochs] if losses is not None else None


def tn_mlp_destroy(net):
    _mlp_lib().tn_mlp_destroy(net)


class MLP:
    """Owns a tn_mlp handle (3-layer tanh perceptron, FP32, device kernels)."""

    def __init__(self, d_in, hidden=64, seed=0):
        self.d_in, self.hidden = d_in, hidden
        self.handle = tn_mlp_create(d_in, hidden, seed)

    @property
    def num_params(self):
        return tn_mlp_num_params(self.handle)

    def params(self):
        return tn_mlp_get_params(self.handle)

    def set_params(self, p):
        tn_mlp_set_params(self.handle, p)

    def _rows(self, X, y=None):
        """Check a feature batch (n, d_in) FP32 and its targets (n) FP32."""
        if X.dim() != 2 or X.shape[1] != self.d_in:
            raise ValueError(f"X must be (n, {self.d_in}), got {tuple(X.shape)}")
        _device_buffer(X, torch.float32, X.shape[0] * self.d_in, "X")
        if y is not None:
            _device_buffer(y, torch.float32, X.shape[0], "y")

    def predict(self, X, stream=None):
        self._rows(X)
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        tn_mlp_predict(self.handle, X, stream, out)
        return out

    def grad(self, X, y, stream=None):
        self._rows(X, y)
        g = torch.empty(self.num_params, dtype=torch.float32, device=X.device)
        loss = tn_mlp_grad(self.handle, X, y, stream, g)
        return g, loss

    def step(self, X, y, lr, stream=None):
        self._rows(X, y)
        tn_mlp_step(self.handle, X, y, lr, stream)

    def train(self, X, y, batch=4096, epochs=100, lr=1e-3, stream=None):
        self._rows(X, y)
        return tn_mlp_train(self.handle, X, y, batch, epochs, lr, stream)

    def save(self, path, meta=()):
        tn_mlp_save(self.handle, path, meta)

    @classmethod
    def load(cls, path):
        """A network read from a tn_mlp_save file, and the file's meta values."""
        h, meta = tn_mlp_load(path)
        obj = cls.__new__(cls)
        obj.handle = h
        d, hdn = ctypes.c_int32(), ctypes.c_int32()
        _check(_mlp_lib().tn_mlp_shape(h, ctypes.byref(d), ctypes.byref(hdn)))
        obj.d_in, obj.hidden = d.value, hdn.value
        return obj, meta

    def close(self):
        if self.handle is not None and self.handle.value:
            tn_mlp_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Owns a tn_plan handle; thin methods over the C calls."""

    def __init__(self, specs, method, m, samples, seed, root=-1, flags=0):
        self.specs = list(specs)
        self._arr = _array(self.specs)   # marshalled once; rebinding data goes through the specs
        self.handle = tn_sketch_plan(self._arr, method, m, samples, seed, root, flags)
        self.n_nets = len(self.specs)
        self.S = self.query(2)      # the chosen values when m <= 0
        self.m = self.query(3)

    def query(self, key):
        return tn_plan_query(self.handle, key)

    def estimate(self, stats=None, samples_out=None, stream=None):
        dev = torch.device("cuda", torch.cuda.current_device())
        if stats is None:
            stats = torch.empty(2 * self.n_nets, dtype=torch.float64, device=dev)
        _device_buffer(stats, torch.float64, 2 * self.n_nets, "stats")
        if samples_out is not None:
            _device_buffer(samples_out, torch.float64, self.n_nets * self.S, "samples_out")
        tn_sketch_estimate(self.handle, self._arr, stream, stats, samples_out)
        return stats

    def update(self, tensor, index, delta, net=0, stream=None):
        """Turnstile update of a resident plan: X_tensor(index[u]) += delta[u]
        (index: int64 device tensor of row-major entry indices, delta: float64)."""
        n = index.numel()
        _device_buffer(index, torch.int64, n, "index")
        _device_buffer(delta, torch.float64, n, "delta")
        _check(load().tn_sketch_update(self.handle, net, tensor, n, _ptr(index), _ptr(delta), _stream(stream)))

    def combine(self, stats=None, samples_out=None, stream=None):
        """Estimates of a resident plan's current sketches (no scan of the tensors)."""
        dev = torch.device("cuda", torch.cuda.current_device())
        if stats is None:
            stats = torch.empty(2 * self.n_nets, dtype=torch.float64, device=dev)
        _device_buffer(stats, torch.float64, 2 * self.n_nets, "stats")
        if samples_out is not None:
            _device_buffer(samples_out, torch.float64, self.n_nets * self.S, "samples_out")
        _check(load().tn_sketch_combine(self.handle, _stream(stream), _ptr(stats), _ptr(samples_out)))
        return stats

    def reset(self, stream=None):
        _check(load().tn_sketch_reset(self.handle, _stream(stream)))

    def hashes(self, first=0, count=None, stream=None):
        count = self.S - first if count is None else count
        W = self.query(0)
        out = torch.empty(count * W, dtype=torch.int32, device="cuda")
        tn_plan_get_hashes(self.handle, first, count, stream, out)
        return out.view(count, W)

    def set_hashes(self, tables, stream=None):
        if tables is not None:
            _device_buffer(tables, torch.int32, self.S * self.query(0), "hash tables")
        tn_plan_set_hashes(self.handle, tables, stream)

    def sketches(self, first=0, count=1, stream=None):
        slots = self.query(6)
        out = torch.empty(count * slots * self.m, dtype=torch.float64, device="cuda")
        tn_plan_get_sketches(self.handle, self.specs, first, count, stream, out)
        return out.view(count, slots, self.m)

    def kernel_time(self, kind):
        return tn_plan_kernel_time(self.handle, kind)

    def streams(self):
        return [tn_plan_stream(self.handle, i) for i in range(self.query(1))]

    def close(self):
        if self.handle is not None and self.handle.value:
            tn_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PartialPlan(Plan):
    """A tn_partial_plan: estimates every entry of the output tensor over the
    free modes (row-major in increasing mode order).  estimate() returns the
    stats of n_out entries; out_shape gives the output tensor's shape."""

    def __init__(self, spec, m, samples, seed, flags=0):
        self.specs = [spec]
        self._arr = _array(self.specs)
        self.handle = tn_partial_plan(self._arr, m, samples, seed, flags)
        self.n_nets = tn_plan_query(self.handle, 12)
        self.S = samples
        self.m = m
        used = set(spec.edges)
        self.out_shape = tuple(spec.dims[u] for u in range(len(spec.dims)) if u not in used)
