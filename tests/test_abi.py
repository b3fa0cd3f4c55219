"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and validates networks (error codes) before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

import tn_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(tn_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def T():
    import paper_2603_07387_amd as T
    T.load()
    return T


def test_exports_every_declared_symbol(T):
    names = _declared()
    assert "tn_sketch_plan" in names and "tn_sketch_estimate" in names and "tn_contract_exact" in names
    lib = ctypes.CDLL(T.lib_path())
    for n in names:
        assert hasattr(lib, n), n


def _spec(T, net, dtype="float32"):
    import torch
    return T.NetworkSpec.from_network(net, dtype=getattr(torch, dtype))


@pytest.mark.parametrize("net,method,code", [
    (W.Network([2, 2], [3, 3, 4, 3], [(0, 2), (1, 3)]), 1, -2),            # n_u != n_v
    (W.Network([2, 1], [3, 3, 3], [(0, 2), (1, 2)]), 1, -3),               # mode 2 twice
    (W.Network([2, 2], [3, 3, 3, 3], [(0, 2)]), 1, -6),                    # free modes
    (W.Network([2, 1], [3, 3, 3], [(0, 0)]), 1, -1),                       # u == v
    (W.Network([2, 2], [3, 3, 3, 3], [(0, 2), (1, 3)]), 2, -5),            # double bond: cycle
    (W.Network([2], [3, 3], [(0, 1)]), 2, -4),                             # trace: self-loop
])
def test_validation_codes(T, net, method, code):
    with pytest.raises(T.TNError) as ei:
        T.tn_sketch_plan([_spec(T, net)], method, 16, 4, 0)
    assert ei.value.code == code
    assert T.tn_last_error()


def test_argument_codes(T):
    net = W.triangle(4)
    s = _spec(T, net, "float64")
    for m in (3, 100):          # m <= 0 asks the plan to choose m (tested on the GPU)
        with pytest.raises(T.TNError) as ei:
            T.tn_sketch_plan([s], 1, m, 4, 0)
        assert ei.value.code == T.TN_ERR_ARG
    with pytest.raises(T.TNError) as ei:  # sizing flags only with m <= 0, and not both
        T.tn_sketch_plan([s], 1, 16, 4, 0, flags=T.TN_FLAG_SIZE_PILOT)
    assert ei.value.code == T.TN_ERR_ARG
    with pytest.raises(T.TNError) as ei:
        T.tn_sketch_plan([s], 1, 0, 4, 0, flags=T.TN_FLAG_SIZE_PILOT | T.TN_FLAG_SIZE_LEARNED)
    assert ei.value.code == T.TN_ERR_ARG
    with pytest.raises(T.TNError) as ei:
        T.tn_sketch_plan([s], 1, 16, 0, 0)
    assert ei.value.code == T.TN_ERR_ARG
    with pytest.raises(T.TNError) as ei:
        T.tn_sketch_plan([s], 3, 16, 4, 0)
    assert ei.value.code == T.TN_ERR_ARG
    with pytest.raises(T.TNError) as ei:
        T.tn_sketch_plan([s], 1, 16, 4, 0, flags=0x40000000)
    assert ei.value.code == T.TN_ERR_ARG
    big = W.Network([1, 1], [1 << 21, 1 << 21], [(0, 1)])
    with pytest.raises(T.TNError) as ei:
        T.tn_sketch_plan([_spec(T, big)], 1, 16, 4, 0)
    assert ei.value.code == T.TN_ERR_UNSUPPORTED
    # a second network of another dtype
    with pytest.raises(T.TNError) as ei:
        T.tn_sketch_plan([s, _spec(T, net, "float32")], 1, 16, 4, 0)
    assert ei.value.code == T.TN_ERR_ARG


def test_exact_validation(T):
    with pytest.raises(T.TNError) as ei:
        T.tn_contract_exact(_spec(T, W.Network([2, 2], [3, 3, 3, 3], [(0, 2)])))
    assert ei.value.code == T.TN_ERR_PARTIAL


def test_binding_rejects_bad_buffers(T):
    """The C ABI trusts the device pointers and sizes it is given; the binding
    checks them before any call: host tensors, tensors whose entry count is not
    the product of their mode sizes, wrong dtypes and non-contiguous views are
    refused with ValueError (no device work is queued)."""
    import torch
    net = W.triangle(4)
    with pytest.raises(ValueError, match="entries"):
        T.NetworkSpec.from_network(net, [torch.zeros(16, dtype=torch.float64),
                                         torch.zeros(15, dtype=torch.float64),
                                         torch.zeros(16, dtype=torch.float64)])
    with pytest.raises(ValueError, match="device"):
        T.NetworkSpec.from_network(net, [torch.zeros(4, 4, dtype=torch.float64) for _ in range(3)])
    with pytest.raises(ValueError, match="dtype"):
        T.NetworkSpec.from_network(net, [torch.zeros(4, 4, dtype=torch.float64),
                                         torch.zeros(4, 4, dtype=torch.float32),
                                         torch.zeros(4, 4, dtype=torch.float64)])
    with pytest.raises(ValueError, match="contiguous"):
        T.NetworkSpec.from_network(net, [torch.zeros(4, 4, dtype=torch.float64).t() if k == 1 else
                                         torch.zeros(4, 4, dtype=torch.float64) for k in range(3)])
    from paper_2603_07387_amd._binding import _device_buffer
    with pytest.raises(ValueError, match="at least"):
        _device_buffer(torch.zeros(3, dtype=torch.float64), torch.float64, 4, "stats")
    with pytest.raises(ValueError, match="device"):
        _device_buffer(torch.zeros(4, dtype=torch.float64), torch.float64, 4, "stats")
    with pytest.raises(ValueError):
        T.median_of_means(torch.zeros(2, 8, dtype=torch.float64), 2)


def test_regressor_file_rejections(T, tmp_path):
    """tn_mlp_load refuses, before any device work, a file that is not a
    regressor file, one with a bad header, and one larger than the largest
    legal file (it stops reading there)."""
    junk = tmp_path / "junk.bin"
    junk.write_bytes(b"not a regressor file at all" * 4)
    with pytest.raises(T.TNError) as e:
        T.tn_mlp_load(str(junk))
    assert e.value.code == T.TN_ERR_ARG
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"TNMLP\0\0\1" + (7).to_bytes(4, "little") + bytes(40))
    with pytest.raises(T.TNError) as e:
        T.tn_mlp_load(str(bad))
    assert e.value.code == T.TN_ERR_ARG and "header" in str(e.value)
    big = tmp_path / "big.bin"
    with open(big, "wb") as f:
        f.write(b"TNMLP\0\0\1")
        f.truncate(300 << 20)  # sparse: no disk blocks
    with pytest.raises(T.TNError) as e:
        T.tn_mlp_load(str(big))
    assert e.value.code == T.TN_ERR_ARG and "too large" in str(e.value)


def test_tn_log_levels(T, capfd, monkeypatch):
    """TN_LOG=1 prints the size choice of an auto-sized plan (made on the host,
    before any device work) as one "[tn] size: ..." line on stderr; unset, the
    library prints nothing."""
    spec = _spec(T, W.triangle(16))

    def attempt():
        try:
            h = T.tn_sketch_plan([spec], 1, 0, 0, 0)
            T.tn_plan_destroy(h)
        except T.TNError:
            pass  # no device here: the plan stops after choosing its size

    monkeypatch.delenv("TN_LOG", raising=False)
    attempt()
    assert "[tn]" not in capfd.readouterr().err
    monkeypatch.setenv("TN_LOG", "1")
    attempt()
    err = capfd.readouterr().err
    assert "[tn] size: bound variance, eps 0.01, delta 0.25, 1 networks: m " in err, err
