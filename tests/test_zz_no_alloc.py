"""The allocation-free entry point tn_tensor_stats_noalloc against the
allocating tn_tensor_stats, through the C ABI: the same kernel in the same
order, so the statistics must agree bit for bit (counts exactly).  Two calls
in a row share the library's fixed device scratch, the second with fewer
tensors (a stale tail of the first must not leak into it); then the two entry
points alternate."""
import numpy as np
import pytest

import tn_workloads as W

pytestmark = pytest.mark.gpu


def _specs(T, nets, dtype):
    import torch
    td = getattr(torch, dtype)
    return [T.NetworkSpec.from_network(n, [torch.from_numpy(np.ascontiguousarray(x)).to("cuda", td)
                                           for x in n.data]) for n in nets]


@pytest.mark.parametrize("dtype", ["float32", "float64", "bfloat16"])
def test_noalloc_matches_allocating(dtype):
    import torch
    import paper_2603_07387_amd as T
    assert torch.cuda.is_available()
    T.load()
    big = _specs(T, W.random_batch(count=300, seed=4), dtype)          # about 2,200 tensors
    small = _specs(T, [W.triangle(16, seed=3), W.torus(L=2, D=8, seed=5)], dtype)
    for specs in (big, small, big[:7], small):
        ref = T.tn_tensor_stats(specs)
        got = T.tn_tensor_stats_noalloc(specs)
        assert got.shape == ref.shape
        assert np.array_equal(got, ref)
        assert np.array_equal(got[:, 3], np.round(got[:, 3]))


def test_noalloc_limit():
    """More tensors than the fixed scratch holds: TN_ERR_UNSUPPORTED before any
    device work, and the next call still works."""
    import torch
    import paper_2603_07387_amd as T
    T.load()
    one = _specs(T, [W.Network([1, 1], [4, 4], [(0, 1)], [np.arange(4.0), np.ones(4)])], "float64")
    with pytest.raises(T.TNError) as e:
        T.tn_tensor_stats_noalloc(one * 16385)
    assert e.value.code == T.TN_ERR_UNSUPPORTED
    got = T.tn_tensor_stats_noalloc(one)
    assert np.array_equal(got, np.array([[6.0, 14.0, 6.0, 4.0], [4.0, 4.0, 4.0, 4.0]]))
