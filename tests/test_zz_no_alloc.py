"""GPU check of ss_partition_noalloc (the entry point that allocates nothing):
through the C ABI, its output equals ss_partition_ex's (same split, same bytes)
on calls in a row, the second on a smaller input, and the split equals the
oracle's count."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from test_gpu_partition import gen, to_device, to_host

pytestmark = pytest.mark.gpu


def _noalloc(ss, t, pivot, **kw):
    import torch
    d = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    ss.partition_noalloc(t, pivot, d, **kw)
    return d


@pytest.mark.parametrize("kind", ["u64", "u32", "kv"])
def test_noalloc_equals_partition_ex_on_calls_in_a_row(ss, kind):
    import torch
    cases = ((1 << 23) + 1234, 50001, 3000, 0)  # each smaller than the one before; the last two fit one group
    for n, seed in zip(cases, (71, 72, 73, 74)):
        a0 = gen(kind, n, seed)
        p = workloads.pivot_at_quantile_np(a0, 0.37) if n else 5
        t1 = to_device(a0)
        d1 = _noalloc(ss, t1, p)
        t2 = to_device(a0)
        d2 = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        ss.partition_async(t2, p, d2)
        torch.cuda.synchronize()
        split = int(d1.item())
        assert split == int(d2.item()) == oracle.count_less(a0, p), (kind, n)
        assert np.array_equal(to_host(t1, a0), to_host(t2, a0)), (kind, n)


def test_noalloc_skewed_pivot_and_strided(ss):
    import torch
    a0 = workloads.keys_u64((1 << 22) + 5, 75)   # the automatic exchange choice applies from 2^22 on
    for kw, q in (({}, 0.02), ({"algo": "strided"}, 0.5), ({"exchange": False}, 0.5)):
        p = workloads.pivot_at_quantile_np(a0, q)
        t1 = to_device(a0)
        d1 = _noalloc(ss, t1, p, **kw)
        t2 = to_device(a0)
        d2 = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        ss.partition_async(t2, p, d2, **kw)
        torch.cuda.synchronize()
        assert int(d1.item()) == int(d2.item()) == oracle.count_less(a0, p), kw
        assert np.array_equal(to_host(t1, a0), to_host(t2, a0)), kw


def test_noalloc_rejects_beyond_its_limit(ss):
    import torch
    t = to_device(workloads.keys_u64(1000, 76))
    d = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    p = ss.make_params(max_levels=17)
    rc = ss.lib.ss_partition_noalloc(ctypes.c_void_p(t.data_ptr()), 1000, ss.SS_U64, 5, ctypes.byref(p), None,
                                     ctypes.c_void_p(d.data_ptr()))
    assert rc == -1 and b"16" in ss.lib.ss_last_error()
    p = ss.make_params(time=True)
    rc = ss.lib.ss_partition_noalloc(ctypes.c_void_p(t.data_ptr()), 1000, ss.SS_U64, 5, ctypes.byref(p), None,
                                     ctypes.c_void_p(d.data_ptr()))
    assert rc == -1
    assert int(d.item()) == -7  # untouched on argument errors
