"""GPU parity of the quicksort built on the partition against the oracle's sort."""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_partition import gen, to_device, to_host

pytestmark = pytest.mark.gpu


def _check_sorted(ss, a0):
    t = to_device(a0)
    st = ss.quicksort(t, stats=True)
    out = to_host(t, a0)
    ref = a0.copy()
    oracle.quicksort(ref)
    if a0.ndim == 2:
        assert np.array_equal(out[:, 0], ref[:, 0])          # the key sequence is unique
        assert oracle.is_sorted(out)
        # records intact: same multiset of (key, payload)
        o = out[np.lexsort((out[:, 1], out[:, 0]))]
        r = ref[np.lexsort((ref[:, 1], ref[:, 0]))]
        assert np.array_equal(o, r)
    else:
        assert np.array_equal(out, ref)
    return st


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_quicksort_sizes(ss, kind):
    for n in (0, 1, 2, 3, 17, 1000, 8191, 8192, 8193, 16384, 16385, 40000, 100003, 1 << 20):
        _check_sorted(ss, gen(kind, n, 40 + n))


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_quicksort_duplicates_and_orders(ss, kind):
    n = 300001
    base = gen(kind, n, 12)
    keys = base[:, 0] if base.ndim == 2 else base
    top = np.iinfo(keys.dtype).max
    variants = {
        "few": keys % 3,
        "one_value": np.zeros_like(keys) + 5,
        "max_key": np.full_like(keys, top),
        "two_values_with_max": np.where(keys % 2 == 0, top, 0).astype(keys.dtype),
        "ascending": np.sort(keys),
        "descending": np.sort(keys)[::-1].copy(),
        "few_distinct_1024": (workloads.keys_few_distinct_u32(n, 3, 1024).astype(keys.dtype)),
        # periodic inputs whose period divides the pivot's sample spacing: every sampled key
        # of a segment can be equal, so the pivot is extreme and only the key <= p pass progresses
        "period_64": (np.arange(n) % 64).astype(keys.dtype),
        "period_4096_sawtooth": (np.arange(n) % 4096).astype(keys.dtype) * 1000003,
        "organ_pipe": np.minimum(np.arange(n), n - 1 - np.arange(n)).astype(keys.dtype),
    }
    for name, k in variants.items():
        a0 = base.copy()
        if a0.ndim == 2:
            a0[:, 0] = k
        else:
            a0[:] = k
        _check_sorted(ss, a0)


def test_quicksort_parity_2p26_u32(ss):
    for a0 in (workloads.keys_u32(1 << 26, workloads.config_seed(2)),
               workloads.keys_few_distinct_u32(1 << 26, workloads.config_seed(2), 1024)):
        st = _check_sorted(ss, a0)
        assert st["levels"] >= 8


def test_quicksort_config_2p28_u32_properties(ss):
    """The sort benchmark shape (2^28 uint32, uniform and 1024 distinct values):
    sorted and the same multiset as the input."""
    import torch
    n = 1 << 28
    for t in (workloads.keys_u32_torch(n, workloads.config_seed(2), "cuda"),
              workloads.keys_few_distinct_u32_torch(n, workloads.config_seed(2), "cuda", 1024)):
        h0 = t.cpu().numpy().view(np.uint32)
        fp = oracle.fingerprint(h0)
        del h0
        ss.quicksort(t)
        h = t.cpu().numpy().view(np.uint32)
        assert oracle.is_sorted(h)
        assert oracle.fingerprint(h) == fp
        del t, h
        torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_sort_segments_and_median3(ss, kind):
    import torch
    rng = np.random.default_rng(4)
    cap = ss.sort_segment_cap({"u32": ss.SS_U32, "u64": ss.SS_U64, "kv": ss.SS_KV16}[kind])
    n = 600000
    data = gen(kind, n, 91)
    lens = rng.integers(1, cap + 1, size=40)
    starts = np.cumsum(np.concatenate([[5], lens[:-1] + rng.integers(0, 50, size=39)])).astype(np.uint64)
    assert int(starts[-1] + lens[-1]) <= n
    t = to_device(data)
    keys = data[:, 0] if data.ndim == 2 else data
    d_piv = torch.empty(len(lens), dtype=torch.int64, device="cuda")
    hp = ss.median3_pivots(t, starts, lens, d_piv)
    for k, (s, l) in enumerate(zip(starts, lens)):
        s, l = int(s), int(l)
        trio = sorted([int(keys[s]), int(keys[s + l // 2]), int(keys[s + l - 1])])
        assert int(hp[k]) == trio[1]
    assert np.array_equal(d_piv.cpu().numpy().view(np.uint64), hp)
    ss.sort_segments(t, starts, lens)
    out = to_host(t, data)
    for s, l in zip(starts, lens):
        s, l = int(s), int(l)
        ref = data[s:s + l].copy()
        oracle.quicksort(ref)
        seg = out[s:s + l]
        if data.ndim == 2:
            assert np.array_equal(seg[:, 0], ref[:, 0])
            # the LDS sort is stable: equal keys keep their input order
            order = np.argsort(data[s:s + l, 0], kind="stable")
            assert np.array_equal(seg, data[s:s + l][order])
        else:
            assert np.array_equal(seg, ref)
    with pytest.raises(ss.SSError):
        ss.sort_segments(t, [0], [cap + 1])


@pytest.mark.parametrize("kind", ["u32", "kv"])
def test_quicksort_lds_engine(ss, kind):
    a0 = gen(kind, 300001, 77)
    t = to_device(a0)
    ss.quicksort(t, engine="lds")
    out = to_host(t, a0)
    ref = a0.copy()
    oracle.quicksort(ref)
    if a0.ndim == 2:
        assert np.array_equal(out[:, 0], ref[:, 0])
        o = out[np.lexsort((out[:, 1], out[:, 0]))]
        r = ref[np.lexsort((ref[:, 1], ref[:, 0]))]
        assert np.array_equal(o, r)
    else:
        assert np.array_equal(out, ref)


def _leaf_inputs(kind, cap, rng):
    """Segments that take each path of the workgroup sort: keys spread evenly
    over a wide span (bucketed, a few keys per bucket), a narrow span of
    repeated values (one key value per bucket, no insertion sort), and a
    dense cluster with a far outlier (a bucket above the insertion limit, so
    the radix sort runs), plus a span just above and just below 4096."""
    dt = np.uint32 if kind == "u32" else np.uint64
    top = np.iinfo(dt).max
    segs = []
    segs.append(rng.integers(0, top, size=cap, dtype=dt, endpoint=True))            # wide, even
    segs.append(rng.integers(0, 100, size=cap - 3, dtype=dt))                        # narrow, repeated
    c = rng.integers(1000, 1064, size=cap // 2 - 1, dtype=dt)                        # dense cluster
    segs.append(np.concatenate([c, np.array([top, 0], dtype=dt), c[::-1]]))          # ... with outliers
    segs.append(rng.integers(7, 7 + 4096, size=cap // 3, dtype=dt))                  # span below 2^12
    segs.append(rng.integers(7, 7 + 4097 * 3, size=cap // 3 + 1, dtype=dt))          # span above 2^12
    segs.append(rng.integers(5, 9, size=17, dtype=dt))                               # tiny
    return segs


@pytest.mark.parametrize("kind", ["u32", "u64"])
def test_sort_segments_leaf_paths(ss, kind):
    rng = np.random.default_rng(12)
    cap = ss.sort_segment_cap(ss.SS_U32 if kind == "u32" else ss.SS_U64)
    segs = _leaf_inputs(kind, cap, rng)
    gap = 13
    starts, pos = [], 3
    for s in segs:
        starts.append(pos)
        pos += len(s) + gap
    data = np.zeros(pos, dtype=segs[0].dtype)
    data[:] = rng.integers(0, 1 << 30, size=pos).astype(data.dtype)
    for st, s in zip(starts, segs):
        data[st:st + len(s)] = s
    t = to_device(data)
    ss.sort_segments(t, np.array(starts, dtype=np.uint64), np.array([len(s) for s in segs], dtype=np.uint64))
    out = to_host(t, data)
    expect = data.copy()
    for st, s in zip(starts, segs):
        ref = s.copy()
        oracle.quicksort(ref)
        expect[st:st + len(s)] = ref
    assert np.array_equal(out, expect)   # sorted segments, untouched gaps
