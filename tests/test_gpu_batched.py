"""GPU parity of the batched partition: every array against the oracle, and
identical bytes for an array partitioned alone and inside a batch."""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_partition import to_device, to_host

pytestmark = pytest.mark.gpu


def _batch(kind, lengths, seed):
    n = int(np.sum(lengths))
    if kind == "u32":
        data = workloads.keys_u32(n, seed)
    elif kind == "u64":
        data = workloads.keys_u64(n, seed)
    else:
        data = workloads.records_kv(n, seed)
    offsets = np.zeros(len(lengths) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(lengths)
    qs = workloads.uniform_quantiles(len(lengths), seed)
    pivots = np.zeros(len(lengths), dtype=np.uint64)
    for k in range(len(lengths)):
        a, b = int(offsets[k]), int(offsets[k + 1])
        pivots[k] = workloads.pivot_at_quantile_np(data[a:b], qs[k]) if b > a else 0
    return data, offsets, pivots


def _run_batched(ss, data, offsets, pivots, **kw):
    import torch
    t = to_device(data)
    pv = torch.from_numpy(pivots.view(np.int64).copy()).cuda()
    sp = torch.full((len(pivots),), -7, dtype=torch.int64, device="cuda")
    st = ss.partition_batched(t, offsets, pv, sp, stats=True, **kw)
    return to_host(t, data), sp.cpu().numpy().view(np.uint64), st


def _check(data, out, offsets, pivots, splits):
    for k in range(len(pivots)):
        a, b = int(offsets[k]), int(offsets[k + 1])
        ref = data[a:b].copy()
        rs = oracle.partition(ref, int(pivots[k]))
        assert int(splits[k]) == rs, (k, int(splits[k]), rs)
        gl, gr = oracle.sorted_sides(out[a:b], rs)
        rl, rr = oracle.sorted_sides(ref, rs)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr), k


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_batched_uneven_lengths(ss, kind):
    rng = np.random.default_rng(5)
    lengths = np.concatenate([[0, 1, 2, 63, 64, 65, 0, 4095, 16384, 16385],
                              workloads.lognormal_lengths(300, 9, median_log2=12.0, sigma_log2=1.5, lo=1, hi=1 << 19),
                              [1 << 20, (1 << 20) + 3, 7]]).astype(np.int64)
    data, offsets, pivots = _batch(kind, lengths, 3)
    out, splits, st = _run_batched(ss, data, offsets, pivots)
    _check(data, out, offsets, pivots, splits)
    assert st["levels"] >= 1


def test_batched_same_bytes_alone_and_in_mix(ss):
    lengths = workloads.lognormal_lengths(200, 21, median_log2=13.0)
    data, offsets, pivots = _batch("u64", lengths, 8)
    out_mix, splits_mix, _ = _run_batched(ss, data, offsets, pivots)
    for k in (0, 17, 99, 199):
        a, b = int(offsets[k]), int(offsets[k + 1])
        alone = data[a:b].copy()
        out_alone, splits_alone, _ = _run_batched(ss, alone, np.array([0, b - a], dtype=np.uint64), pivots[k:k + 1])
        assert int(splits_alone[0]) == int(splits_mix[k])
        assert np.array_equal(out_alone, out_mix[a:b])


def test_batched_unaligned_starts_and_tiles(ss):
    lengths = np.array([5, 100003, 3, 70001, 1, 1 << 18, 33, 9999], dtype=np.int64)
    data, offsets, pivots = _batch("u64", lengths, 4)
    for tile in (32768, 65536, 131072):
        for b in (16, 64):
            out, splits, _ = _run_batched(ss, data, offsets, pivots, tile_bytes=tile, b=b, engine="regs")
            _check(data, out, offsets, pivots, splits)


def test_batched_config_shape_properties(ss):
    """The batched benchmark shape (20,000 log-normal arrays around 2^14): for every
    array the split equals the oracle's count, the array is partitioned and its own
    multiset fingerprint is unchanged (so no element moved between arrays)."""
    lengths = workloads.lognormal_lengths(20000, workloads.config_seed(3))
    data, offsets, pivots = _batch("u64", lengths, workloads.config_seed(3))
    out, splits, st = _run_batched(ss, data, offsets, pivots)
    for k in range(20000):
        a, b = int(offsets[k]), int(offsets[k + 1])
        assert int(splits[k]) == oracle.count_less(data[a:b], int(pivots[k])), k
        assert oracle.is_partitioned(out[a:b], int(pivots[k]), int(splits[k])), k
        assert oracle.fingerprint(out[a:b]) == oracle.fingerprint(data[a:b]), k
    # sampled arrays element by element: both sides' sorted contents equal the oracle's
    for k in range(0, 20000, 97):
        a, b = int(offsets[k]), int(offsets[k + 1])
        ref = data[a:b].copy()
        rs = oracle.partition(ref, int(pivots[k]))
        gl, gr = oracle.sorted_sides(out[a:b], rs)
        rl, rr = oracle.sorted_sides(ref, rs)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr), k


def test_segments_any_order_with_gaps(ss):
    import torch
    rng = np.random.default_rng(2)
    n = 400000
    data = workloads.keys_u64(n, 77)
    # disjoint segments with gaps, given out of order
    cuts = np.sort(rng.choice(np.arange(1, n), size=120, replace=False))
    bounds = np.concatenate([[0], cuts, [n]])
    segs = [(int(bounds[i]) + 3, int(bounds[i + 1] - bounds[i]) - 3) for i in range(len(bounds) - 1)
            if bounds[i + 1] - bounds[i] > 3]
    order = rng.permutation(len(segs))
    starts = np.array([segs[i][0] for i in order], dtype=np.uint64)
    lens = np.array([segs[i][1] for i in order], dtype=np.uint64)
    pivots = np.array([workloads.pivot_at_quantile_np(data[s:s + l], 0.3) for s, l in zip(starts, lens)],
                      dtype=np.uint64)
    t = to_device(data)
    pv = torch.from_numpy(pivots.view(np.int64).copy()).cuda()
    sp = torch.empty(len(starts), dtype=torch.int64, device="cuda")
    ss.partition_segments(t, starts, lens, pv, sp)
    out = to_host(t, data)
    splits = sp.cpu().numpy().view(np.uint64)
    covered = np.zeros(n, dtype=bool)
    for k, (s, l) in enumerate(zip(starts, lens)):
        s, l = int(s), int(l)
        covered[s:s + l] = True
        ref = data[s:s + l].copy()
        rs = oracle.partition(ref, int(pivots[k]))
        assert int(splits[k]) == rs
        gl, gr = oracle.sorted_sides(out[s:s + l], rs)
        rl, rr = oracle.sorted_sides(ref, rs)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr)
    assert np.array_equal(out[~covered], data[~covered])   # the gaps are untouched


def test_segments_reject_overlap(ss):
    import torch
    t = to_device(workloads.keys_u64(1000, 1))
    pv = torch.zeros(2, dtype=torch.int64, device="cuda")
    sp = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(ss.SSError):
        ss.partition_segments(t, [0, 50], [100, 100], pv, sp)


@pytest.mark.parametrize("kind", ["u64", "kv"])
def test_batched_graph_replays_match_eager(ss, kind):
    """The level chain replayed from a captured HIP graph gives the eager call's
    bytes on every replay, with eager work and synchronizations in between."""
    import torch
    lengths = np.concatenate([[0, 1, 5, 16385],
                              workloads.lognormal_lengths(200, 4, median_log2=12.0, sigma_log2=1.5, lo=1,
                                                          hi=1 << 18)]).astype(np.int64)
    data, offsets, pivots = _batch(kind, lengths, 8)
    eager_out, eager_splits, _ = _run_batched(ss, data, offsets, pivots)
    _check(data, eager_out, offsets, pivots, eager_splits)
    pristine = to_device(data)
    t = pristine.clone()
    pv = torch.from_numpy(pivots.view(np.int64).copy()).cuda()
    sp = torch.empty((len(pivots),), dtype=torch.int64, device="cuda")
    for rep in range(4):
        t.copy_(pristine)
        sp.fill_(-7)
        noise = torch.randn(1 << 16, device="cuda").sum()      # unrelated eager work between replays
        ss.partition_batched(t, offsets, pv, sp, graph=True)
        torch.cuda.synchronize()
        assert torch.isfinite(noise)
        assert np.array_equal(sp.cpu().numpy().view(np.uint64), eager_splits), rep
        assert np.array_equal(to_host(t, data), eager_out), rep


def test_size_class_tables_keep_parity(ss):
    """Per-class line and group sizes change the work, never the result."""
    table = {"classes": [{"max_len": 1 << 10, "b": 16, "group_bytes": 32768},
                         {"max_len": 1 << 14, "b": 32, "group_bytes": 65536},
                         {"max_len": 1 << 62, "b": 128, "group_bytes": 131072}]}
    try:
        ss.set_batched_tuning("u64", table)
        got = ss.get_batched_tuning("u64")["classes"]
        assert [(c["b"], c["group_bytes"]) for c in got] == [(16, 32768), (32, 65536), (128, 131072)]
        assert got[-1]["max_len"] == (1 << 64) - 1                 # the last class is unbounded
        lengths = np.concatenate([[0, 1, 1000, 1024, 1025, 16384, 16385, 70000],
                                  workloads.lognormal_lengths(200, 2, median_log2=13.0, sigma_log2=2.0, lo=1,
                                                              hi=1 << 19)]).astype(np.int64)
        data, offsets, pivots = _batch("u64", lengths, 6)
        out, splits, st = _run_batched(ss, data, offsets, pivots)
        _check(data, out, offsets, pivots, splits)
        for bad in ({"classes": [{"max_len": 5, "b": 3, "group_bytes": 32768}]},
                    {"classes": [{"max_len": 5, "b": 16, "group_bytes": 262144}]},
                    {"classes": [{"max_len": 9, "b": 16, "group_bytes": 32768},
                                 {"max_len": 5, "b": 16, "group_bytes": 32768}]}):
            with pytest.raises(ss.SSError):
                ss.set_batched_tuning("u64", bad)
    finally:
        ss.set_batched_tuning("u64", None)
    assert ss.get_batched_tuning("u64")["classes"][0]["group_bytes"] == 131072


@pytest.mark.parametrize("kind", ["u32", "kv"])
def test_autotune_installs_a_table_that_keeps_parity(ss, kind):
    try:
        t = ss.autotune_batched(kind)
        assert len(t["classes"]) == 7
        assert all(c["ms"] > 0 for c in t["classes"])
        assert ss.get_batched_tuning(kind)["classes"] == [{**c, "ms": 0.0} for c in t["classes"]]
        lengths = workloads.lognormal_lengths(400, 12, median_log2=13.0, sigma_log2=2.0, lo=1, hi=1 << 20)
        data, offsets, pivots = _batch(kind, lengths.astype(np.int64), 13)
        out, splits, _ = _run_batched(ss, data, offsets, pivots)
        _check(data, out, offsets, pivots, splits)
        # the table is measured on the register body; 4-byte keys use it when asked for that body
        out, splits, _ = _run_batched(ss, data, offsets, pivots, engine="regs")
        _check(data, out, offsets, pivots, splits)
    finally:
        ss.set_batched_tuning(kind, None)


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
@pytest.mark.parametrize("tile", [32768, 65536])
def test_batched_lds_engine_parity(ss, kind, tile):
    """The LDS-tile group body gives the register body's bytes (same stable partition of every group)."""
    lengths = np.concatenate([[0, 1, 2, 65, 4095, 16385],
                              workloads.lognormal_lengths(150, 21, median_log2=12.0, sigma_log2=1.5, lo=1,
                                                          hi=1 << 18)]).astype(np.int64)
    data, offsets, pivots = _batch(kind, lengths, 17)
    out, splits, _ = _run_batched(ss, data, offsets, pivots, engine="lds", tile_bytes=tile)
    _check(data, out, offsets, pivots, splits)
    out_r, splits_r, _ = _run_batched(ss, data, offsets, pivots, engine="regs", tile_bytes=tile)
    assert np.array_equal(splits, splits_r) and np.array_equal(out, out_r)


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_partition_each_matches_oracle_and_single_calls(ss, kind):
    """The per-array loop issued from C: every array's split and sides equal the
    oracle's, and its bytes equal a separate single-array call's (arrays that fit
    one group take the single-launch path, longer ones the planned chain)."""
    import torch
    lengths = np.concatenate([[0, 1, 2, 63, 64, 65, 4095, 16384, 16385, 70001],
                              workloads.lognormal_lengths(120, 19, median_log2=12.0, sigma_log2=1.5, lo=1,
                                                          hi=1 << 19),
                              [1 << 20, 7]]).astype(np.int64)
    data, offsets, pivots = _batch(kind, lengths, 13)
    t = to_device(data)
    sp = torch.full((len(pivots),), -7, dtype=torch.int64, device="cuda")
    lat = ss.partition_each(t, offsets, [int(x) for x in pivots], sp, latencies=True)
    out = to_host(t, data)
    splits = sp.cpu().numpy().view(np.uint64)
    _check(data, out, offsets, pivots, splits)
    assert lat.shape == (len(pivots),) and np.all(np.diff(lat) >= 0) and lat[-1] > 0
    for k in (0, 3, 7, 9, len(pivots) - 2):
        a, b = int(offsets[k]), int(offsets[k + 1])
        one = to_device(data[a:b].copy())
        s1 = ss.partition(one, int(pivots[k])) if b > a else 0
        assert s1 == int(splits[k])
        assert np.array_equal(to_host(one, data[a:b]), out[a:b]), k
    # without latencies the call does not synchronize; the splits land on the stream
    t2 = to_device(data)
    sp2 = torch.full((len(pivots),), -7, dtype=torch.int64, device="cuda")
    ss.partition_each(t2, offsets, [int(x) for x in pivots], sp2)
    torch.cuda.synchronize()
    assert np.array_equal(sp2.cpu().numpy().view(np.uint64), splits)
    assert np.array_equal(to_host(t2, data), out)
