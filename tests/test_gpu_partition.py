"""GPU parity of the Smoothed Striding / Strided partition against the CPU oracle.

Every case generates its input on the host from the shared seeded generator,
copies it to the device, runs the library through its C ABI, and compares
with the oracle run on the same input: the split index exactly and the sorted
contents of both sides exactly (the arrangement inside a side is not unique).
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

U64MAX = (1 << 64) - 1


def _torch():
    import torch
    return torch


def to_device(a: np.ndarray):
    torch = _torch()
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32).copy()).cuda()
    return torch.from_numpy(a.view(np.int64).copy()).cuda()


def to_host(t, like: np.ndarray) -> np.ndarray:
    h = t.cpu().numpy()
    return h.view(like.dtype).reshape(like.shape)


def gen(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "u32":
        return workloads.keys_u32(n, seed)
    if kind == "u64":
        return workloads.keys_u64(n, seed)
    return workloads.records_kv(n, seed)


def check_against_oracle(ss, a0: np.ndarray, pivot: int, **kw):
    t = to_device(a0)
    split = ss.partition(t, pivot, **kw)
    out = to_host(t, a0)
    ref = a0.copy()
    rsplit = oracle.partition(ref, pivot)
    assert split == rsplit, (split, rsplit)
    gl, gr = oracle.sorted_sides(out, split)
    rl, rr = oracle.sorted_sides(ref, rsplit)
    assert np.array_equal(gl, rl) and np.array_equal(gr, rr)
    assert oracle.is_partitioned(out, pivot, split)
    return out, split


def test_config1_median_u64(ss):
    # 2^20 uint64 keys, exact median pivot, 128-byte lines (b = 16)
    a0 = workloads.keys_u64(1 << 20, workloads.config_seed(0))
    p = workloads.pivot_at_quantile_np(a0, 0.5)
    out, split = check_against_oracle(ss, a0, p, b=16)
    assert split == 1 << 19


SIZES = [1, 2, 3, 15, 16, 17, 31, 127, 128, 129, 1000, 8191, 8192, 8193, 16385, 65535, 65537, 100003, 300001]


ENGINES = ["lds", "regs", "staged"]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_shapes_and_pivots(ss, kind, engine):
    for n in SIZES:
        a0 = gen(kind, n, 1000 + n)
        keys = a0[:, 0] if a0.ndim == 2 else a0
        kmin, kmax = int(keys.min()), int(keys.max())
        pivots = {0, kmin, kmin + 1, kmax, kmax + 1, U64MAX, workloads.pivot_at_quantile_np(a0, 0.5),
                  workloads.pivot_at_quantile_np(a0, 0.01)}
        if kind == "u32":
            pivots |= {1 << 32, (1 << 32) - 1}
        for p in sorted(pivots):
            check_against_oracle(ss, a0, p, engine=engine)


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_duplicates_and_structured_inputs(ss, kind):
    n = 70001
    base = gen(kind, n, 5)
    keys = base[:, 0] if base.ndim == 2 else base
    variants = {
        "few": keys % 7,
        "equal": np.zeros_like(keys) + 3,
        "ascending": np.sort(keys),
        "descending": np.sort(keys)[::-1].copy(),
    }
    for name, k in variants.items():
        a0 = base.copy()
        if a0.ndim == 2:
            a0[:, 0] = k
        else:
            a0[:] = k
        for q in (0.0, 0.3, 0.5, 0.99):
            check_against_oracle(ss, a0, workloads.pivot_at_quantile_np(a0, q))


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_unaligned_subarrays(ss, kind, engine):
    # Sub-tensors starting at every element offset inside a 128-byte line.
    torch = _torch()
    n = 50000
    full = gen(kind, n + 64, 77)
    t_full = to_device(full)
    for off in range(0, 33):
        if off + 1000 > n:
            break
        length = n - off - (off * 37) % 500
        sub_host = full[off:off + length].copy()
        p = workloads.pivot_at_quantile_np(sub_host, 0.4)
        t = t_full.clone()
        view = t[off:off + length]
        assert view.is_contiguous()
        split = ss.partition(view, p, engine=engine)
        out = to_host(t, full)
        # outside the sub-array nothing changed
        assert np.array_equal(out[:off], full[:off]) and np.array_equal(out[off + length:], full[off + length:])
        ref = sub_host.copy()
        assert split == oracle.partition(ref, p)
        gl, gr = oracle.sorted_sides(out[off:off + length], split)
        rl, rr = oracle.sorted_sides(ref, split)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr)


def _group_of_position(n, b, g, s, X):
    line = np.arange((n + b - 1) // b)
    j = line // g
    r = line % g
    grp = (r - X[j].astype(np.int64)) % g
    return np.repeat(grp, b)[:n]


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
@pytest.mark.parametrize("algo", ["smoothed", "strided"])
def test_one_level_matches_oracle_level(ss, kind, algo, engine):
    """One Partial Partition Step: (v_min, v_max), the side of every position and
    the multiset of every group equal the oracle's step with the same offsets."""
    for n, seed, q in ((1 << 18, 1, 0.5), (123457, 2, 0.1), (300000, 3, 0.9), (40000, 4, 0.5)):
        a0 = gen(kind, n, seed)
        p = workloads.pivot_at_quantile_np(a0, q)
        t = to_device(a0)
        split, st = ss.partition(t, p, stats=True, one_level=True, algo=algo, seed=1234 + seed, engine=engine)
        out = to_host(t, a0)
        g, s, b = st["level_g"][0], st["level_s"][0], st["b"]
        assert st["level_lo"][0] == 0 and st["level_hi"][0] == n
        assert g >= 2
        assert s * g * b >= n > (s - 1) * g * b
        X = np.zeros(s, np.uint32) if algo == "strided" else oracle.ss_offsets(1234 + seed, 0, g, s)
        ref = a0.copy()
        vmin, vmax, c, v = oracle.ss_partial_step(ref, b, g, s, X, p)
        assert (st["vmin"], st["vmax"]) == (vmin, vmax)
        gk = out[:, 0] if out.ndim == 2 else out
        rk = ref[:, 0] if ref.ndim == 2 else ref
        assert np.array_equal(gk < p, rk < p)
        grp = _group_of_position(n, b, g, s, X)
        order_g = np.lexsort((gk, grp))
        order_r = np.lexsort((rk, grp))
        assert np.array_equal(gk[order_g], rk[order_r])


def test_same_seed_same_bytes_and_other_seeds_correct(ss):
    a0 = workloads.keys_u64(500000, 9)
    p = workloads.pivot_at_quantile_np(a0, 0.5)
    t1, t2 = to_device(a0), to_device(a0)
    s1 = ss.partition(t1, p, seed=42)
    s2 = ss.partition(t2, p, seed=42)
    assert s1 == s2
    assert bool((t1 == t2).all())
    for sd in (1, 2, 3):
        check_against_oracle(ss, a0, p, seed=sd)


@pytest.mark.parametrize("engine,tile", [("lds", 32768), ("lds", 65536), ("regs", 32768), ("regs", 65536),
                                         ("regs", 131072)])
@pytest.mark.parametrize("line_bytes", [64, 128, 256, 512, 1024, 4096])
def test_tiles_and_line_sizes(ss, engine, tile, line_bytes):
    for kind, w in (("u32", 4), ("u64", 8), ("kv", 16)):
        if line_bytes > tile:
            continue
        a0 = gen(kind, 200003, line_bytes + w)
        p = workloads.pivot_at_quantile_np(a0, 0.37)
        check_against_oracle(ss, a0, p, b=line_bytes // w, tile_bytes=tile, engine=engine)


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_engines_give_identical_bytes(ss, kind):
    """Every workgroup body computes the same stable partition of every group."""
    for n, q, tile in ((1 << 20, 0.5, 32768), (777777, 0.05, 65536), (3001, 0.5, 32768)):
        a0 = gen(kind, n, 55 + n)
        p = workloads.pivot_at_quantile_np(a0, q)
        t1 = to_device(a0)
        s1 = ss.partition(t1, p, engine="lds", tile_bytes=tile, seed=5)
        t2 = to_device(a0)
        s2 = ss.partition(t2, p, engine="regs", tile_bytes=tile, seed=5)
        assert s1 == s2
        assert bool((t1 == t2).all())
        t3 = to_device(a0)
        s3 = ss.partition(t3, p, engine="staged", tile_bytes=tile, seed=5)
        assert s3 == s1
        assert bool((t3 == t1).all())


def test_small_level_budget_ends_in_base_case(ss):
    """With a level budget below the plan, the serial base case partitions the
    larger region the levels leave, asynchronously as well."""
    torch = _torch()
    a0 = workloads.keys_u64(1 << 20, 3)
    p = workloads.pivot_at_quantile_np(a0, 0.5)
    for lv in (1, 2):
        _, split = check_against_oracle(ss, a0, p, max_levels=lv)
        t = to_device(a0)
        split2, st = ss.partition(t, p, stats=True, max_levels=lv)
        assert split2 == split and st["levels"] == lv
        assert st["vmax"] - st["vmin"] > 0  # the base case had a region to finish
        t = to_device(a0)
        d = torch.full((1,), -7, dtype=torch.int64, device="cuda")
        ss.partition_async(t, p, d, max_levels=lv)
        torch.cuda.synchronize()
        assert int(d.item()) == split


def test_planned_levels_leave_small_base_case(ss):
    """The default plan for 2^20 keys leaves the base case a region that one
    or two of its passes finish (parity pinned by the oracle check)."""
    a0 = workloads.keys_u64(1 << 20, 8)
    p = workloads.pivot_at_quantile_np(a0, 0.5)
    check_against_oracle(ss, a0, p)
    t = to_device(a0)
    split, st = ss.partition(t, p, stats=True)
    assert 1 <= st["levels"] <= 4
    assert st["vmax"] - st["vmin"] <= 4 * 8192


def test_async_split_and_empty(ss):
    torch = _torch()
    a0 = workloads.keys_u64(1 << 18, 4)
    p = workloads.pivot_at_quantile_np(a0, 0.25)
    t = to_device(a0)
    d = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    ss.partition_async(t, p, d)
    torch.cuda.synchronize()
    assert int(d.item()) == oracle.count_less(a0, p)
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    assert ss.partition(e, 5) == 0
    assert ss.partition_plain(to_device(a0), p) == oracle.count_less(a0, p)


def test_stats_levels_and_bytes(ss):
    a0 = workloads.keys_u64(1 << 22, 6)
    p = workloads.pivot_at_quantile_np(a0, 0.5)
    t = to_device(a0)
    split, st = ss.partition(t, p, stats=True, time=True)
    assert split == 1 << 21
    assert st["levels"] >= 2 and st["level_lo"][0] == 0 and st["level_hi"][0] == 1 << 22
    for k in range(1, st["levels"]):  # each level works inside the previous one's middle
        assert st["level_lo"][k - 1] <= st["level_lo"][k] < st["level_hi"][k] <= st["level_hi"][k - 1]
    assert st["bytes_moved"] >= 2 * 8 * (1 << 22)
    assert st["first_level_ms"] > 0 and st["total_ms"] >= st["first_level_ms"]
    assert st["aux_bytes"] == ss.aux_bytes(1 << 22, ss.SS_U64)


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_strided_parity(ss, kind):
    for n, q in ((1 << 20, 0.5), (99991, 0.2), (5000, 0.7), (1, 0.5)):
        a0 = gen(kind, n, 31 + n)
        check_against_oracle(ss, a0, workloads.pivot_at_quantile_np(a0, q), algo="strided")


@pytest.mark.slow
@pytest.mark.parametrize("algo,q", [("smoothed", 0.5), ("smoothed", 0.1), ("smoothed", 0.01), ("smoothed", "desc"),
                                    ("strided", 0.5), ("lowspace", 0.5), ("lowspace", 0.1)])
def test_full_size_2p30_properties(ss, algo, q):
    """2^30 uint64 keys, every input of the large single-array workload (pivot at the
    0.5, 0.1 and 0.01 quantiles, and the keys sorted descending with the median
    pivot) with the default call as the benchmark times it, and the Strided and
    Low-Space comparators: the split equals the oracle's count on the host copy,
    every element is on its side, and the multiset is unchanged."""
    torch = _torch()
    n = 1 << 30
    t = workloads.keys_u64_torch(n, workloads.config_seed(1), "cuda")
    p = workloads.pivot_at_quantile_torch(t, 0.5 if q == "desc" else q)
    if q == "desc":
        t = workloads.sort_descending_u64_torch(t)
    host_in = t.cpu().numpy().view(np.uint64)
    if q == "desc":
        assert bool(np.all(host_in[:-1] >= host_in[1:]))
    count = oracle.count_less(host_in, p)
    fp_in = oracle.fingerprint(host_in)
    del host_in
    split, st = ss.partition(t, p, stats=True, algo=algo)
    assert split == count == workloads.quantile_rank(n, 0.5 if q == "desc" else q)
    host_out = t.cpu().numpy().view(np.uint64)
    assert oracle.is_partitioned(host_out, p, split)
    assert oracle.fingerprint(host_out) == fp_in
    if algo == "smoothed":
        assert st["levels"] >= 2
    del t, host_out
    torch.cuda.empty_cache()


@pytest.mark.slow
def test_more_than_2p32_elements_u32(ss):
    """2^32 + 1000 uint32 keys (16 GiB): the 64-bit index paths, with 64-byte lines."""
    torch = _torch()
    n = (1 << 32) + 1000
    t = workloads.keys_u32_torch(n, 99, "cuda")
    pivot = 1 << 31
    host_in = t.cpu().numpy().view(np.uint32)
    count = oracle.count_less(host_in, pivot)
    fp_in = oracle.fingerprint(host_in)
    del host_in
    split, st = ss.partition(t, pivot, stats=True, b=16)
    assert split == count
    host_out = t.cpu().numpy().view(np.uint32)
    assert oracle.is_partitioned(host_out, pivot, split)
    assert oracle.fingerprint(host_out) == fp_in
    del t, host_out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("algo", ["smoothed", "strided", "lowspace"])
def test_stride_adversary_parity(ss, algo):
    """Keys whose predecessors fill exactly the lines l with (l mod g) < g/2."""
    n = (1 << 20) + 77
    g = workloads.stride_groups(n, 64, 256)   # default geometry: 512-byte lines, 256 lines per group
    a0 = workloads.stride_adversarial_u64(n, 8, 64, g)
    check_against_oracle(ss, a0, 1 << 63, algo=algo)


def test_stride_adversary_middle_regions(ss):
    """Section 4's motivation for the random offsets: with every offset 0 each
    stride set of this input is all predecessors or all successors, so one
    Strided step leaves almost the whole array between v_min and v_max; the
    offsets of Smoothed Striding mix every group and leave a fraction of it."""
    n = 1 << 22
    g = workloads.stride_groups(n, 64, 256)
    a0 = workloads.stride_adversarial_u64(n, 9, 64, g)
    mids = {}
    for algo in ("strided", "smoothed"):
        t = to_device(a0)
        _, st = ss.partition(t, 1 << 63, algo=algo, one_level=True, stats=True)
        out = to_host(t, a0)
        assert oracle.fingerprint(out) == oracle.fingerprint(a0)
        mids[algo] = st["vmax"] - st["vmin"]
    assert mids["strided"] > 0.95 * n, mids
    assert mids["smoothed"] < 0.5 * n, mids


XCH_ENGINES = [("regs", 32768), ("regs", 65536), ("regs", 131072)]


@pytest.mark.parametrize("engine,tile", XCH_ENGINES)
@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
@pytest.mark.parametrize("algo", ["smoothed", "strided"])
def test_exchange_level_equals_serial_step(ss, kind, algo, engine, tile):
    """Write-minimal exchange: one Partial Partition Step leaves the array byte for
    byte as the oracle's serial two-pointer step over every group's slot sequence."""
    for n, seed, q in ((1 << 18, 1, 0.5), (123457, 2, 0.1), (300000, 3, 0.99), (40000, 4, 0.01), (5000, 5, 0.5)):
        a0 = gen(kind, n, seed)
        p = workloads.pivot_at_quantile_np(a0, q)
        t = to_device(a0)
        split, st = ss.partition(t, p, stats=True, one_level=True, algo=algo, seed=77 + seed, engine=engine,
                                 tile_bytes=tile, exchange=True)
        out = to_host(t, a0)
        g, s, b = st["level_g"][0], st["level_s"][0], st["b"]
        assert s * g * b >= n > (s - 1) * g * b
        X = np.zeros(s, np.uint32) if algo == "strided" else oracle.ss_offsets(77 + seed, 0, g, s)
        ref = a0.copy()
        vmin, vmax, c, v = oracle.ss_partial_step(ref, b, g, s, X, p)
        assert (st["vmin"], st["vmax"]) == (vmin, vmax)
        assert np.array_equal(out, ref), (n, q)


@pytest.mark.parametrize("mode", [True, "skewed"])
@pytest.mark.parametrize("engine,tile", XCH_ENGINES)
@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_exchange_parity(ss, kind, engine, tile, mode):
    """The whole recursion with the exchange form (every group, or only the skewed
    ones): split and sides equal the oracle's."""
    for n in (1, 2, 15, 16, 17, 127, 129, 8193, 65537, 300001, 1 << 20):
        a0 = gen(kind, n, 2000 + n)
        for q in (0.0, 0.01, 0.03, 0.1, 0.5, 0.97, 1.0):
            p = workloads.pivot_at_quantile_np(a0, q) if q < 1.0 else U64MAX
            check_against_oracle(ss, a0, p, engine=engine, tile_bytes=tile, exchange=mode)


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_skewed_exchange_level_groups(ss, kind):
    """Skewed mode, one level: each group is either exchanged or stably partitioned,
    so (v_min, v_max), the side of every position and every group's multiset equal
    the oracle's step; an already partitioned input is left byte for byte as it was."""
    for n, seed, q in ((1 << 18, 1, 0.5), (300000, 3, 0.02), (123457, 2, 0.97)):
        a0 = gen(kind, n, seed)
        p = workloads.pivot_at_quantile_np(a0, q)
        t = to_device(a0)
        _, st = ss.partition(t, p, stats=True, one_level=True, seed=88 + seed, exchange="skewed")
        out = to_host(t, a0)
        g, s, b = st["level_g"][0], st["level_s"][0], st["b"]
        X = oracle.ss_offsets(88 + seed, 0, g, s)
        ref = a0.copy()
        vmin, vmax, _, _ = oracle.ss_partial_step(ref, b, g, s, X, p)
        assert (st["vmin"], st["vmax"]) == (vmin, vmax)
        gk = out[:, 0] if out.ndim == 2 else out
        rk = ref[:, 0] if ref.ndim == 2 else ref
        assert np.array_equal(gk < p, rk < p)
        grp = _group_of_position(n, b, g, s, X)
        assert np.array_equal(gk[np.lexsort((gk, grp))], rk[np.lexsort((rk, grp))])
        done = ref.copy()
        oracle.partition(done, p)
        t = to_device(done)
        ss.partition(t, p, exchange="skewed")
        assert np.array_equal(to_host(t, done), done)


def test_exchange_structured_and_unaligned(ss):
    base = workloads.keys_u64(70001, 15)
    for k in (base % 7, np.zeros_like(base) + 3, np.sort(base), np.sort(base)[::-1].copy()):
        for q in (0.0, 0.3, 0.5, 0.99):
            check_against_oracle(ss, k, workloads.pivot_at_quantile_np(k, q), exchange=True)
    full = gen("u64", 50064, 78)
    t_full = to_device(full)
    for off in (0, 1, 3, 7, 13, 31):
        length = 50000 - off
        sub = full[off:off + length].copy()
        p = workloads.pivot_at_quantile_np(sub, 0.05)
        t = t_full.clone()
        split = ss.partition(t[off:off + length], p, exchange=True)
        out = to_host(t, full)
        assert np.array_equal(out[:off], full[:off]) and np.array_equal(out[off + length:], full[off + length:])
        ref = sub.copy()
        assert split == oracle.partition(ref, p)
        gl, gr = oracle.sorted_sides(out[off:off + length], split)
        rl, rr = oracle.sorted_sides(ref, split)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr)


def test_exchange_hybrid_and_stride_adversary(ss):
    n = (1 << 20) + 77
    g = workloads.stride_groups(n, 64, 256)
    a0 = workloads.stride_adversarial_u64(n, 8, 64, g)
    for algo in ("smoothed", "strided", "hybrid"):
        check_against_oracle(ss, a0, 1 << 63, algo=algo, exchange=True)
    a1 = workloads.keys_u64(1 << 21, 16)
    check_against_oracle(ss, a1, workloads.pivot_at_quantile_np(a1, 0.02), algo="hybrid", exchange=True)


@pytest.mark.slow
@pytest.mark.parametrize("q", [0.5, 0.01])
def test_exchange_full_size_2p30_properties(ss, q):
    """2^30 uint64 keys with the exchange form: split, sides and multiset."""
    torch = _torch()
    n = 1 << 30
    t = workloads.keys_u64_torch(n, workloads.config_seed(1), "cuda")
    p = workloads.pivot_at_quantile_torch(t, q)
    host_in = t.cpu().numpy().view(np.uint64)
    count = oracle.count_less(host_in, p)
    fp_in = oracle.fingerprint(host_in)
    del host_in
    split = ss.partition(t, p, exchange=True)
    assert split == count
    host_out = t.cpu().numpy().view(np.uint64)
    assert oracle.is_partitioned(host_out, p, split)
    assert oracle.fingerprint(host_out) == fp_in
    del t, host_out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", ["u64", "kv"])
def test_automatic_exchange_choice(ss, kind):
    """From 2^22 elements on, the default call samples the keys: a skewed pivot
    selects the exchange form for the first level, a central one the stable form,
    and both give the oracle's split and sides; the stable flag turns it off."""
    n = (1 << 22) + 1234
    a0 = gen(kind, n, 4242)
    for q, want in ((0.01, 1), (0.98, 1), (0.5, 0), (0.2, 0)):
        p = workloads.pivot_at_quantile_np(a0, q)
        t = to_device(a0)
        split, st = ss.partition(t, p, stats=True)
        assert st["exchange_mask"] & 1 == want, (q, st["exchange_mask"])
        out = to_host(t, a0)
        ref = a0.copy()
        assert split == oracle.partition(ref, p)
        gl, gr = oracle.sorted_sides(out, split)
        rl, rr = oracle.sorted_sides(ref, split)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr)
        w = 16 if kind == "kv" else 8
        if want:
            # reads n w, writes fewer than 2 (q (1 - q) + slack) n w in the first level
            assert st["bytes_moved"] < 2 * n * w
        t2 = to_device(a0)
        split2, st2 = ss.partition(t2, p, stats=True, exchange=False)
        assert split2 == split and st2["exchange_levels"] == 0 and st2["exchange_mask"] == 0
        t3 = to_device(a0)
        ss.partition(t3, p)
        assert bool((t3 == t).all())   # the choice depends only on the input


def test_automatic_exchange_strided_and_hybrid(ss):
    a0 = workloads.keys_u64((1 << 22) + 99, 4343)
    p = workloads.pivot_at_quantile_np(a0, 0.02)
    for algo in ("strided", "hybrid"):
        t = to_device(a0)
        split, st = ss.partition(t, p, stats=True, algo=algo)
        assert st["exchange_mask"] & 1 == 1, algo
        out = to_host(t, a0)
        ref = a0.copy()
        assert split == oracle.partition(ref, p)
        gl, gr = oracle.sorted_sides(out, split)
        rl, rr = oracle.sorted_sides(ref, split)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr)
