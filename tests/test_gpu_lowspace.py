"""GPU parity of the Low-Space Blocked-Prefix-Sum partition against the CPU oracle,
and the preprocessing lemma checked on the library's intermediate state."""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_partition import check_against_oracle, gen, to_device, to_host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 63, 64, 65, 127, 1000, 4095, 4096, 4097, 8191, 8192, 8193, 16385, 65537, 100003, 300001,
         (1 << 20) + 7]


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_lowspace_parity_both_majorities(ss, kind):
    for n in SIZES:
        a0 = gen(kind, n, 300 + n)
        keys = a0[:, 0] if a0.ndim == 2 else a0
        pivots = {0, int(keys.max()) + 1}
        for q in (0.1, 0.5, 0.9):  # successor majority, balanced, predecessor majority (roles swapped)
            pivots.add(workloads.pivot_at_quantile_np(a0, q))
        for p in sorted(pivots):
            check_against_oracle(ss, a0, p, algo="lowspace")


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_lowspace_structured_inputs(ss, kind):
    n = 200003
    base = gen(kind, n, 7)
    keys = base[:, 0] if base.ndim == 2 else base
    for name, k in {"few": keys % 5, "ascending": np.sort(keys), "descending": np.sort(keys)[::-1].copy()}.items():
        a0 = base.copy()
        if a0.ndim == 2:
            a0[:, 0] = k
        else:
            a0[:] = k
        for q in (0.2, 0.5, 0.8):
            check_against_oracle(ss, a0, workloads.pivot_at_quantile_np(a0, q), algo="lowspace")


@pytest.mark.parametrize("q", [0.05, 0.3, 0.5, 0.7, 0.95])
def test_preprocessing_makes_every_prefix_successor_heavy(ss, q):
    """Lemma preprocessingphase: after the preprocessing phase every prefix of the
    (possibly reversed) array holds at least a quarter successors."""
    for n in (1000, 65537, 1 << 20):
        a0 = workloads.keys_u64(n, 11 + n)
        p = workloads.pivot_at_quantile_np(a0, q)
        t = to_device(a0)
        _, st = ss.partition(t, p, algo="lowspace", one_level=True, stats=True)
        out = to_host(t, a0)
        assert st["vmin"] == oracle.count_less(a0, p)          # the counted predecessors
        reversed_ = bool(st["vmax"])
        assert reversed_ == (2 * st["vmin"] > n)
        assert oracle.fingerprint(out) == oracle.fingerprint(a0)
        L = out[::-1] if reversed_ else out
        succ_L = (L < p) if reversed_ else (L >= p)              # successors of the logical array
        csum = np.cumsum(succ_L.astype(np.int64))
        tt = np.arange(1, n + 1)
        assert (4 * csum >= tt).all()


def test_lowspace_unaligned_and_async(ss):
    import torch
    full = workloads.keys_u64(100000, 3)
    t_full = to_device(full)
    for off in (1, 3, 7):
        sub = full[off:off + 90000].copy()
        p = workloads.pivot_at_quantile_np(sub, 0.6)
        t = t_full.clone()
        split = ss.partition(t[off:off + 90000], p, algo="lowspace")
        out = to_host(t, full)
        assert np.array_equal(out[:off], full[:off]) and np.array_equal(out[off + 90000:], full[off + 90000:])
        ref = sub.copy()
        assert split == oracle.partition(ref, p)
        gl, gr = oracle.sorted_sides(out[off:off + 90000], split)
        rl, rr = oracle.sorted_sides(ref, split)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr)
    d = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    a0 = workloads.keys_u64(1 << 18, 4)
    p = workloads.pivot_at_quantile_np(a0, 0.75)
    t = to_device(a0)
    ss.partition_async(t, p, d, algo="lowspace")
    torch.cuda.synchronize()
    assert int(d.item()) == oracle.count_less(a0, p)


def test_lowspace_large_properties(ss):
    n = (1 << 26) + 12345
    a0 = workloads.keys_u64(n, 21)
    for q in (0.5, 0.9):
        p = workloads.pivot_at_quantile_np(a0, q)
        t = to_device(a0)
        split, st = ss.partition(t, p, algo="lowspace", stats=True)
        out = to_host(t, a0)
        assert split == oracle.count_less(a0, p)
        assert oracle.is_partitioned(out, p, split)
        assert oracle.fingerprint(out) == oracle.fingerprint(a0)
        assert st["aux_bytes"] >= n // 64 * 4


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_hybrid_parity(ss, kind):
    """Hybrid Smoothed Striding: one Partial Partition Step, then Low-Space on the middle region."""
    for n in (1, 2, 1000, 65537, 300001, (1 << 20) + 7):
        a0 = gen(kind, n, 500 + n)
        keys = a0[:, 0] if a0.ndim == 2 else a0
        pivots = {0, int(keys.max()) + 1}
        for q in (0.1, 0.5, 0.9):
            pivots.add(workloads.pivot_at_quantile_np(a0, q))
        for p in sorted(pivots):
            check_against_oracle(ss, a0, p, algo="hybrid")


def test_hybrid_large_and_async(ss):
    import torch
    n = (1 << 26) + 3
    a0 = workloads.keys_u64(n, 77)
    p = workloads.pivot_at_quantile_np(a0, 0.5)
    t = to_device(a0)
    d = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ss.partition_async(t, p, d, algo="hybrid")
    torch.cuda.synchronize()
    out = to_host(t, a0)
    split = int(d.item())
    assert split == oracle.count_less(a0, p)
    assert oracle.is_partitioned(out, p, split)
    assert oracle.fingerprint(out) == oracle.fingerprint(a0)


@pytest.mark.parametrize("algo", ["mediumspace", "highspace"])
@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_explicit_space_comparators_parity(ss, algo, kind):
    """Medium- and High-Space: the standard parallel partition into an n-sized output array."""
    for n in (1, 2, 63, 64, 65, 4097, 100003, (1 << 20) + 7):
        a0 = gen(kind, n, 900 + n)
        keys = a0[:, 0] if a0.ndim == 2 else a0
        pivots = {0, int(keys.max()) + 1}
        for q in (0.1, 0.5, 0.9):
            pivots.add(workloads.pivot_at_quantile_np(a0, q))
        for p in sorted(pivots):
            check_against_oracle(ss, a0, p, algo=algo)


def test_explicit_space_async_and_aux(ss):
    import torch
    n = (1 << 22) + 5
    a0 = workloads.keys_u64(n, 31)
    p = workloads.pivot_at_quantile_np(a0, 0.3)
    for algo in ("mediumspace", "highspace"):
        t = to_device(a0)
        d = torch.full((1,), -1, dtype=torch.int64, device="cuda")
        ss.partition_async(t, p, d, algo=algo)
        torch.cuda.synchronize()
        out = to_host(t, a0)
        split = int(d.item())
        assert split == oracle.count_less(a0, p)
        assert oracle.is_partitioned(out, p, split)
        assert oracle.fingerprint(out) == oracle.fingerprint(a0)
    med = ss.aux_bytes(n, ss.SS_U64, "mediumspace")
    high = ss.aux_bytes(n, ss.SS_U64, "highspace")
    assert med >= n * 8 and high - med == n * 8


def test_preprocessing_equals_oracle_phase(ss):
    """The Low-Space preprocessing phase (one_level) leaves the array byte for byte
    as the oracle's MakeSuccessorHeavy does."""
    for kind in ("u32", "u64", "kv"):
        for n, q in ((1000, 0.3), (65537, 0.7), ((1 << 20) + 3, 0.5), (300001, 0.95)):
            a0 = gen(kind, n, 17 + n)
            p = workloads.pivot_at_quantile_np(a0, q)
            t = to_device(a0)
            ss.partition(t, p, algo="lowspace", one_level=True)
            ref = a0.copy()
            oracle.make_successor_heavy(ref, p)
            assert np.array_equal(to_host(t, a0), ref), (kind, n, q)


IMPLICIT_SIZES = [1, 2, 100, 4095, 4096, 4097, 8191, 8192, 8193, 16384, 16385, 65537, 100003, 300001,
                  (1 << 20) + 7, (1 << 21) + 300]


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_implicit_parity(ss, kind):
    """The implicit Blocked-Prefix-Sum partition: split and sides equal the oracle's,
    for both majorities (roles swapped when predecessors are the majority)."""
    for n in IMPLICIT_SIZES:
        a0 = gen(kind, n, 900 + n)
        keys = a0[:, 0] if a0.ndim == 2 else a0
        pivots = {0, int(keys.max()) + 1}
        for q in (0.01, 0.2, 0.5, 0.8, 0.99):
            pivots.add(workloads.pivot_at_quantile_np(a0, q))
        for p in sorted(pivots):
            check_against_oracle(ss, a0, p, algo="implicit")


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_implicit_repeated_elements(ss, kind):
    """Lemma bitstore2: blocks full of equal pairs (few distinct keys, all equal,
    sorted runs) store their values by flipping and restoring elements."""
    n = 300007
    base = gen(kind, n, 23)
    keys = base[:, 0] if base.ndim == 2 else base
    variants = {"few": keys % 3, "equal": np.zeros_like(keys) + 5, "ascending": np.sort(keys % 1000),
                "descending": np.sort(keys)[::-1].copy()}
    for name, k in variants.items():
        a0 = base.copy()
        if a0.ndim == 2:
            a0[:, 0] = k
            if name in ("few", "equal"):
                a0[:, 1] = a0[:, 1] % 2      # equal records too, not only equal keys
        else:
            a0[:] = k
        for q in (0.0, 0.3, 0.5, 0.9, 1.0):
            p = workloads.pivot_at_quantile_np(a0, q) if q < 1.0 else U64MAX
            check_against_oracle(ss, a0, p, algo="implicit")


U64MAX = (1 << 64) - 1


def _decode_blocks(L: np.ndarray, nb: int):
    """Host reading of the block values (Lemma bitstore / bitstore2 as the library
    lays them out: blocks of 256, pair j = elements 2j, 2j + 1; pair 0 unequal
    marks ordered pairs, equal marks flipped ones).  Returns the values and a copy
    of L with every flipped element restored."""
    R = L.copy()
    if L.ndim == 2:
        X = R[:nb * 256].reshape(nb, 128, 2, 2)[:, :64]      # block, pair, element, (key, payload)
        a, b = X[:, :, 0, :], X[:, :, 1, :]
        eq = (a == b).all(axis=2)
        lt = (a[:, :, 0] < b[:, :, 0]) | ((a[:, :, 0] == b[:, :, 0]) & (a[:, :, 1] < b[:, :, 1]))
    else:
        X = R[:nb * 256].reshape(nb, 128, 2)[:, :64]
        a, b = X[:, :, 0], X[:, :, 1]
        eq = a == b
        lt = a < b
    type1 = ~eq[:, 0]
    bits = np.where(type1[:, None], lt, ~eq)[:, 1:].astype(np.uint64)
    vals = (bits << np.arange(63, dtype=np.uint64)[None, :]).sum(axis=1, dtype=np.uint64)
    restore = (~type1)[:, None] & ~eq
    restore[:, 0] = False
    bi, pj = np.nonzero(restore)
    X[bi, pj, 1] = X[bi, pj, 0]
    return vals, R


@pytest.mark.parametrize("kind", ["u32", "u64", "kv"])
def test_implicit_prefix_sum_in_the_element_order(ss, kind):
    """one_level stops the implicit variant once the prefix sum is stored: read on
    the host, block b holds the predecessors of L in blocks 0..b of the oracle's
    preprocessed array, and each block (restored) holds that block's elements."""
    for n, q, dup in ((300001, 0.3, False), ((1 << 20) + 77, 0.7, False), (200003, 0.4, True),
                      ((1 << 18) + 5, 0.5, True)):
        a0 = gen(kind, n, 70 + n)
        if dup:
            if a0.ndim == 2:
                a0[:, 0] %= 4
                a0[:, 1] %= 2
            else:
                a0 %= 4
        p = workloads.pivot_at_quantile_np(a0, q)
        t = to_device(a0)
        _, st = ss.partition(t, p, algo="implicit", one_level=True, stats=True)
        out = to_host(t, a0)
        ref = a0.copy()
        rev = oracle.make_successor_heavy(ref, p)
        assert bool(st["vmax"]) == rev
        Lg = out[::-1] if rev else out
        Lr = ref[::-1] if rev else ref
        nb = n // 256
        vals, restored = _decode_blocks(np.ascontiguousarray(Lg), nb)
        kr = Lr[:, 0] if Lr.ndim == 2 else Lr
        predL = (kr.astype(np.uint64) < np.uint64(p)) != rev
        ends = np.minimum((np.arange(nb) + 1) * 256, n)
        ends[-1] = n
        expect = np.cumsum(predL.astype(np.int64))[ends - 1].astype(np.uint64)
        assert np.array_equal(vals, expect), (kind, n, q, dup)
        for b in range(nb):                                  # each block's multiset
            lo, hi = b * 256, (n if b == nb - 1 else (b + 1) * 256)
            gl, _ = oracle.sorted_sides(np.ascontiguousarray(restored[lo:hi]), hi - lo)
            rl, _ = oracle.sorted_sides(np.ascontiguousarray(Lr[lo:hi]), hi - lo)
            assert np.array_equal(gl, rl), (kind, n, b)


def test_implicit_aux_and_async(ss):
    torch = __import__("torch")
    n = (1 << 22) + 11
    assert ss.aux_bytes(n, ss.SS_U64, "implicit") < ss.aux_bytes(n, ss.SS_U64, "smoothed") + (64 << 10)
    assert ss.aux_bytes(n, ss.SS_U64, "lowspace") > ss.aux_bytes(n, ss.SS_U64, "implicit") + n // 64 * 4
    a0 = workloads.keys_u64(n, 5)
    p = workloads.pivot_at_quantile_np(a0, 0.6)
    t = to_device(a0)
    d = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ss.partition_async(t, p, d, algo="implicit")
    torch.cuda.synchronize()
    split = int(d.item())
    assert split == oracle.count_less(a0, p)
    out = to_host(t, a0)
    assert oracle.is_partitioned(out, p, split)
    assert oracle.fingerprint(out) == oracle.fingerprint(a0)
    _, st = ss.partition(to_device(a0), p, algo="implicit", stats=True)
    assert st["aux_bytes"] == ss.aux_bytes(n, ss.SS_U64, "implicit")


def test_implicit_large_properties(ss):
    """Above 512 MiB the implicit variant's passes write whole lines: 2^26 + 777 u64
    keys, distinct and with few distinct values (flipped-element encoding), both
    majorities, checked by count, side property and multiset."""
    n = (1 << 26) + 777
    a0 = workloads.keys_u64(n, 29)
    few = a0 % np.uint64(5)
    for keys, q in ((a0, 0.3), (a0, 0.8), (few, 0.5)):
        p = workloads.pivot_at_quantile_np(keys, q)
        t = to_device(keys)
        split = ss.partition(t, p, algo="implicit")
        out = to_host(t, keys)
        assert split == oracle.count_less(keys, p)
        assert oracle.is_partitioned(out, p, split)
        assert oracle.fingerprint(out) == oracle.fingerprint(keys)
