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
