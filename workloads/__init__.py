"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds no partition or sorting arithmetic.  It only produces inputs:

* keys from a counter-based generator: key[k] is the (k+1)-th output of a
  SplitMix64 stream started at ``seed`` (Steele, Lea & Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014), i.e. the SplitMix64 finalizer
  applied to ``seed + (k + 1) * 0x9E3779B97F4A7C15`` modulo 2**64;
* a host version (numpy, uint64 arithmetic wraps) and a device version
  (PyTorch int64 ops, whose wrap-around is the same two's-complement result);
* the shape recipes of the paper's workloads: i.i.d. uniform 64-bit keys that
  fall randomly on either side of a pivot (Section 5, experimental setup),
  the same keys sorted descending, 32-bit keys with only a few distinct values,
  log-normal batch lengths and Poisson job arrivals.

Quantile pivots are ranks in sorted order (rank floor(q * n), 0-indexed); they
are found with library selection routines (numpy.partition on the host,
torch.kthvalue on the device), never with the library under test.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

# Seeds of the named workloads (one per benchmark configuration).
SEED_BASE = 0x55AA0000


def config_seed(index: int) -> int:
    return SEED_BASE + index


# ----------------------------------------------------------------------------- host (numpy)

def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
    return z ^ (z >> np.uint64(31))


def splitmix64_np(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start..start+count-1 (0-based) of the SplitMix64 stream at ``seed``."""
    with np.errstate(over="ignore"):
        k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & MASK64) + k * np.uint64(GAMMA)
        return _mix64_np(z)


def keys_u64(n: int, seed: int, start: int = 0) -> np.ndarray:
    return splitmix64_np(seed, start, n)


def stride_groups(n: int, line_elems: int, s_max: int) -> int:
    """Groups g of a Partial Partition Step over n elements with lines of
    line_elems elements and at most s_max lines per group (g = ceil(L / s_max))."""
    lines = -(-n // line_elems)
    return max(1, -(-lines // s_max))


def stride_adversarial_u64(n: int, seed: int, line_elems: int, g: int) -> np.ndarray:
    """Keys whose predecessors (key < 2^63) fill exactly the lines l with
    (l mod g) < g/2: every stride set of the Strided Algorithm (offsets 0) is
    then all predecessors or all successors.  Low 63 bits are uniform."""
    k = splitmix64_np(seed, 0, n) >> np.uint64(1)
    line = np.arange(n, dtype=np.uint64) // np.uint64(line_elems)
    succ = (line % np.uint64(g)) >= np.uint64(g // 2)
    return k | (succ.astype(np.uint64) << np.uint64(63))


def keys_u32(n: int, seed: int, start: int = 0) -> np.ndarray:
    return (splitmix64_np(seed, start, n) >> np.uint64(32)).astype(np.uint32)


def records_kv(n: int, seed: int, payload_base: int = 0) -> np.ndarray:
    """Key-value records, shape (n, 2) uint64: column 0 key, column 1 payload (global record id)."""
    out = np.empty((n, 2), dtype=np.uint64)
    out[:, 0] = splitmix64_np(seed, 0, n)
    out[:, 1] = np.arange(payload_base, payload_base + n, dtype=np.uint64)
    return out


def keys_few_distinct_u32(n: int, seed: int, distinct: int = 1024) -> np.ndarray:
    """32-bit keys drawn uniformly from ``distinct`` values (a power of two) fixed by the seed."""
    assert distinct & (distinct - 1) == 0
    values = (splitmix64_np(seed ^ 0xD15C, 0, distinct) >> np.uint64(32)).astype(np.uint32)
    bits = int(math.log2(distinct))
    pick = (splitmix64_np(seed, 0, n) >> np.uint64(64 - bits)).astype(np.int64) if bits else np.zeros(n, np.int64)
    return values[pick]


def quantile_rank(n: int, q: float) -> int:
    return min(n - 1, max(0, int(math.floor(q * n))))


def pivot_at_quantile_np(keys: np.ndarray, q: float) -> int:
    """Key of rank floor(q * n) in ascending unsigned order (n >= 1)."""
    k = keys[:, 0] if keys.ndim == 2 else keys
    r = quantile_rank(len(k), q)
    return int(np.partition(k, r)[r])


def lognormal_lengths(count: int, seed: int, median_log2: float = 14.0, sigma_log2: float = 1.0,
                      lo: int = 1 << 8, hi: int = 1 << 22) -> np.ndarray:
    """Batch lengths: round(2**Z) with Z ~ N(median_log2, sigma_log2), clipped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    z = rng.normal(median_log2, sigma_log2, size=count)
    return np.clip(np.rint(np.exp2(z)), lo, hi).astype(np.int64)


def uniform_quantiles(count: int, seed: int, lo: float = 0.05, hi: float = 0.95) -> np.ndarray:
    return np.random.default_rng(seed ^ 0x9A).uniform(lo, hi, size=count)


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def job_mix(count: int, seed: int, p_partition: float = 0.7,
            lo_log2: float = 10.0, hi_log2: float = 26.0):
    """Serving jobs: kinds (0 partition, 1 quicksort), log-uniform lengths, pivot quantiles."""
    rng = np.random.default_rng(seed ^ 0x5E)
    kinds = (rng.uniform(size=count) >= p_partition).astype(np.int32)
    lengths = np.rint(np.exp2(rng.uniform(lo_log2, hi_log2, size=count))).astype(np.int64)
    quantiles = rng.uniform(0.05, 0.95, size=count)
    return kinds, lengths, quantiles


# ----------------------------------------------------------------------------- device (torch)

def _s64(x: int) -> int:
    x &= MASK64
    return x - (1 << 64) if x >> 63 else x


def _srl(t, k: int):
    """Logical right shift of an int64 tensor."""
    import torch
    return torch.bitwise_and(torch.bitwise_right_shift(t, k), (1 << (64 - k)) - 1)


def splitmix64_torch(seed: int, start: int, count: int, device, out=None, chunk: int = 1 << 26):
    """Device twin of ``splitmix64_np``: an int64 tensor holding the same 64-bit patterns."""
    import torch
    if out is None:
        out = torch.empty(count, dtype=torch.int64, device=device)
    g, m1, m2, sd = _s64(GAMMA), _s64(M1), _s64(M2), _s64(seed)
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        z = torch.arange(start + c0 + 1, start + c1 + 1, dtype=torch.int64, device=device)
        z.mul_(g).add_(sd)
        z = torch.bitwise_xor(z, _srl(z, 30)).mul_(m1)
        z = torch.bitwise_xor(z, _srl(z, 27)).mul_(m2)
        out[c0:c1] = torch.bitwise_xor(z, _srl(z, 31))
    return out


def keys_u64_torch(n: int, seed: int, device, out=None):
    return splitmix64_torch(seed, 0, n, device, out=out)


def stride_adversarial_u64_torch(n: int, seed: int, line_elems: int, g: int, device, chunk: int = 1 << 26):
    """Device twin of stride_adversarial_u64 (same values)."""
    import torch
    out = splitmix64_torch(seed, 0, n, device)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        z = _srl(out[c0:c1], 1)
        line = torch.arange(c0, c1, dtype=torch.int64, device=device) // line_elems
        succ = (line % g) >= (g // 2)
        out[c0:c1] = torch.where(succ, z | torch.tensor(-(1 << 63), dtype=torch.int64, device=device), z)
    return out


def keys_u32_torch(n: int, seed: int, device, chunk: int = 1 << 26):
    import torch
    out = torch.empty(n, dtype=torch.int32, device=device)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        z = splitmix64_torch(seed, c0, c1 - c0, device)
        out[c0:c1] = _srl(z, 32).to(torch.int32)  # wraps to the same 32-bit pattern
    return out


def keys_few_distinct_u32_torch(n: int, seed: int, device, distinct: int = 1024, chunk: int = 1 << 26):
    import torch
    values = torch.from_numpy(keys_few_distinct_values(seed, distinct).view(np.int32)).to(device)
    bits = int(math.log2(distinct))
    out = torch.empty(n, dtype=torch.int32, device=device)
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        z = splitmix64_torch(seed, c0, c1 - c0, device)
        out[c0:c1] = values[_srl(z, 64 - bits)] if bits else values[0]
    return out


def keys_few_distinct_values(seed: int, distinct: int = 1024) -> np.ndarray:
    return (splitmix64_np(seed ^ 0xD15C, 0, distinct) >> np.uint64(32)).astype(np.uint32)


def records_kv_torch(n: int, seed: int, device, payload_base: int = 0):
    import torch
    out = torch.empty((n, 2), dtype=torch.int64, device=device)
    out[:, 0] = splitmix64_torch(seed, 0, n, device)
    out[:, 1] = torch.arange(payload_base, payload_base + n, dtype=torch.int64, device=device)
    return out


_SIGN = -(1 << 63)


def to_unsigned_order(t):
    """int64 tensor -> int64 tensor whose signed order is the unsigned order of ``t``."""
    import torch
    return torch.bitwise_xor(t, _SIGN)


def pivot_at_quantile_torch(keys, q: float) -> int:
    """Key (as an unsigned Python int) of rank floor(q * n) in ascending unsigned order."""
    import torch
    k = keys[:, 0] if keys.dim() == 2 else keys
    n = k.numel()
    r = quantile_rank(n, q)
    if k.dtype == torch.int32:
        v = torch.kthvalue(k.to(torch.int64) & 0xFFFFFFFF, r + 1).values.item()
        return int(v)
    v = torch.kthvalue(to_unsigned_order(k), r + 1).values.item()
    return (v ^ _SIGN) & MASK64


def sort_descending_u64_torch(keys):
    """Same multiset, sorted descending in unsigned order (in a new tensor)."""
    import torch
    s = torch.sort(to_unsigned_order(keys), descending=True).values
    return to_unsigned_order(s)
