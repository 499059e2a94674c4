"""CPU oracle for the in-place partition and quicksort -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and it shares no code with the GPU library.  The arithmetic lives in
``oracle.c`` (plain serial C, see its header for what each routine follows in
the paper); this module only marshals numpy arrays through ctypes.

Arrays: u32 -> numpy uint32 1-D, u64 -> numpy uint64 1-D, kv -> numpy uint64
of shape (n, 2) (column 0 key, column 1 payload).  Keys compare unsigned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (in place)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        sz, u64, u32, vp, i32 = ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
        for s in ("u32", "u64", "kv"):
            getattr(L, "oracle_count_less_" + s).argtypes = [vp, sz, u64]
            getattr(L, "oracle_count_less_" + s).restype = sz
            for nm in ("oracle_partition_", "oracle_partition_le_"):
                getattr(L, nm + s).argtypes = [vp, sz, u64]
                getattr(L, nm + s).restype = sz
            getattr(L, "oracle_quicksort_" + s).argtypes = [vp, sz]
            getattr(L, "oracle_quicksort_" + s).restype = None
            getattr(L, "oracle_is_partitioned_" + s).argtypes = [vp, sz, u64, sz]
            getattr(L, "oracle_is_partitioned_" + s).restype = i32
            getattr(L, "oracle_is_sorted_" + s).argtypes = [vp, sz]
            getattr(L, "oracle_is_sorted_" + s).restype = i32
            getattr(L, "oracle_fingerprint_" + s).argtypes = [vp, sz, vp]
            getattr(L, "oracle_fingerprint_" + s).restype = None
            getattr(L, "oracle_ss_partial_step_" + s).argtypes = [vp, sz, u32, u32, u32, vp, u64, vp, vp, vp, vp]
            getattr(L, "oracle_ss_partial_step_" + s).restype = i32
        L.oracle_splitmix64.argtypes = [u64, u64]
        L.oracle_splitmix64.restype = u64
        L.oracle_ss_offsets.argtypes = [u64, u32, u32, u32, vp]
        L.oracle_ss_offsets.restype = None
        _lib = L
    return _lib


def _kind(a: np.ndarray) -> str:
    if a.dtype == np.uint32 and a.ndim == 1:
        return "u32"
    if a.dtype == np.uint64 and a.ndim == 1:
        return "u64"
    if a.dtype == np.uint64 and a.ndim == 2 and a.shape[1] == 2:
        return "kv"
    raise TypeError("oracle arrays are uint32[n], uint64[n] or uint64[n,2], got %s%s" % (a.dtype, a.shape))


def _ptr(a: np.ndarray):
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return ctypes.c_void_p(a.ctypes.data)


def _n(a):
    return a.shape[0]


def count_less(a: np.ndarray, pivot: int) -> int:
    """Plain definition of the split: #{k : key(a[k]) < pivot}."""
    return getattr(lib(), "oracle_count_less_" + _kind(a))(_ptr(a), _n(a), pivot)


def partition(a: np.ndarray, pivot: int) -> int:
    """Serial two-pointer partition in place (decider key < pivot); returns the split."""
    return getattr(lib(), "oracle_partition_" + _kind(a))(_ptr(a), _n(a), pivot)


def partition_le(a: np.ndarray, pivot: int) -> int:
    """Same with the decider key <= pivot."""
    return getattr(lib(), "oracle_partition_le_" + _kind(a))(_ptr(a), _n(a), pivot)


def quicksort(a: np.ndarray) -> None:
    """Serial quicksort in place, ascending by key."""
    getattr(lib(), "oracle_quicksort_" + _kind(a))(_ptr(a), _n(a))


def is_partitioned(a: np.ndarray, pivot: int, split: int) -> bool:
    return bool(getattr(lib(), "oracle_is_partitioned_" + _kind(a))(_ptr(a), _n(a), pivot, split))


def is_sorted(a: np.ndarray) -> bool:
    return bool(getattr(lib(), "oracle_is_sorted_" + _kind(a))(_ptr(a), _n(a)))


def fingerprint(a: np.ndarray) -> tuple:
    """Order-independent multiset fingerprint (count, sum h, sum h^2, xor h')."""
    out = np.zeros(4, dtype=np.uint64)
    getattr(lib(), "oracle_fingerprint_" + _kind(a))(_ptr(a), _n(a), _ptr(out))
    return tuple(int(x) for x in out)


def splitmix64(seed: int, ctr: int) -> int:
    return int(lib().oracle_splitmix64(seed, ctr))


def ss_offsets(seed: int, level: int, g: int, s: int) -> np.ndarray:
    """X_0..X_{s-1} in [0, g) for one Smoothed Striding level."""
    X = np.zeros(max(1, s), dtype=np.uint32)
    lib().oracle_ss_offsets(seed, level, g, s, _ptr(X))
    return X[:s]


def ss_partial_step(a: np.ndarray, b: int, g: int, s: int, X: np.ndarray, pivot: int):
    """One Partial Partition Step in place.  Returns (v_min, v_max, c[g], v[g])."""
    X = np.ascontiguousarray(X, dtype=np.uint32)
    if X.shape != (s,):
        raise ValueError("X must hold s offsets")
    c = np.zeros(g, dtype=np.uint64)
    v = np.zeros(g, dtype=np.uint64)
    vmin = np.zeros(1, dtype=np.uint64)
    vmax = np.zeros(1, dtype=np.uint64)
    rc = getattr(lib(), "oracle_ss_partial_step_" + _kind(a))(
        _ptr(a), _n(a), b, g, s, _ptr(X), pivot, _ptr(vmin), _ptr(vmax), _ptr(c), _ptr(v))
    if rc != 0:
        raise ValueError("invalid geometry: need s*g*b >= n > (s-1)*g*b and X_j < g")
    return int(vmin[0]), int(vmax[0]), c, v


def make_successor_heavy(a: np.ndarray, pivot: int) -> bool:
    """Preprocessing phase of the Blocked-Prefix-Sum partition (Section 3,
    MakeSuccessorHeavy; Lemma preprocessingphase), in place.  The roles are
    swapped first when predecessors (key < pivot) are the majority
    (ParallelPartition): the logical array L is then `a` read backwards with
    the decider negated.  For m = n, ceil(n/2), ceil(n/4), ... while m >= 2,
    and every i < floor(m/2) in parallel: if L[i] is a predecessor of L and
    L[m-1-i] a successor of L, they are swapped.  Returns whether the roles
    were swapped."""
    keys = a[:, 0] if a.ndim == 2 else a
    n = keys.shape[0]
    rev = 2 * count_less(a, pivot) > n
    L = a[::-1]
    if not rev:
        L = a
    m = n
    while m >= 2:
        half = m // 2
        lk = L[:, 0] if L.ndim == 2 else L
        pred = lk.astype(np.uint64) < np.uint64(pivot)
        if rev:
            pred = ~pred
        i = np.arange(half)
        j = m - 1 - i
        sw = pred[i] & ~pred[j]
        ii, jj = i[sw], j[sw]
        tmp = L[ii].copy()
        L[ii] = L[jj]
        L[jj] = tmp
        m = (m + 1) // 2
    return bool(rev)


def sorted_sides(a: np.ndarray, split: int):
    """(sorted left side, sorted right side) -- the unique content of a partition.

    kv records sort by (key, payload)."""
    if a.ndim == 2:
        def srt(x):
            idx = np.lexsort((x[:, 1], x[:, 0]))
            return x[idx]
        return srt(a[:split]), srt(a[split:])
    return np.sort(a[:split]), np.sort(a[split:])
