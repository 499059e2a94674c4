"""Python binding of libss.so: argument marshalling only.

Every call goes through the C ABI declared in include/ss.h; all work runs in
the library's HIP kernels.  PyTorch is used for device memory and streams:

* SS_U32 arrays are int32 CUDA tensors (bit patterns read as uint32),
* SS_U64 arrays are int64 CUDA tensors (bit patterns read as uint64),
* SS_KV16 arrays are int64 CUDA tensors of shape (n, 2): key, payload.

There is no fallback: if libss.so is missing, importing this package fails.
"""
from __future__ import annotations

import ctypes
import os

# PyTorch ships its own HIP runtime under the same soname as ROCm's.  Loading
# torch first makes libss.so bind to that already-loaded runtime, so the
# process has one HIP runtime whichever package the caller imports first.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libss.so")
if not os.path.exists(_SO):
    raise ImportError("libss.so is not built; run `python paper_2004_12532_amd/build.py` "
                      "(or __graft_entry__.build())")
_lib = ctypes.CDLL(_SO)

SS_U32, SS_U64, SS_KV16 = 1, 2, 3
SMOOTHED, STRIDED, LOWSPACE, HYBRID, MEDIUMSPACE, HIGHSPACE, IMPLICIT = 0, 1, 2, 3, 4, 5, 6
ALGOS = {"smoothed": SMOOTHED, "strided": STRIDED, "lowspace": LOWSPACE, "hybrid": HYBRID,
         "mediumspace": MEDIUMSPACE, "highspace": HIGHSPACE, "implicit": IMPLICIT}
FLAG_ONE_LEVEL, FLAG_TIME, FLAG_GRAPH, FLAG_EXCHANGE, FLAG_EXCHANGE_SKEWED, FLAG_STABLE = 1, 2, 16, 32, 64, 128
MAX_LEVELS = 32
STATUS = {0: "SS_OK", -1: "SS_EINVAL", -2: "SS_ENOMEM", -3: "SS_EDEVICE", -4: "SS_EUNSUPPORTED",
          -5: "SS_EINCOMPLETE"}


class Params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("b", ctypes.c_uint32), ("tile_bytes", ctypes.c_uint32),
                ("max_levels", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("engine", ctypes.c_uint32)]


MAX_CLASSES = 8


class Tuning(ctypes.Structure):
    """ss_batched_tuning: size classes of the batched calls."""
    _fields_ = [("nclass", ctypes.c_uint32), ("b", ctypes.c_uint32 * MAX_CLASSES),
                ("group_bytes", ctypes.c_uint32 * MAX_CLASSES), ("max_len", ctypes.c_uint64 * MAX_CLASSES),
                ("ms", ctypes.c_float * MAX_CLASSES)]

    def as_dict(self) -> dict:
        n = self.nclass
        return {"classes": [{"max_len": int(self.max_len[c]), "b": int(self.b[c]),
                             "group_bytes": int(self.group_bytes[c]), "ms": round(float(self.ms[c]), 4)}
                            for c in range(n)]}

    @classmethod
    def from_dict(cls, d: dict) -> "Tuning":
        t = cls()
        cl = d["classes"]
        t.nclass = len(cl)
        for c, x in enumerate(cl):
            t.b[c], t.group_bytes[c], t.max_len[c] = x["b"], x["group_bytes"], x["max_len"]
            t.ms[c] = x.get("ms", 0.0)
        return t


class Stats(ctypes.Structure):
    _fields_ = [("split", ctypes.c_uint64), ("aux_bytes", ctypes.c_uint64), ("lds_bytes", ctypes.c_uint32),
                ("grid", ctypes.c_uint32), ("b", ctypes.c_uint32), ("s_max", ctypes.c_uint32),
                ("levels", ctypes.c_uint32), ("launches", ctypes.c_uint32),
                ("level_lo", ctypes.c_uint64 * MAX_LEVELS), ("level_hi", ctypes.c_uint64 * MAX_LEVELS),
                ("level_g", ctypes.c_uint32 * MAX_LEVELS), ("level_s", ctypes.c_uint32 * MAX_LEVELS),
                ("vmin", ctypes.c_uint64), ("vmax", ctypes.c_uint64),
                ("first_level_ms", ctypes.c_float), ("total_ms", ctypes.c_float),
                ("bytes_moved", ctypes.c_uint64), ("exchange_levels", ctypes.c_uint32), ("exchange_mask", ctypes.c_uint32),
                ("first_level_bytes", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        nl = self.levels
        return {
            "split": self.split, "aux_bytes": self.aux_bytes, "lds_bytes": self.lds_bytes, "grid": self.grid,
            "b": self.b, "s_max": self.s_max, "levels": nl, "launches": self.launches,
            "level_lo": list(self.level_lo[:nl]), "level_hi": list(self.level_hi[:nl]),
            "level_g": list(self.level_g[:nl]), "level_s": list(self.level_s[:nl]),
            "vmin": self.vmin, "vmax": self.vmax, "first_level_ms": self.first_level_ms,
            "total_ms": self.total_ms, "bytes_moved": self.bytes_moved, "exchange_levels": self.exchange_levels,
            "exchange_mask": self.exchange_mask, "first_level_bytes": self.first_level_bytes,
        }


_vp, _sz, _u64, _int = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int
_lib.ss_partition.argtypes = [_vp, _sz, _int, _u64, ctypes.POINTER(_sz)]
_lib.ss_partition_ex.argtypes = [_vp, _sz, _int, _u64, ctypes.POINTER(Params), _vp, _vp, ctypes.POINTER(_sz),
                                 ctypes.POINTER(Stats)]
_lib.ss_quicksort.argtypes = [_vp, _sz, _int]
_lib.ss_quicksort_ex.argtypes = [_vp, _sz, _int, ctypes.POINTER(Params), _vp, ctypes.POINTER(Stats)]
_lib.ss_partition_batched.argtypes = [_vp, _vp, _sz, _int, _vp, _vp, ctypes.POINTER(Params), _vp,
                                      ctypes.POINTER(Stats)]
_lib.ss_partition_segments.argtypes = [_vp, _vp, _vp, _sz, _int, _vp, _vp, ctypes.POINTER(Params), _vp,
                                       ctypes.POINTER(Stats)]
_lib.ss_partition_each.argtypes = [_vp, _vp, _sz, _int, _vp, _vp, ctypes.POINTER(Params), _vp, _vp]
_lib.ss_partition_noalloc.argtypes = [_vp, _sz, _int, _u64, ctypes.POINTER(Params), _vp, _vp]
_lib.ss_median3_pivots.argtypes = [_vp, _vp, _vp, _sz, _int, _vp, _vp, _vp]
_lib.ss_sort_segments.argtypes = [_vp, _vp, _vp, _sz, _int, _vp]
_lib.ss_autotune_batched.argtypes = [_int, _vp, ctypes.POINTER(Tuning)]
_lib.ss_set_batched_tuning.argtypes = [_int, ctypes.POINTER(Tuning)]
_lib.ss_get_batched_tuning.argtypes = [_int, ctypes.POINTER(Tuning)]
_u32 = ctypes.c_uint32
_lib.ss_server_create.argtypes = [_vp, _sz, _int, _u32, _u32, _vp, ctypes.POINTER(_vp)]
_lib.ss_server_destroy.argtypes = [_vp]
_lib.ss_server_submit.argtypes = [_vp, _u32, _u64, _u64, _int, _u64]
_lib.ss_server_tick.argtypes = [_vp, _u64]
_lib.ss_server_wait.argtypes = [_vp, _u32, ctypes.POINTER(_u32)]
_lib.ss_server_done.argtypes = [_vp, _u32, ctypes.POINTER(_u64)]
_lib.ss_server_status.argtypes = [_vp, ctypes.POINTER(_u32)]
_lib.ss_server_job_aux_bytes.argtypes = [_int, _int, _u64]
_lib.ss_server_job_aux_bytes.restype = _sz
_lib.ss_sort_segment_cap.argtypes = [_int]
_lib.ss_sort_segment_cap.restype = _sz
_lib.ss_aux_bytes.argtypes = [_sz, _int, _int]
_lib.ss_aux_bytes.restype = _sz
_lib.ss_strerror.argtypes = [_int]
_lib.ss_strerror.restype = ctypes.c_char_p
_lib.ss_last_error.argtypes = []
_lib.ss_last_error.restype = ctypes.c_char_p
_lib.ss_probe_bandwidth.argtypes = [_vp, _sz, _int, _vp, ctypes.POINTER(ctypes.c_float)]
_lib.ss_device_info.argtypes = [ctypes.POINTER(_int)] * 4
for _f in ("ss_partition", "ss_partition_ex", "ss_quicksort", "ss_quicksort_ex", "ss_partition_batched",
           "ss_probe_bandwidth", "ss_device_info", "ss_partition_segments", "ss_median3_pivots",
           "ss_sort_segments"):
    getattr(_lib, _f).restype = _int

LIB_PATH = _SO
lib = _lib


class SSError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        detail = _lib.ss_last_error().decode()
        super().__init__("%s failed: %s (%s)%s" % (what, STATUS.get(code, code), _lib.ss_strerror(code).decode(),
                                                   (": " + detail) if detail else ""))


def _check(code: int, what: str):
    if code != 0:
        raise SSError(code, what)


def dtype_of(t) -> int:
    """ss_dtype of a tensor: int32[n] -> U32, int64[n] -> U64, int64[n,2] -> KV16."""
    import torch
    if t.dim() == 1 and t.dtype in (torch.int32, getattr(torch, "uint32", torch.int32)):
        return SS_U32
    if t.dim() == 1 and t.dtype in (torch.int64, getattr(torch, "uint64", torch.int64)):
        return SS_U64
    if t.dim() == 2 and t.shape[1] == 2 and t.dtype in (torch.int64, getattr(torch, "uint64", torch.int64)):
        return SS_KV16
    raise TypeError("expected int32[n], int64[n] or int64[n,2], got %s%s" % (t.dtype, tuple(t.shape)))


def _array(t):
    if not t.is_cuda:
        raise ValueError("the array must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("the array must be contiguous")
    return ctypes.c_void_p(t.data_ptr()), t.shape[0], dtype_of(t)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


ENGINES = {"auto": 0, "lds": 1, "regs": 2, "staged": 3}


def make_params(algo="smoothed", b=0, tile_bytes=0, max_levels=0, seed=0, one_level=False, time=False,
                engine="auto", graph=False, exchange="auto") -> Params:
    """exchange: "auto" (the library chooses the first level's form from a
    sample), False (stable partition of every group), True (write-minimal
    exchange of every group) or "skewed" (exchange only the groups with few
    misplaced pairs)."""
    a = ALGOS[algo] if isinstance(algo, str) else int(algo)
    flags = (FLAG_ONE_LEVEL if one_level else 0) | (FLAG_TIME if time else 0) | (FLAG_GRAPH if graph else 0) \
        | {"auto": 0, "skewed": FLAG_EXCHANGE_SKEWED, True: FLAG_EXCHANGE, False: FLAG_STABLE}[exchange]
    e = ENGINES[engine] if isinstance(engine, str) else int(engine)
    return Params(a, b, tile_bytes, max_levels, seed, flags, e)


def partition(t, pivot: int, *, stats: bool = False, stream=None, **kw):
    """Partition the tensor in place by key < pivot; returns the split (and the stats dict)."""
    ptr, n, dt = _array(t)
    p = make_params(**kw)
    split = _sz(0)
    st = Stats()
    _check(_lib.ss_partition_ex(ptr, n, dt, pivot & ((1 << 64) - 1), ctypes.byref(p), _stream(stream), None,
                                ctypes.byref(split), ctypes.byref(st) if stats else None), "ss_partition_ex")
    return (split.value, st.as_dict()) if stats else split.value


def partition_async(t, pivot: int, d_split, *, stream=None, **kw) -> None:
    """Partition without synchronizing; the split lands in d_split[0] (an int64 CUDA tensor)."""
    ptr, n, dt = _array(t)
    p = make_params(**kw)
    _check(_lib.ss_partition_ex(ptr, n, dt, pivot & ((1 << 64) - 1), ctypes.byref(p), _stream(stream),
                                ctypes.c_void_p(d_split.data_ptr()), None, None), "ss_partition_ex")


def partition_noalloc(t, pivot: int, d_split, *, stream=None, **kw) -> None:
    """ss_partition_noalloc: asynchronous partition that allocates no device memory; the split lands
    in d_split[0] (an int64 CUDA tensor)."""
    ptr, n, dt = _array(t)
    p = make_params(**kw)
    _check(_lib.ss_partition_noalloc(ptr, n, dt, pivot & ((1 << 64) - 1), ctypes.byref(p), _stream(stream),
                                     ctypes.c_void_p(d_split.data_ptr())), "ss_partition_noalloc")


def partition_plain(t, pivot: int) -> int:
    """ss_partition: default parameters, default stream, blocking."""
    ptr, n, dt = _array(t)
    split = _sz(0)
    _check(_lib.ss_partition(ptr, n, dt, pivot & ((1 << 64) - 1), ctypes.byref(split)), "ss_partition")
    return split.value


def quicksort(t, *, stats: bool = False, stream=None, **kw):
    """Sort the tensor in place ascending by (unsigned) key."""
    ptr, n, dt = _array(t)
    p = make_params(**kw)
    st = Stats()
    _check(_lib.ss_quicksort_ex(ptr, n, dt, ctypes.byref(p), _stream(stream), ctypes.byref(st) if stats else None),
           "ss_quicksort_ex")
    return st.as_dict() if stats else None


def partition_each(base, offsets, pivots, splits, *, latencies: bool = False, stream=None, **kw):
    """ss_partition_each: one single-array call per array base[offsets[k]:offsets[k+1]] with pivot
    pivots[k] (host sequences), issued from C back to back; splits (int64 CUDA tensor of num entries)
    receives the splits.  With latencies=True it waits and returns each array's completion time in ms
    after the first launch (numpy float32 array)."""
    import numpy as np

    ptr, _, dt = _array(base)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    piv = np.ascontiguousarray(np.asarray([int(x) & ((1 << 64) - 1) for x in pivots], dtype=np.uint64))
    num = off.size - 1
    p = make_params(**kw)
    ms = np.zeros(max(num, 1), dtype=np.float32) if latencies else None
    _check(_lib.ss_partition_each(ptr, off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), num, dt,
                                  piv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  ctypes.c_void_p(splits.data_ptr()), ctypes.byref(p), _stream(stream),
                                  ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if latencies else None),
           "ss_partition_each")
    return ms[:num] if latencies else None


def partition_batched(base, offsets, pivots, splits, *, stats: bool = False, stream=None, **kw):
    """Partition base[offsets[k]:offsets[k+1]] by pivots[k] for every k.

    offsets: host sequence of num+1 element offsets; pivots, splits: int64 CUDA tensors of num entries."""
    import numpy as np
    ptr, _, dt = _array(base)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
    num = len(off) - 1
    p = make_params(**kw)
    st = Stats()
    _check(_lib.ss_partition_batched(ptr, ctypes.c_void_p(off.ctypes.data), num, dt,
                                     ctypes.c_void_p(pivots.data_ptr()), ctypes.c_void_p(splits.data_ptr()),
                                     ctypes.byref(p), _stream(stream), ctypes.byref(st) if stats else None),
           "ss_partition_batched")
    return st.as_dict() if stats else None


def autotune_batched(dtype, stream=None) -> dict:
    """Time every candidate line and group size per length class on synthetic
    batches and install the fastest for later batched calls of dtype."""
    t = Tuning()
    _check(_lib.ss_autotune_batched(_dtype_code(dtype), _stream(stream), ctypes.byref(t)), "ss_autotune_batched")
    return t.as_dict()


def set_batched_tuning(dtype, table) -> None:
    """Install a table (a dict as returned by autotune_batched), or None for the default."""
    t = Tuning.from_dict(table) if table is not None else None
    _check(_lib.ss_set_batched_tuning(_dtype_code(dtype), ctypes.byref(t) if t is not None else None),
           "ss_set_batched_tuning")


def get_batched_tuning(dtype) -> dict:
    t = Tuning()
    _check(_lib.ss_get_batched_tuning(_dtype_code(dtype), ctypes.byref(t)), "ss_get_batched_tuning")
    return t.as_dict()


def _dtype_code(dtype) -> int:
    if isinstance(dtype, int):
        return dtype
    return {"u32": SS_U32, "u64": SS_U64, "kv": SS_KV16, "kv16": SS_KV16}[dtype]


def _u64_host(x):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    return a, ctypes.c_void_p(a.ctypes.data)


def partition_segments(base, starts, lens, pivots, splits, *, stats: bool = False, stream=None, **kw):
    """Partition disjoint segments base[starts[k]:starts[k]+lens[k]] by pivots[k] (int64 CUDA
    tensor); splits (int64 CUDA tensor) receives each segment's split."""
    ptr, _, dt = _array(base)
    s_arr, s_ptr = _u64_host(starts)
    l_arr, l_ptr = _u64_host(lens)
    p = make_params(**kw)
    st = Stats()
    _check(_lib.ss_partition_segments(ptr, s_ptr, l_ptr, len(s_arr), dt, ctypes.c_void_p(pivots.data_ptr()),
                                      ctypes.c_void_p(splits.data_ptr()), ctypes.byref(p), _stream(stream),
                                      ctypes.byref(st) if stats else None), "ss_partition_segments")
    return st.as_dict() if stats else None


def median3_pivots(base, starts, lens, d_pivots, *, host=True, stream=None):
    """Median-of-3 pivot of every segment into d_pivots (int64 CUDA tensor); returns them
    as a numpy uint64 array when host is true."""
    import numpy as np
    ptr, _, dt = _array(base)
    s_arr, s_ptr = _u64_host(starts)
    l_arr, l_ptr = _u64_host(lens)
    out = np.zeros(len(s_arr), dtype=np.uint64) if host else None
    _check(_lib.ss_median3_pivots(ptr, s_ptr, l_ptr, len(s_arr), dt, ctypes.c_void_p(d_pivots.data_ptr()),
                                  ctypes.c_void_p(out.ctypes.data) if host else None, _stream(stream)),
           "ss_median3_pivots")
    return out


def sort_segments(base, starts, lens, *, stream=None):
    """Sort every segment (length <= sort_segment_cap) in place with the LDS sort."""
    ptr, _, dt = _array(base)
    s_arr, s_ptr = _u64_host(starts)
    l_arr, l_ptr = _u64_host(lens)
    _check(_lib.ss_sort_segments(ptr, s_ptr, l_ptr, len(s_arr), dt, _stream(stream)), "ss_sort_segments")


class ServerEngine:
    """The device-resident serving engine (ss_server_*) over one CUDA tensor."""

    def __init__(self, base, max_jobs: int, max_segments: int, stream=None):
        ptr, n, dt = _array(base)
        self.dtype = dt
        self._h = _vp()
        _check(_lib.ss_server_create(ptr, n, dt, max_jobs, max_segments, _stream(stream), ctypes.byref(self._h)),
               "ss_server_create")

    def submit(self, slot: int, start: int, length: int, kind: int, pivot: int = 0) -> None:
        _check(_lib.ss_server_submit(self._h, slot, start, length, kind, pivot & ((1 << 64) - 1)),
               "ss_server_submit")

    def tick(self, max_len: int) -> None:
        _check(_lib.ss_server_tick(self._h, max_len), "ss_server_tick")

    def wait(self, in_flight: int = 0) -> int:
        """Wait until at most `in_flight` ticks run; returns the overflow flags
        mirrored in host memory (nonzero: a device list overflowed or a
        partition was left unfinished)."""
        f = _u32(0)
        _check(_lib.ss_server_wait(self._h, in_flight, ctypes.byref(f)), "ss_server_wait")
        return int(f.value)

    def done(self, slot: int):
        """(finished, split) for the job in slot; split only for partition jobs."""
        sp = _u64(0)
        rc = _lib.ss_server_done(self._h, slot, ctypes.byref(sp))
        if rc < 0:
            _check(rc, "ss_server_done")
        return bool(rc), int(sp.value)

    def status(self) -> int:
        f = _u32(0)
        _check(_lib.ss_server_status(self._h, ctypes.byref(f)), "ss_server_status")
        return int(f.value)

    def close(self) -> None:
        if self._h:
            _lib.ss_server_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_job_aux_bytes(dtype: int, kind: int, length: int) -> int:
    return _lib.ss_server_job_aux_bytes(dtype, kind, length)


def sort_segment_cap(dtype: int) -> int:
    return _lib.ss_sort_segment_cap(dtype)


def aux_bytes(n: int, dtype: int, algo="smoothed") -> int:
    return _lib.ss_aux_bytes(n, dtype, ALGOS[algo] if isinstance(algo, str) else int(algo))


def probe_bandwidth(t, mode: int, stream=None) -> float:
    """Duration in ms of the read (mode 0), grid-stride read/overwrite (mode 1) or contiguous-block
    read/overwrite (mode 2) probe over the tensor's bytes."""
    ms = ctypes.c_float(0)
    nbytes = t.numel() * t.element_size()
    _check(_lib.ss_probe_bandwidth(ctypes.c_void_p(t.data_ptr()), nbytes, mode, _stream(stream),
                                   ctypes.byref(ms)), "ss_probe_bandwidth")
    return ms.value


def device_info() -> dict:
    v = [_int(0) for _ in range(4)]
    _check(_lib.ss_device_info(*[ctypes.byref(x) for x in v]), "ss_device_info")
    return {"compute_units": v[0].value, "lds_per_block": v[1].value, "major": v[2].value, "minor": v[3].value}
