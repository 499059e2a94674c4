"""The C-ABI library loads and exports what include/ss.h declares; host-side
argument validation (runs before any device work, so no GPU is needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ss.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ss_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("ss_partition", "ss_partition_ex", "ss_quicksort", "ss_quicksort_ex", "ss_partition_batched",
                 "ss_aux_bytes", "ss_strerror", "ss_last_error", "ss_probe_bandwidth", "ss_device_info"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2004_12532_amd as ss
    lib = ctypes.CDLL(ss.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    import paper_2004_12532_amd as ss
    assert ctypes.sizeof(ss.Params) == 32
    # split, aux, 6 x u32, 2 x 32 x u64, 2 x 32 x u32, vmin, vmax, 2 floats, bytes_moved, 2 x u32,
    # first_level_bytes
    assert ctypes.sizeof(ss.Stats) == 8 + 8 + 24 + 2 * 32 * 8 + 2 * 32 * 4 + 16 + 8 + 8 + 8 + 8
    # nclass, 8 x b, 8 x group_bytes, (pad), 8 x max_len, 8 x ms
    assert ctypes.sizeof(ss.Tuning) == 4 + 32 + 32 + 4 + 64 + 32


def _rc(fn, *args):
    return fn(*args)


def test_argument_validation_without_device():
    import paper_2004_12532_amd as ss
    L = ss.lib
    split = ctypes.c_size_t(7)
    assert L.ss_partition(None, 10, ss.SS_U64, 5, ctypes.byref(split)) == -1          # null with n > 0
    assert L.ss_partition(ctypes.c_void_p(0x1004), 10, ss.SS_U64, 5, ctypes.byref(split)) == -1  # misaligned
    assert L.ss_partition(ctypes.c_void_p(0x1008), 10, ss.SS_KV16, 5, ctypes.byref(split)) == -1  # kv needs 16
    assert L.ss_partition(ctypes.c_void_p(0x1000), 10, 9, 5, ctypes.byref(split)) == -1  # bad dtype
    assert L.ss_partition(ctypes.c_void_p(0x1000), 10, ss.SS_U64, 5, None) == -1        # no split out
    for bad in (ss.make_params(b=3), ss.make_params(b=4), ss.make_params(b=1024), ss.make_params(tile_bytes=4096),
                ss.make_params(max_levels=33), ss.make_params(algo=7),
                ss.make_params(engine="lds", tile_bytes=131072), ss.make_params(engine="lds", exchange=True)):
        rc = L.ss_partition_ex(ctypes.c_void_p(0x1000), 10, ss.SS_U64, 5, ctypes.byref(bad), None, None,
                               ctypes.byref(split), None)
        assert rc == -1, (bad.b, bad.tile_bytes, bad.max_levels, bad.algo)
    bad = ss.make_params()
    bad.engine = 9
    assert L.ss_partition_ex(ctypes.c_void_p(0x1000), 10, ss.SS_U64, 5, ctypes.byref(bad), None, None,
                             ctypes.byref(split), None) == -1
    assert split.value == 7  # untouched on argument errors
    assert L.ss_quicksort(None, 5, ss.SS_U32) == -1
    # the per-array loop: null or decreasing offsets, null pivots or splits
    off = (ctypes.c_uint64 * 3)(0, 8, 4)
    piv = (ctypes.c_uint64 * 2)(1, 2)
    p = ss.make_params()
    each = L.ss_partition_each
    assert each(ctypes.c_void_p(0x1000), None, 2, ss.SS_U64, piv, ctypes.c_void_p(0x2000), ctypes.byref(p), None,
                None) == -1
    assert each(ctypes.c_void_p(0x1000), off, 2, ss.SS_U64, piv, ctypes.c_void_p(0x2000), ctypes.byref(p), None,
                None) == -1
    off[2] = 12
    assert each(ctypes.c_void_p(0x1000), off, 2, ss.SS_U64, None, ctypes.c_void_p(0x2000), ctypes.byref(p), None,
                None) == -1
    assert each(ctypes.c_void_p(0x1000), off, 2, ss.SS_U64, piv, None, ctypes.byref(p), None, None) == -1
    assert each(ctypes.c_void_p(0x1000), off, 2, ss.SS_U64, piv, ctypes.c_void_p(0x2004), ctypes.byref(p), None,
                None) == -1
    assert each(ctypes.c_void_p(0x1000), off, 0, ss.SS_U64, piv, None, ctypes.byref(p), None, None) == 0  # nothing


def test_strerror_and_aux_bytes():
    import paper_2004_12532_amd as ss
    for code in (0, -1, -2, -3, -4, -5):
        assert ss.lib.ss_strerror(code)
    small = ss.aux_bytes(1 << 30, ss.SS_U64, "smoothed")
    assert small < (1 << 22)                                   # polylog-sized workspace
    assert small == ss.aux_bytes(1 << 20, ss.SS_U64, "smoothed")
    ls = ss.aux_bytes(1 << 30, ss.SS_U64, "lowspace")
    # per 64 elements: a 32-bit block count/prefix of the array read forward and a 32-bit count of it
    # read reversed (the top preprocessing level counts both before the roles are known)
    assert ls - small >= 2 * (1 << 30) // 64 * 4
    assert ls - small < 2 * (1 << 30) // 64 * 4 + (1 << 20)


def test_line_count_limit_rejected_before_device_work():
    import paper_2004_12532_amd as ss
    split = ctypes.c_size_t(3)
    p = ss.make_params(b=16)  # 64-byte u32 lines
    rc = ss.lib.ss_partition_ex(ctypes.c_void_p(0x1000), (1 << 36) + 5, ss.SS_U32, 5, ctypes.byref(p), None, None,
                                ctypes.byref(split), None)
    assert rc == -1 and b"lines" in ss.lib.ss_last_error()


def test_server_engine_argument_validation_without_device():
    import paper_2004_12532_amd as ss
    L = ss.lib
    out = ctypes.c_void_p(1)
    assert L.ss_server_create(None, 10, ss.SS_KV16, 4, 4, None, ctypes.byref(out)) == -1        # null base
    assert L.ss_server_create(ctypes.c_void_p(0x1008), 10, ss.SS_KV16, 4, 4, None, ctypes.byref(out)) == -1
    assert L.ss_server_create(ctypes.c_void_p(0x1000), 10, ss.SS_KV16, 0, 4, None, ctypes.byref(out)) == -1
    assert out.value is None                                  # cleared on error
    assert L.ss_server_submit(None, 0, 0, 1, 0, 0) == -1
    assert L.ss_server_tick(None, 1) == -1
    assert ss.server_job_aux_bytes(ss.SS_KV16, 1, 1 << 20) > ss.server_job_aux_bytes(ss.SS_KV16, 0, 1 << 20)


def test_struct_sizes_equal_the_c_compilers(tmp_path):
    """The ctypes mirrors have the sizes a C compiler gives the header's structs."""
    import subprocess
    import paper_2004_12532_amd as ss
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "ss.h"\nint main(void) { printf("%zu %zu %zu\\n", '
                   'sizeof(ss_params), sizeof(ss_stats), sizeof(ss_batched_tuning)); return 0; }\n')
    exe = tmp_path / "sizes"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    sizes = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert sizes == [ctypes.sizeof(ss.Params), ctypes.sizeof(ss.Stats), ctypes.sizeof(ss.Tuning)]
