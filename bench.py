#!/usr/bin/env python3
"""Benchmark: in-place partition of 2^30 uint64 keys on one MI355X.

One step = one complete partition (every Partial Partition Step of the
recursion, the final reduction and the split read back) of a fresh copy of
the input, already resident in HBM.  The K timed steps use K distinct copies
restored before the timed region, so every step sees the same i.i.d.
workload.  `value` is the effective partition bandwidth 2 * n * 8 bytes per
step over the wall time of the K steps (bracketed by device synchronization).

The roofline object describes the dominant kernel (the first Partial
Partition Step, which moves every element once): its algorithmic bytes
2 * n * 8 over its average duration measured by HIP events that the library
records on the launch stream, against the MI355X HBM peak of 8 TB/s.

The CPU baseline is the serial oracle partition (single thread) on a bounded
sample of the same workload on this host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
WORKLOADS = {
    # name: (dtype, log2 n, pivot quantile or "desc")
    "partition_u64_2p30_q0.5": ("u64", 30, 0.5),
    "partition_u64_2p30_q0.1": ("u64", 30, 0.1),
    "partition_u64_2p30_q0.01": ("u64", 30, 0.01),
    "partition_u64_2p30_desc": ("u64", 30, "desc"),
    # stride-aligned adversary: predecessors fill exactly the lines l with (l mod g) < g/2 for the
    # default geometry (512-byte lines, 256 lines per group), pivot 2^63
    "partition_u64_2p30_stride_adv": ("u64", 30, "adv"),
}
LEVEL_SOURCES = ["paper_2004_12532_amd/csrc/ss_level_rs.hip", "paper_2004_12532_amd/csrc/ss_level_rs.h",
                 "paper_2004_12532_amd/csrc/ss_level_xch.hip", "paper_2004_12532_amd/csrc/ss_levelctx.h",
                 "paper_2004_12532_amd/csrc/ss_device.h", "paper_2004_12532_amd/csrc/ss_common.h"]
# Counter summaries of the first level per workload (taken with rocprofv3 --pmc).
COUNTER_FILES = {"partition_u64_2p30_q0.5": os.path.join(ROOT, "profiles", "level0_u64_2p30_counters.json"),
                 "partition_u64_2p30_q0.01": os.path.join(ROOT, "profiles", "level0_u64_2p30_q0.01_counters.json")}


def level_source_digest() -> str:
    h = hashlib.sha256()
    for p in LEVEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(workload: str):
    """HBM bytes per launch of the first-level kernel from the committed counter
    summary of this workload, if it was taken on the current kernel source; else None."""
    try:
        with open(COUNTER_FILES[workload]) as f:
            c = json.load(f)
    except (KeyError, OSError, ValueError):
        return None
    if c.get("kernel_source_digest") != level_source_digest():
        return None
    return c.get("traffic_bytes_per_launch")


def cpu_baseline(host_keys, pivot: int, runs: int = 3):
    """The serial oracle partition of the same 2^30 keys (copied from the GPU to
    the host), median of `runs`, on one core: the calling thread is pinned with
    os.sched_setaffinity for the timed runs and its mask restored afterwards
    (the affinity of a thread is its own, so the HIP runtime's threads keep
    theirs)."""
    import numpy as np

    import oracle

    n = host_keys.size
    work = np.empty_like(host_keys)
    mask = os.sched_getaffinity(0)
    core = min(mask)
    times = []
    try:
        os.sched_setaffinity(0, {core})
        for _ in range(runs):
            np.copyto(work, host_keys)
            t0 = time.perf_counter()
            oracle.partition(work, pivot)
            times.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, mask)
    del work
    t = sorted(times)[len(times) // 2]
    return {"value": round(2 * n * 8 / t / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "serial two-pointer partition of the same 2^30 i.i.d. uint64 keys at the median (copied to "
                      "the host), %d runs pinned to core %d, median %.3f s (%.3g elements/s)" % (runs, core, t, n / t),
            "seconds": [round(x, 3) for x in times], "host_cpu": _host_cpu(), "host_threads": os.cpu_count()}


def _host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _exit_multi_gpu(gpus):
    if gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU (it has no multi-GPU path); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)


def _u64_tensor_scalar(torch, v, dev):
    return torch.tensor([v - (1 << 64) if v >> 63 else v], dtype=torch.int64, device=dev)


def run_partition(args, workload, algo="smoothed"):
    """The headline: K partitions of fresh resident copies of 2^30 uint64 keys."""
    import numpy as np
    import torch

    import paper_2004_12532_amd as ss
    import workloads

    algo, _, mode = algo.partition("+")
    modes = {"auto": "auto", "off": False, "all": True, "skewed": "skewed"}
    exchange = modes[mode] if mode else modes[args.exchange]
    dtype, log2n, q = WORKLOADS[workload]
    n = 1 << log2n
    w = 8
    dev = torch.device("cuda", 0)

    if q == "adv":
        g = workloads.stride_groups(n, 64, 256)
        pristine = workloads.stride_adversarial_u64_torch(n, workloads.config_seed(1), 64, g, dev)
        pivot = 1 << 63
    else:
        pristine = workloads.keys_u64_torch(n, workloads.config_seed(1), dev)
        pivot = workloads.pivot_at_quantile_torch(pristine, 0.5 if q == "desc" else q)
    if q == "desc":
        pristine = workloads.sort_descending_u64_torch(pristine)
    expected = int((workloads.to_unsigned_order(pristine) <
                    workloads.to_unsigned_order(_u64_tensor_scalar(torch, pivot, dev))).sum().item())
    bufs = [torch.empty_like(pristine) for _ in range(args.steps)]
    kw = dict(algo=algo, b=args.b, tile_bytes=args.tile_bytes, exchange=exchange)

    def restore(k):
        bufs[k].copy_(pristine)

    for k in range(args.steps):
        restore(k)
    for k in range(args.warmup):
        ss.partition(bufs[k % args.steps], pivot, **kw)
        restore(k % args.steps)
    d_splits = torch.empty(args.steps, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    # The timed region: K partitions of K resident copies, issued back to back
    # on the current stream (each call runs its whole level chain and its base
    # case on the device and writes its split there).
    t0 = time.perf_counter()
    for k in range(args.steps):
        ss.partition_async(bufs[k], pivot, d_splits[k:k + 1], **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    splits = [int(x) for x in d_splits.cpu().tolist()]
    ok = all(sp == expected for sp in splits)

    # Per-call figures, after the timed region: synchronous calls with HIP
    # events recorded by the library on the launch stream around the first
    # level's kernel and around the whole call.
    nstat = min(args.steps, 5)
    for k in range(nstat):
        restore(k)
    torch.cuda.synchronize()
    level_ms, total_ms, sync_ms, stats = [], [], [], None
    for k in range(nstat):
        c0 = time.perf_counter()
        split, st = ss.partition(bufs[k], pivot, stats=True, time=True, **kw)
        sync_ms.append((time.perf_counter() - c0) * 1e3)
        ok = ok and split == expected
        level_ms.append(st["first_level_ms"])
        total_ms.append(st["total_ms"])
        stats = st

    alg_bytes = 2.0 * n * w
    value = alg_bytes * args.steps / wall / 1e9
    mean_level_ms = sum(level_ms) / len(level_ms)
    # The first level's algorithmic bytes: 2 n w in the stable form; in the
    # exchange form it reads n w and writes only the elements it stored.
    first_bytes = float(stats["first_level_bytes"])
    achieved = first_bytes / (mean_level_ms / 1e3) / 1e9

    probe = None
    if not args.no_probe:
        ms_rw = min(ss.probe_bandwidth(bufs[0], 2) for _ in range(3))
        ms_rws = min(ss.probe_bandwidth(bufs[0], 1) for _ in range(3))
        ms_r = min(ss.probe_bandwidth(bufs[0], 0) for _ in range(3))
        probe = {"rw_GBps": round(alg_bytes / ms_rw / 1e6, 1), "rw_gridstride_GBps": round(alg_bytes / ms_rws / 1e6, 1),
                 "read_GBps": round(n * w / ms_r / 1e6, 1),
                 "note": "rw: every workgroup reads and overwrites one contiguous block of the 8 GiB array in "
                         "32 KiB steps (the fastest in-place pattern measured); rw_gridstride: the same bytes "
                         "grid-stride; read: read only"}
    host_keys = None
    if not args.no_cpu_baseline and q != "adv":
        host_keys = pristine.cpu().numpy().view(np.uint64)
    del bufs
    torch.cuda.empty_cache()

    traffic = counter_traffic(workload) if (algo == "smoothed" and exchange == "auto"
                                            and not args.b and not args.tile_bytes) else None
    # the exchange kernel: 512 threads per 32 KiB group when the library chooses the form, the
    # forced form's 256-thread shape otherwise
    xshape = ("512,4", " chosen from the key sample") if exchange == "auto" else ("256,8", "")
    out = {
        "metric": "partition GB/s & % HBM peak, 2^30 u64; batched vs per-array launch; p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 4),
        "timing": "K asynchronous calls on one stream, wall clock between device synchronizations",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "n": n,
            "pivot_quantile": q,
            "algo": algo,
            "exchange": exchange,
            "b": stats["b"],
            "s_max": stats["s_max"],
            "grid": stats["grid"],
            "parallelism": "single GPU",
        },
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBPS, 2),
        "elements_per_s": round(n * args.steps / wall, 1),
        "splits_correct": ok,
        "levels": stats["levels"],
        "level_sizes": [hi - lo for lo, hi in zip(stats["level_lo"], stats["level_hi"])],
        "first_level_ms": round(mean_level_ms, 4),
        "call_ms_device": round(sum(total_ms) / len(total_ms), 4),
        "call_ms_sync": round(sorted(sync_ms)[len(sync_ms) // 2], 4),
        "aux_bytes": stats["aux_bytes"],
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "frac_of_probe": round(achieved / probe["rw_GBps"], 4) if probe else None,
            "traffic": traffic,
            "kernel": ({"smoothed": "k_level_rs<uint64_t,%s,first,exchange> (first Partial Partition Step, "
                                    "write-minimal exchange form%s)" % xshape,
                        "strided": "k_level_rs<uint64_t,%s,first,exchange> (Partial Partition Step, offsets 0, "
                                   "exchange form%s)" % xshape,
                        "hybrid": "k_level_rs<uint64_t,%s,first,exchange> (Partial Partition Step before the "
                                  "Low-Space pass over the middle, exchange form%s)" % xshape}.get(algo)
                       if stats["exchange_mask"] & 1 else None) or
                      {"smoothed": "k_level_rs<uint64_t,512,16,first,staged> (first Partial Partition Step)",
                       "strided": "k_level_rs<uint64_t,512,16,first,staged> (Partial Partition Step, offsets 0)",
                       "lowspace": "whole Low-Space call (all its kernels)",
                       "hybrid": "k_level_rs<uint64_t,512,16,first,staged> (Partial Partition Step before the "
                                 "Low-Space pass over the middle)",
                       "mediumspace": "whole Medium-Space call (all its kernels and the copy back)",
                       "highspace": "whole High-Space call (all its kernels and the copy back)",
                       "implicit": "whole implicit Blocked-Prefix-Sum call (all its kernels)"}[algo],
            "algorithmic_bytes_per_launch": first_bytes,
        },
        "probe": probe,
    }
    if host_keys is not None:
        out["cpu_baseline"] = cpu_baseline(host_keys, pivot)
        del host_keys
    if not ok:
        out["error"] = "split mismatch %s vs expected %d" % (splits, expected)
    return out


def run_quicksort(args, distinct):
    """K quicksorts of fresh copies of 2^28 uint32 keys (uniform, or 1024 distinct values)."""
    import numpy as np
    import torch

    import oracle
    import paper_2004_12532_amd as ss
    import workloads

    n = 1 << 28
    dev = torch.device("cuda", 0)
    seed = workloads.config_seed(2)
    pristine = (workloads.keys_few_distinct_u32_torch(n, seed, dev, distinct) if distinct
                else workloads.keys_u32_torch(n, seed, dev))
    steps = min(args.steps, 8)
    bufs = [pristine.clone() for _ in range(steps)]
    ss.quicksort(pristine.clone())  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        stats.append(ss.quicksort(bufs[k], stats=True, time=True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ok = bool((bufs[0][1:].to(torch.int64) & 0xFFFFFFFF >= bufs[0][:-1].to(torch.int64) & 0xFFFFFFFF).all())
    # CPU oracle sort on a 2^24 sample of the same generator
    m = 1 << 24
    a = workloads.keys_few_distinct_u32(m, seed, distinct) if distinct else workloads.keys_u32(m, seed)
    t1 = time.perf_counter()
    oracle.quicksort(a)
    tc = time.perf_counter() - t1
    return {"metric": "quicksort elements/s, 2^28 uint32" + (" (%d distinct values)" % distinct if distinct else ""),
            "value": round(n * steps / wall, 1), "unit": "elements/s", "ms_per_sort": round(wall / steps * 1e3, 3),
            "device_ms": round(sum(x["total_ms"] for x in stats) / steps, 3),
            "partition_levels": stats[0]["levels"], "sorted": ok,
            "effective_GBps_per_level": round(2 * n * 4 * stats[0]["levels"] / (wall / steps) / 1e9, 1),
            "config": {"workload": "quicksort_u32_2p28" + ("_d%d" % distinct if distinct else ""), "n": n,
                       "leaf": 1 << 14, "pivot": "median of 64 sampled keys"},
            "cpu_baseline": {"value": round(m / tc, 1), "unit": "elements/s", "cores": 1, "kind": "oracle",
                             "sample": "serial quicksort of 2^24 keys of the same generator, %.3f s" % tc}}


def run_batched(args):
    """20,000 uint64 arrays, log-normal lengths around 2^14: one batched call against one
    single-array call per array (ss_partition_each: the loop runs in C, each array's level
    chain planned from its length, one launch for arrays that fit one group)."""
    import numpy as np
    import torch

    import paper_2004_12532_amd as ss
    import workloads

    dev = torch.device("cuda", 0)
    seed = workloads.config_seed(3)
    lens = workloads.lognormal_lengths(20000, seed)
    offs = np.zeros(len(lens) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lens)
    total = int(offs[-1])
    pristine = workloads.keys_u64_torch(total, seed, dev)
    qs = workloads.uniform_quantiles(len(lens), seed)
    piv = np.array([min((1 << 64) - 1, int(q * (1 << 64))) for q in qs], dtype=np.uint64)
    d_piv = torch.from_numpy(piv.view(np.int64).copy()).to(dev)
    d_split = torch.empty(len(lens), dtype=torch.int64, device=dev)
    buf = torch.empty_like(pristine)
    reps = max(1, min(args.steps, 5))

    def timed(graph):
        ts = []
        for r in range(reps + 1):   # with graph=True the first call captures the graph
            buf.copy_(pristine)
            d_split.fill_(-1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ss.partition_batched(buf, offs, d_piv, d_split, graph=graph)
            torch.cuda.synchronize()
            if r:
                ts.append(time.perf_counter() - t0)
        return min(ts), d_split.cpu().numpy().copy()

    # batched, one call over all arrays: the autotuned size classes, with eager launches and
    # with the level chain replayed from a captured HIP graph, then the default geometry
    # (measured after the others, so that every configuration runs on an equally warm GPU)
    ss.set_batched_tuning("u64", None)
    tune_t0 = time.perf_counter()
    tuning = ss.autotune_batched("u64")
    tune_s = time.perf_counter() - tune_t0
    te, splits_e = timed(False)
    tg, splits_g = timed(True)
    ss.set_batched_tuning("u64", None)
    t_default, splits_b = timed(False)
    ss.set_batched_tuning("u64", tuning)   # leave the tuned table installed, as the autotuner does

    # per array: one single-array call per array, issued from C on one stream; the
    # throughput run does not synchronize, the latency run records an event after
    # every array (completion time since the first launch)
    pivots = [int(x) for x in piv]
    pt = []
    for r in range(reps + 1):
        buf.copy_(pristine)
        d_split.fill_(-1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ss.partition_each(buf, offs, pivots, d_split)
        torch.cuda.synchronize()
        if r:
            pt.append(time.perf_counter() - t0)
    splits_p = d_split.cpu().numpy()
    buf.copy_(pristine)
    torch.cuda.synchronize()
    lat = ss.partition_each(buf, offs, pivots, d_split, latencies=True)
    bytes_ = 2 * 8 * total
    # the batched call as a user would configure it: the fastest of the measured configurations
    timings = {"tuned, eager": te, "tuned, graph": tg, "default geometry, eager": t_default}
    best_cfg = min(timings, key=timings.get)
    tb = timings[best_cfg]
    tp = min(pt)
    return {"metric": "batched partition GB/s and p99 latency, 20000 uint64 arrays (log-normal, median 2^14)",
            "value": round(bytes_ / tb / 1e9, 1), "unit": "GB/s",
            "batched": {"ms": round(tb * 1e3, 3), "GBps": round(bytes_ / tb / 1e9, 1),
                        "elements_per_s": round(total / tb, 1),
                        # every array of a batched call completes when the call does
                        "p50_ms": round(tb * 1e3, 3), "p99_ms": round(tb * 1e3, 3),
                        "eager_ms": round(te * 1e3, 3), "graph_ms": round(tg * 1e3, 3),
                        "configuration": best_cfg, "default_geometry_ms": round(t_default * 1e3, 3)},
            "autotune": {"seconds": round(tune_s, 2),
                         "classes": [{k: c[k] for k in ("max_len", "b", "group_bytes")} for c in tuning["classes"]]},
            "per_array": {"ms": round(tp * 1e3, 3), "GBps": round(bytes_ / tp / 1e9, 1),
                          "elements_per_s": round(total / tp, 1), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                          "p99_ms": round(float(np.percentile(lat, 99)), 3),
                          "issue": "ss_partition_each: one single-array call per array from C, level chain "
                                   "planned per array, one launch for arrays that fit one group"},
            "speedup": round(tp / tb, 2),
            "p99_ratio": round(float(np.percentile(lat, 99)) / (tb * 1e3), 2),
            "splits_agree": bool(np.array_equal(splits_b, splits_p) and np.array_equal(splits_b, splits_g)
                                 and np.array_equal(splits_b, splits_e)),
            "config": {"workload": "batched_u64_20000", "arrays": len(lens), "elements": total,
                       "pivot": "u-quantile of the key distribution, u ~ U[0.05, 0.95]"}}


def run_serving(args):
    """KV16 jobs (70% partition, 30% sort), log-uniform lengths 2^10..2^26, 64 GiB budget:
    closed-loop capacity, then Poisson arrivals at 50%, 80% and 95% of it."""
    from paper_2004_12532_amd.serving import Server, latency_summary, make_jobs

    njobs = args.serving_jobs
    srv = Server(budget_bytes=64 << 30)
    srv.run(make_jobs(args.serving_warmup, 0.0, 11), realtime=False)   # warm-up jobs, not counted
    cap_jobs = make_jobs(njobs, 0.0, 12)
    srv.run(cap_jobs, realtime=False)
    cap = latency_summary(cap_jobs)
    C = cap["jobs_per_s"]
    print("serving: capacity %.2f jobs/s" % C, file=sys.stderr, flush=True)
    loads = {}
    for frac in (0.5, 0.8, 0.95):
        jobs = make_jobs(njobs, frac * C, 13 + int(frac * 100))
        srv.run(jobs, realtime=True)
        loads["%.2f" % frac] = latency_summary(jobs)
        print("serving: load %.2f done: %s" % (frac, loads["%.2f" % frac]), file=sys.stderr, flush=True)
    return {"metric": "serving p50/p99 latency and records/s (KV16 partition and sort jobs)",
            "value": loads["0.80"]["p99_ms"], "unit": "ms (p99 at 80% load)", "higher_is_better": False,
            "capacity": cap, "loads": loads, "ticks": srv.ticks, "max_jobs_per_tick": srv.max_batch,
            "config": {"workload": "serving_kv16", "jobs_per_load": njobs, "warmup_jobs": args.serving_warmup,
                       "budget_GiB": 64, "mix": "70% partition, 30% quicksort", "lengths": "log-uniform 2^10..2^26",
                       "p99_sample": "%d completed jobs per load" % njobs}}


SUITE = ["partition_u64_2p30_q0.1", "partition_u64_2p30_q0.01", "partition_u64_2p30_desc",
         "partition_u64_2p30_stride_adv", "partition_u64_2p30_stride_adv:strided",
         "partition_u64_2p30_q0.5:strided", "partition_u64_2p30_q0.5:lowspace", "partition_u64_2p30_q0.5:hybrid",
         "partition_u64_2p30_q0.5:mediumspace", "partition_u64_2p30_q0.5:highspace",
         "partition_u64_2p30_q0.5:implicit",
         "quicksort_u32_2p28", "quicksort_u32_2p28_d1024", "batched_u64_20000", "serving_kv16"]


def run_named(args, name):
    if name.startswith("partition_"):
        wl, _, algo = name.partition(":")
        return run_partition(args, wl, algo or args.algo)
    if name == "quicksort_u32_2p28":
        return run_quicksort(args, None)
    if name == "quicksort_u32_2p28_d1024":
        return run_quicksort(args, 1024)
    if name == "batched_u64_20000":
        return run_batched(args)
    if name == "serving_kv16":
        return run_serving(args)
    raise SystemExit("unknown workload " + name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="partition_u64_2p30_q0.5",
                    choices=sorted(WORKLOADS) + ["quicksort_u32_2p28", "quicksort_u32_2p28_d1024",
                                                 "batched_u64_20000", "serving_kv16"])
    ap.add_argument("--algo", default="smoothed",
                    choices=["smoothed", "strided", "lowspace", "hybrid", "mediumspace", "highspace", "implicit"])
    ap.add_argument("--b", type=int, default=0)
    ap.add_argument("--tile-bytes", type=int, default=0)
    ap.add_argument("--exchange", choices=["auto", "off", "all", "skewed"], default="auto",
                    help="single-array partitions: the library's choice from a key sample (auto), the stable "
                         "partition of every group (off), the write-minimal exchange of misplaced pairs in every "
                         "group (all) or only in groups with few of them (skewed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=4000)
    ap.add_argument("--serving-warmup", type=int, default=200)
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: leave out the batched and serving sub-objects of the default run")
    ap.add_argument("--suite", default="", help="also run the other workloads, writing their lines to this file")
    args = ap.parse_args()
    _exit_multi_gpu(args.gpus)
    if not 1 <= args.steps <= 24:
        print("bench.py: --steps must be in [1, 24] (one input copy per timed step)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    out = run_named(args, args.workload)
    if args.workload == "partition_u64_2p30_q0.5" and not args.no_extras and not out.get("error"):
        # the rest of the metric: batched vs per-array launch and serving latency, as sub-objects
        # of the same line (each workload keeps its own config inside)
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        b = run_batched(args)
        b["bench_wall_s"] = round(time.perf_counter() - t0, 1)
        out["batched"] = {k: b[k] for k in ("batched", "per_array", "speedup", "p99_ratio", "splits_agree",
                                            "autotune", "config", "bench_wall_s")}
        print("bench: batched done in %.1f s" % b["bench_wall_s"], file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        sv = run_serving(args)
        sv["bench_wall_s"] = round(time.perf_counter() - t0, 1)
        out["serving"] = {k: sv[k] for k in ("capacity", "loads", "ticks", "max_jobs_per_tick", "config",
                                             "bench_wall_s")}
        print("bench: serving done in %.1f s" % sv["bench_wall_s"], file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    if args.suite:
        sub = argparse.Namespace(**vars(args))
        sub.no_cpu_baseline = True
        sub.no_probe = True
        sub.steps = min(args.steps, 5)
        sub.warmup = 1
        with open(args.suite, "w") as f:
            for name in SUITE:
                t0 = time.perf_counter()
                res = run_named(sub, name)
                res["bench_wall_s"] = round(time.perf_counter() - t0, 1)
                f.write(json.dumps(res) + "\n")
                f.flush()
                print("suite: %s done in %.1f s" % (name, res["bench_wall_s"]), file=sys.stderr, flush=True)
                torch.cuda.empty_cache()
    if out.get("error"):
        print("bench.py: " + out["error"], file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
