"""Continuous-batching serving loop for partition and sort jobs.

Jobs arrive over time (partition: split records by key < pivot; sort: the
quicksort of Section 5.2).  A job is admitted when the device arena has room
for its records (admission by bytes: the arena is the memory budget), its
records are generated on the device, and from then on its work joins every
*tick*:

* one batched partition (``ss_partition_segments``) over the segments of all
  jobs with pending work: a whole waiting partition job, and one quicksort
  level of every active sort job (a median-of-3 pivot per segment, or the
  ``key <= p`` pass of a segment whose pivot was its minimum);
* one workgroup-local sort (``ss_sort_segments``) of every sort segment that
  has become short enough.

Jobs that arrive while a tick runs are admitted before the next one, so work
from many jobs overlaps in the same launches.  Every segment's result depends
only on its own contents (lines are counted from the segment's start and the
random offsets from its recursion level), so a job's output bytes are the
same alone and inside any mix.

All device work goes through the C ABI in libss.so; this module only keeps
job state and the arena map.
"""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field

import numpy as np

from . import (SS_KV16, make_params, median3_pivots, partition_segments, sort_segment_cap, sort_segments)

U64MASK = (1 << 64) - 1
RECORD_BYTES = 16  # SS_KV16


class Arena:
    """First-fit allocator over [0, capacity) elements, blocks aligned to `align` elements."""

    def __init__(self, capacity: int, align: int = 32):
        self.capacity = capacity
        self.align = align
        self.free = [(0, capacity)]  # sorted, coalesced (start, length)
        self.used = 0

    def alloc(self, n: int):
        need = -(-max(n, 1) // self.align) * self.align
        for i, (s, l) in enumerate(self.free):
            if l >= need:
                if l == need:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + need, l - need)
                self.used += need
                return s, need
        return None

    def release(self, start: int, size: int):
        self.used -= size
        i = bisect.bisect_left(self.free, (start, 0))
        self.free.insert(i, (start, size))
        # coalesce with neighbours
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)


@dataclass
class Job:
    job_id: int
    kind: str            # "partition" or "sort"
    n: int               # records
    seed: int
    arrival: float       # seconds since the start of the run
    quantile: float = 0.5
    pivot: int = 0       # partition jobs: key < pivot
    # runtime state
    off: int = -1
    block: int = 0
    admitted: float = -1.0
    done: float = -1.0
    split: int = -1
    started: bool = False
    segs: list = field(default_factory=list)    # sort: (start, len, mode, pivot) mode 0: median-of-3, 1: <= p
    leaves: list = field(default_factory=list)  # sort: (start, len) waiting for the leaf sort

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_jobs(count: int, rate_per_s: float, seed: int, p_partition: float = 0.7,
              lo_log2: float = 10.0, hi_log2: float = 26.0):
    """Poisson arrivals, 70% partition / 30% sort, log-uniform lengths (the serving workload)."""
    import workloads
    kinds, lengths, qs = workloads.job_mix(count, seed, p_partition, lo_log2, hi_log2)
    arr = workloads.poisson_arrivals(count, rate_per_s, seed) if rate_per_s > 0 else np.zeros(count)
    jobs = []
    for k in range(count):
        q = float(qs[k])
        jobs.append(Job(job_id=k, kind="sort" if kinds[k] else "partition", n=int(lengths[k]),
                        seed=(seed << 20) ^ k, arrival=float(arr[k]), quantile=q,
                        pivot=min(U64MASK, int(q * (1 << 64)))))
    return jobs


class Server:
    """Runs jobs to completion with continuous batching on one GPU."""

    def __init__(self, budget_bytes: int = 64 << 30, device=None, keep_outputs: bool = False, params=None):
        import torch
        self.torch = torch
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.capacity = budget_bytes // RECORD_BYTES
        self.arena_t = torch.empty((self.capacity, 2), dtype=torch.int64, device=self.device)
        self.arena = Arena(self.capacity)
        self.keep_outputs = keep_outputs
        self.outputs = {}
        self.params = params or {}
        self.cap = sort_segment_cap(SS_KV16)
        self.ticks = 0
        self.max_batch = 0

    # ----------------------------------------------------------------- helpers
    def _generate(self, job: Job):
        import workloads
        view = self.arena_t[job.off:job.off + job.n]
        workloads.splitmix64_torch(job.seed, 0, job.n, self.device, out=view[:, 0])
        view[:, 1] = self.torch.arange(job.n, dtype=self.torch.int64, device=self.device) + (job.job_id << 32)

    def _classify(self, job: Job, start: int, length: int):
        if length > self.cap:
            job.segs.append((start, length, 0, 0))
        elif length >= 2:
            job.leaves.append((start, length))

    def _finish(self, job: Job, now: float):
        job.done = now
        if self.keep_outputs:
            self.outputs[job.job_id] = self.arena_t[job.off:job.off + job.n].cpu().numpy().view(np.uint64).copy()
        self.arena.release(job.off, job.block)

    # ----------------------------------------------------------------- one tick
    def _tick(self, active: list, t0: float):
        torch = self.torch
        # segments of this tick: (job, start, len, mode, host pivot or None)
        work = []
        for job in active:
            if job.kind == "partition":
                if not job.started:
                    work.append((job, job.off, job.n, 2, job.pivot))
                    job.started = True
            else:
                for (s, l, mode, p) in job.segs:
                    work.append((job, s, l, mode, p if mode == 1 else None))
                job.segs = []
        if work:
            m = len(work)
            starts = np.array([w[1] for w in work], dtype=np.uint64)
            lens = np.array([w[2] for w in work], dtype=np.uint64)
            pivots = np.array([w[4] if w[4] is not None else 0 for w in work], dtype=np.uint64)
            need = [i for i, w in enumerate(work) if w[4] is None]
            d_piv = torch.empty(m, dtype=torch.int64, device=self.device)
            if need:
                d_tmp = torch.empty(len(need), dtype=torch.int64, device=self.device)
                hp = median3_pivots(self.arena_t, starts[need], lens[need], d_tmp, host=True)
                pivots[need] = hp
            d_piv.copy_(torch.from_numpy(pivots.view(np.int64)))
            d_split = torch.empty(m, dtype=torch.int64, device=self.device)
            partition_segments(self.arena_t, starts, lens, d_piv, d_split, **self.params)
            splits = d_split.cpu().numpy().view(np.uint64)
            self.max_batch = max(self.max_batch, m)
            now = time.perf_counter() - t0
            for i, (job, s, l, mode, _) in enumerate(work):
                sp = int(splits[i])
                if mode == 2:  # partition job
                    job.split = sp
                    continue
                p = int(pivots[i])
                if mode == 0 and sp == 0:
                    # the pivot is the segment's minimum: gather its copies with key <= p
                    if p == U64MASK:
                        continue  # every key equals the largest key: already sorted
                    job.segs.append((s, l, 1, p + 1))
                    continue
                if mode == 0:
                    self._classify(job, s, sp)
                    self._classify(job, s + sp, l - sp)
                else:
                    self._classify(job, s + sp, l - sp)  # [s, s + sp) holds only the pivot's key
        leaves = [(job, s, l) for job in active if job.kind == "sort" for (s, l) in job.leaves]
        if leaves:
            sort_segments(self.arena_t, np.array([x[1] for x in leaves], dtype=np.uint64),
                          np.array([x[2] for x in leaves], dtype=np.uint64))
            for job in active:
                job.leaves = []
        torch.cuda.synchronize()
        self.ticks += 1
        now = time.perf_counter() - t0
        still = []
        for job in active:
            finished = job.split >= 0 if job.kind == "partition" else (not job.segs and not job.leaves)
            if finished:
                self._finish(job, now)
            else:
                still.append(job)
        return still

    # ----------------------------------------------------------------- run
    def run(self, jobs: list, realtime: bool = True):
        """Serve `jobs` (arrival times in seconds from the start).  With realtime,
        a job is not admitted before its arrival time; otherwise all are available
        at once (closed loop).  Returns the jobs with their completion times."""
        pending = sorted(jobs, key=lambda j: (j.arrival, j.job_id))
        active = []
        t0 = time.perf_counter()
        qi = 0
        waiting = []
        while qi < len(pending) or waiting or active:
            now = time.perf_counter() - t0
            while qi < len(pending) and (not realtime or pending[qi].arrival <= now):
                waiting.append(pending[qi])
                qi += 1
            # FIFO admission while the arena has room
            while waiting:
                job = waiting[0]
                got = self.arena.alloc(job.n)
                if got is None:
                    if not active:
                        raise RuntimeError("job %d (%d records) does not fit the memory budget" % (job.job_id, job.n))
                    break
                waiting.pop(0)
                job.off, job.block = got
                job.admitted = time.perf_counter() - t0
                self._generate(job)
                if job.kind == "sort":
                    self._classify(job, job.off, job.n)
                    if not job.segs and not job.leaves:
                        job.split = 0
                active.append(job)
            if not active:
                if qi < len(pending):
                    time.sleep(max(0.0, min(0.001, pending[qi].arrival - now)))
                continue
            active = self._tick(active, t0)
        return jobs


def latency_summary(jobs: list) -> dict:
    lat = np.array([j.latency for j in jobs]) * 1e3
    recs = sum(j.n for j in jobs)
    span = max(j.done for j in jobs) - min(j.arrival for j in jobs)
    return {"jobs": len(jobs), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
            "records_per_s": round(recs / span, 1), "jobs_per_s": round(len(jobs) / span, 2),
            "span_s": round(span, 4)}
