"""Continuous-batching serving loop for partition and sort jobs.

Jobs arrive over time (partition: split records by key < pivot; sort: the
quicksort of Section 5.2).  A job is admitted when the memory budget has room
for it -- its input bytes in the device arena plus the auxiliary bytes its
pending segments, leaves and groups can occupy in the engine's device state
(``ss_server_job_aux_bytes``) -- and a job slot is free.  Its records are then
generated on the device and it is submitted to the device-resident engine
(``ss_server_*`` in libss.so), which keeps every job's state on the device.
Each tick is one fixed launch sequence over the pending work of all admitted
jobs: one batched Smoothed Striding partition over every pending segment (a
whole partition job, or one quicksort segment of a sort job), then the
workgroup-local sort of every short sort segment.  Jobs that arrive while
ticks run are admitted before the next tick, so work from many jobs overlaps
in the same launches.  The host issues tick T + 1 before it looks at tick T's
results (per-job done flags in mapped memory), so the device never idles on
the host.  Every segment's result depends only on its own contents (lines are
counted from the segment's start and the random offsets from its recursion
level), so a job's output bytes are the same alone and inside any mix.

This module only keeps arrival times, the arena map and the admission
accounting; all device work goes through the C ABI.
"""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field

import numpy as np

from . import SS_KV16, ServerEngine, server_job_aux_bytes, sort_segment_cap

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
    cancel_at: float = -1.0  # >= 0: the client withdraws the job at this time (seconds from the start)
    # runtime state
    off: int = -1
    block: int = 0
    slot: int = -1
    aux: int = 0
    admitted: float = -1.0
    done: float = -1.0
    split: int = -1
    status: str = "pending"  # then "done", "rejected" (can never fit the budget) or "cancelled"

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


def never_fits(n: int, aux: int, capacity: int, aux_budget: int) -> bool:
    """A job of n records and `aux` auxiliary bytes cannot be admitted even by an
    idle server: it is rejected at arrival instead of waiting forever."""
    return n > capacity or aux > aux_budget


class Server:
    """Runs jobs to completion with continuous batching on one GPU."""

    def __init__(self, budget_bytes: int = 64 << 30, device=None, keep_outputs: bool = False,
                 max_jobs: int = 4096, max_segments: int = 1 << 16):
        import torch
        self.torch = torch
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        # the budget holds the records' arena and the engine's auxiliary state
        per_seg = server_job_aux_bytes(SS_KV16, 0, 0) - 64
        self.aux_budget = min(budget_bytes // 64, max_segments * per_seg)
        self.capacity = (budget_bytes - self.aux_budget) // RECORD_BYTES
        self.arena_t = torch.empty((self.capacity, 2), dtype=torch.int64, device=self.device)
        self.arena = Arena(self.capacity)
        self.engine = ServerEngine(self.arena_t, max_jobs, max_segments, stream=torch.cuda.current_stream())
        self.free_slots = list(range(max_jobs - 1, -1, -1))
        self.aux_used = 0
        self.keep_outputs = keep_outputs
        self.outputs = {}
        self.cap = sort_segment_cap(SS_KV16)
        self.ticks = 0
        self.max_batch = 0

    # ----------------------------------------------------------------- helpers
    def _generate(self, job: Job):
        import workloads
        view = self.arena_t[job.off:job.off + job.n]
        workloads.splitmix64_torch(job.seed, 0, job.n, self.device, out=view[:, 0])
        view[:, 1] = self.torch.arange(job.n, dtype=self.torch.int64, device=self.device) + (job.job_id << 32)

    def _admit(self, job: Job, t0: float) -> bool:
        kind = 0 if job.kind == "partition" else 1
        aux = server_job_aux_bytes(SS_KV16, kind, job.n)
        if not self.free_slots or self.aux_used + aux > self.aux_budget:
            return False
        got = self.arena.alloc(job.n)
        if got is None:
            return False
        job.off, job.block = got
        job.slot = self.free_slots.pop()
        job.aux = aux
        self.aux_used += aux
        job.admitted = time.perf_counter() - t0
        self._generate(job)
        self.engine.submit(job.slot, job.off, job.n, kind, job.pivot)
        return True

    def _finish(self, job: Job, now: float, split: int):
        job.done = now
        if job.status == "cancelled":
            # withdrawn while on the device: its work ran to the end of a tick; the result is dropped
            pass
        else:
            job.status = "done"
            if job.kind == "partition":
                job.split = split
            if self.keep_outputs:
                self.outputs[job.job_id] = \
                    self.arena_t[job.off:job.off + job.n].cpu().numpy().view(np.uint64).copy()
        self.arena.release(job.off, job.block)
        self.free_slots.append(job.slot)
        self.aux_used -= job.aux

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
                job = pending[qi]
                qi += 1
                kind = 0 if job.kind == "partition" else 1
                if never_fits(job.n, server_job_aux_bytes(SS_KV16, kind, job.n), self.capacity, self.aux_budget):
                    job.status, job.done = "rejected", now
                    continue
                waiting.append(job)
            # withdrawals: a waiting job leaves the queue, an admitted one has its result dropped
            for job in [j for j in waiting if 0 <= j.cancel_at <= now]:
                waiting.remove(job)
                job.status, job.done = "cancelled", now
            for job in active:
                if 0 <= job.cancel_at <= now:
                    job.status = "cancelled"
            # FIFO admission while the budget has room
            while waiting and self._admit(waiting[0], t0):
                active.append(waiting.pop(0))
            if waiting and not active:  # cannot happen: jobs that never fit were rejected
                raise RuntimeError("job %d (%d records) was not admitted by an idle server"
                                   % (waiting[0].job_id, waiting[0].n))
            if not active:
                if qi < len(pending):
                    time.sleep(max(0.0, min(0.001, pending[qi].arrival - now)))
                continue
            self.engine.tick(max(j.n for j in active))
            self.ticks += 1
            self.max_batch = max(self.max_batch, len(active))
            # look at the results of the previous tick while this one runs
            if self.engine.wait(1):
                raise RuntimeError("serving engine capacity exceeded (flags %d)" % self.engine.status())
            now = time.perf_counter() - t0
            still = []
            for job in active:
                fin, split = self.engine.done(job.slot)
                if fin:
                    self._finish(job, now, split)
                else:
                    still.append(job)
            active = still
        self.engine.wait(0)
        flags = self.engine.status()
        if flags:
            raise RuntimeError("serving engine capacity exceeded (flags %d)" % flags)
        return jobs


def latency_summary(jobs: list) -> dict:
    """Latency and throughput over the jobs that completed (rejected and cancelled ones excluded)."""
    jobs = [j for j in jobs if j.status == "done"]
    lat = np.array([j.latency for j in jobs]) * 1e3
    recs = sum(j.n for j in jobs)
    span = max(j.done for j in jobs) - min(j.arrival for j in jobs)
    return {"jobs": len(jobs), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "mean_ms": round(float(lat.mean()), 3),
            "records_per_s": round(recs / span, 1), "jobs_per_s": round(len(jobs) / span, 2),
            "span_s": round(span, 4)}
