"""GPU: the serving loop's results against the oracle, and the same bytes for a
job served alone and inside a mix of concurrently admitted jobs."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _server(ss, budget=4 << 30):
    from paper_2004_12532_amd.serving import Server
    return Server(budget_bytes=budget, keep_outputs=True)


def _input_of(job):
    import workloads
    a = np.empty((job.n, 2), dtype=np.uint64)
    a[:, 0] = workloads.splitmix64_np(job.seed, 0, job.n)
    a[:, 1] = np.arange(job.n, dtype=np.uint64) + np.uint64(job.job_id << 32)
    return a


def _check_job(job, out):
    a0 = _input_of(job)
    if job.kind == "partition":
        ref = a0.copy()
        rs = oracle.partition(ref, job.pivot)
        assert job.split == rs
        gl, gr = oracle.sorted_sides(out, rs)
        rl, rr = oracle.sorted_sides(ref, rs)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr)
    else:
        ref = a0.copy()
        oracle.quicksort(ref)
        assert np.array_equal(out[:, 0], ref[:, 0])
        o = out[np.lexsort((out[:, 1], out[:, 0]))]
        r = ref[np.lexsort((ref[:, 1], ref[:, 0]))]
        assert np.array_equal(o, r)


def test_serving_results_and_alone_vs_mix(ss):
    from paper_2004_12532_amd.serving import make_jobs, latency_summary
    jobs = make_jobs(48, 0.0, 5, lo_log2=10.0, hi_log2=19.0)   # all available at once: one big mix
    srv = _server(ss)
    srv.run(jobs, realtime=False)
    assert srv.max_batch >= 20                                  # many jobs shared the launches
    for job in jobs:
        _check_job(job, srv.outputs[job.job_id])
    # the same jobs one at a time
    for job in jobs[::5]:
        from paper_2004_12532_amd.serving import Job
        solo = Job(job_id=job.job_id, kind=job.kind, n=job.n, seed=job.seed, arrival=0.0,
                   quantile=job.quantile, pivot=job.pivot)
        s2 = _server(ss, budget=1 << 30)
        s2.run([solo], realtime=False)
        assert np.array_equal(s2.outputs[job.job_id], srv.outputs[job.job_id]), job.job_id
        assert solo.split == job.split
    summ = latency_summary(jobs)
    assert summ["jobs"] == 48 and summ["p99_ms"] >= summ["p50_ms"]


def test_serving_realtime_arrivals_and_budget(ss):
    from paper_2004_12532_amd.serving import make_jobs
    jobs = make_jobs(30, 400.0, 9, lo_log2=12.0, hi_log2=20.0)
    srv = _server(ss, budget=64 << 20)   # 64 MiB: forces jobs to wait for memory
    srv.run(jobs, realtime=True)
    for job in jobs:
        assert job.done >= job.admitted >= job.arrival
        _check_job(job, srv.outputs[job.job_id])
    assert srv.arena.used == 0


def test_engine_direct_jobs_and_capacity_flag(ss):
    """The engine through its C ABI: partition splits against the oracle, trivial
    jobs done at once, and a full segment list reported by the status flags."""
    import torch
    import workloads
    n_jobs, L = 6, 5000
    data = workloads.records_kv(n_jobs * L, 4)
    t = torch.from_numpy(data.view(np.int64).copy()).cuda()
    eng = ss.ServerEngine(t, max_jobs=16, max_segments=4)
    pivots = [int(workloads.pivot_at_quantile_np(data[k * L:(k + 1) * L], q))
              for k, q in enumerate((0.1, 0.3, 0.5, 0.7, 0.9, 0.5))]
    for k in range(4):
        eng.submit(k, k * L, L, 0, pivots[k])
    eng.submit(10, 0, 0, 0, 0)          # empty partition: done at once
    eng.submit(11, 0, 1, 1, 0)          # one-record sort: done at once
    eng.tick(L)
    assert eng.wait(0) == 0
    assert eng.done(10)[0] and eng.done(11)[0]
    out = t.cpu().numpy().view(np.uint64)
    for k in range(4):
        fin, split = eng.done(k)
        assert fin
        ref = data[k * L:(k + 1) * L].copy()
        assert split == oracle.partition(ref, pivots[k])
        gl, gr = oracle.sorted_sides(out[k * L:(k + 1) * L], split)
        rl, rr = oracle.sorted_sides(ref, split)
        assert np.array_equal(gl, rl) and np.array_equal(gr, rr)
    assert eng.status() == 0
    # five segments into a list of four: the fifth is refused and flagged, the others finish
    for k in range(5):
        eng.submit(k, (k % n_jobs) * L, L, 0, pivots[k % n_jobs])
    eng.tick(L)
    assert eng.wait(0) & 1            # the mirrored flags show the overflow without a status call
    assert eng.status() & 1
    assert sum(eng.done(k)[0] for k in range(5)) == 4
    eng.close()


def test_serving_rejects_oversized_and_cancels(ss):
    """A job that can never fit the budget is rejected at arrival; withdrawn jobs
    (waiting, or already on the device) end as cancelled without a result; the
    rest are served correctly and every resource is returned."""
    from paper_2004_12532_amd.serving import Job, make_jobs, latency_summary
    jobs = make_jobs(12, 0.0, 31, lo_log2=12.0, hi_log2=17.0)
    srv = _server(ss, budget=256 << 20)
    big = Job(job_id=100, kind="partition", n=srv.capacity + 1, seed=7, arrival=0.0, pivot=1 << 63)
    jobs[3].cancel_at = 0.0                     # withdrawn before it can be admitted
    # a long sort withdrawn shortly after its admission: its ticks run, its result is dropped
    late = Job(job_id=101, kind="sort", n=1 << 21, seed=8, arrival=0.0, cancel_at=5e-4)
    srv.run(jobs + [big, late], realtime=False)
    assert big.status == "rejected"
    assert jobs[3].status == "cancelled" and jobs[3].admitted < 0 and jobs[3].job_id not in srv.outputs
    assert late.status == "cancelled" and late.admitted >= 0 and late.job_id not in srv.outputs
    for job in jobs:
        if job.status == "done":
            _check_job(job, srv.outputs[job.job_id])
    assert sum(j.status == "done" for j in jobs) == 11
    assert srv.arena.used == 0 and srv.aux_used == 0 and len(srv.free_slots) == 4096
    assert latency_summary(jobs + [big, late])["jobs"] == 11


def _check_job_by_payload(job, out):
    """Exact check for large jobs without sorting records: the payload of a record
    is its input position, so the output must be a permutation of the input
    records (each payload once, each key still with its payload), with the
    oracle's split and sides for a partition job and the oracle's key sequence
    for a sort job."""
    a0 = _input_of(job)
    idx = out[:, 1] - np.uint64(job.job_id << 32)
    assert bool(np.all(idx < np.uint64(job.n)))
    seen = np.zeros(job.n, dtype=bool)
    seen[idx.astype(np.int64)] = True
    assert bool(seen.all())
    assert np.array_equal(out[:, 0], a0[idx.astype(np.int64), 0])
    if job.kind == "partition":
        ref = a0.copy()
        rs = oracle.partition(ref, job.pivot)
        assert job.split == rs
        assert oracle.is_partitioned(out, job.pivot, rs)
    else:
        ref = a0.copy()
        oracle.quicksort(ref)
        assert np.array_equal(out[:, 0], ref[:, 0])


@pytest.mark.slow
def test_serving_large_jobs_default_budget(ss):
    """Jobs of 2^24 to 2^26 records (the upper end of the serving workload's length
    range) mixed with small ones under the default 64 GiB budget; one large sort
    job is also served alone and must give the same bytes."""
    from paper_2004_12532_amd.serving import Job, Server, make_jobs
    big = [("partition", 1 << 26, 0.5), ("sort", (1 << 25) + 3, 0.5), ("partition", (1 << 24) + 12345, 0.1),
           ("sort", (1 << 24) + 777, 0.5), ("partition", (1 << 25) + 1, 0.93)]
    jobs = [Job(job_id=200 + k, kind=kind, n=n, seed=(77 << 20) ^ k, arrival=0.0, quantile=q,
                pivot=min((1 << 64) - 1, int(q * (1 << 64)))) for k, (kind, n, q) in enumerate(big)]
    jobs += make_jobs(20, 0.0, 13, lo_log2=10.0, hi_log2=18.0)
    srv = Server(keep_outputs=True)           # default budget: 64 GiB
    srv.run(jobs, realtime=False)
    for job in jobs:
        assert job.status == "done"
        if job.n >= 1 << 20:
            _check_job_by_payload(job, srv.outputs[job.job_id])
        else:
            _check_job(job, srv.outputs[job.job_id])
    solo_src = jobs[3]
    solo = Job(job_id=solo_src.job_id, kind=solo_src.kind, n=solo_src.n, seed=solo_src.seed, arrival=0.0,
               quantile=solo_src.quantile, pivot=solo_src.pivot)
    mix_out = srv.outputs[solo_src.job_id]
    del srv
    import torch
    torch.cuda.empty_cache()
    s2 = Server(budget_bytes=4 << 30, keep_outputs=True)
    s2.run([solo], realtime=False)
    assert np.array_equal(s2.outputs[solo.job_id], mix_out)


@pytest.mark.parametrize("kind", ["u32", "u64"])
def test_engine_plain_key_sorts_and_partitions(ss, kind):
    """A plain-key engine (its leaves take the bucket sort, and leaves with a crowded
    bucket the separate radix kernel): sort jobs on uniform and on clustered keys with far
    outliers, and a partition job, each against the oracle."""
    import torch
    dt = np.uint32 if kind == "u32" else np.uint64
    top = int(np.iinfo(dt).max)
    rng = np.random.default_rng(21)
    uni = rng.integers(0, top, size=200000, dtype=dt, endpoint=True)
    clustered = (1000 + rng.integers(0, 64, size=100000)).astype(dt)
    clustered[rng.integers(0, clustered.size, size=50)] = top - rng.integers(0, 1000, size=50).astype(dt)
    part = rng.integers(0, top, size=50000, dtype=dt, endpoint=True)
    data = np.concatenate([uni, clustered, part])
    starts = [0, uni.size, uni.size + clustered.size]
    lens = [uni.size, clustered.size, part.size]
    pivot = int(np.sort(part)[part.size // 3])
    t = torch.from_numpy(data.view(np.int32 if kind == "u32" else np.int64).copy()).cuda()
    eng = ss.ServerEngine(t, max_jobs=8, max_segments=64)
    eng.submit(0, starts[0], lens[0], 1)
    eng.submit(1, starts[1], lens[1], 1)
    eng.submit(2, starts[2], lens[2], 0, pivot)
    for _ in range(400):
        eng.tick(max(lens))
        assert eng.wait(0) == 0
        if all(eng.done(k)[0] for k in range(3)):
            break
    assert all(eng.done(k)[0] for k in range(3))
    out = t.cpu().numpy().view(dt)
    for k in (0, 1):
        ref = data[starts[k]:starts[k] + lens[k]].copy()
        oracle.quicksort(ref)
        assert np.array_equal(out[starts[k]:starts[k] + lens[k]], ref)
    ref = part.copy()
    split = oracle.partition(ref, pivot)
    assert eng.done(2)[1] == split
    gl, gr = oracle.sorted_sides(out[starts[2]:starts[2] + lens[2]], split)
    rl, rr = oracle.sorted_sides(ref, split)
    assert np.array_equal(gl, rl) and np.array_equal(gr, rr)
    assert eng.status() == 0
    eng.close()
