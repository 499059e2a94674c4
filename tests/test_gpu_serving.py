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
    eng.wait(0)
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
    eng.wait(0)
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
