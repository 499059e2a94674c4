"""Host-side logic of the serving loop (no GPU): the arena allocator and the job mix."""
import numpy as np
import pytest


def _arena():
    # the package loads on a machine without a GPU; only the Server needs one
    import paper_2004_12532_amd.serving as m
    return m


def test_arena_first_fit_alignment_and_coalescing():
    m = _arena()
    a = m.Arena(1000, align=32)
    x = a.alloc(100)   # 128
    y = a.alloc(300)   # 320
    z = a.alloc(500)   # 512 -> 960 used
    assert x == (0, 128) and y == (128, 320) and z == (448, 512)
    assert a.alloc(64) is None        # only 40 left
    a.release(*y)
    assert a.alloc(320) == (128, 320)
    a.release(*x)
    a.release(128, 320)
    a.release(*z)
    assert a.free == [(0, 1000)] and a.used == 0


def test_arena_randomized_never_overlaps():
    m = _arena()
    rng = np.random.default_rng(1)
    a = m.Arena(1 << 20, align=32)
    live = []
    for step in range(3000):
        if live and rng.uniform() < 0.45:
            blk = live.pop(int(rng.integers(len(live))))
            a.release(*blk)
        else:
            got = a.alloc(int(rng.integers(1, 40000)))
            if got:
                live.append(got)
        iv = sorted(live)
        for (s0, l0), (s1, l1) in zip(iv, iv[1:]):
            assert s0 + l0 <= s1
        assert a.used == sum(l for _, l in live)
        assert a.used + sum(l for _, l in a.free) == 1 << 20


def test_job_mix_shape():
    m = _arena()
    jobs = m.make_jobs(4000, 100.0, 7)
    kinds = np.array([j.kind == "sort" for j in jobs])
    assert 0.26 < kinds.mean() < 0.34
    n = np.array([j.n for j in jobs])
    assert n.min() >= 1 << 10 and n.max() <= 1 << 26
    lg = np.log2(n)
    assert abs(lg.mean() - 18.0) < 0.3            # log-uniform over [10, 26]
    arr = np.array([j.arrival for j in jobs])
    assert np.all(np.diff(arr) >= 0)
    assert abs(len(jobs) / arr[-1] - 100.0) < 8.0  # Poisson rate


def test_never_fits_rule():
    m = _arena()
    assert not m.never_fits(100, 1000, capacity=100, aux_budget=1000)     # exactly at the limits
    assert m.never_fits(101, 10, capacity=100, aux_budget=1000)           # more records than the arena
    assert m.never_fits(10, 1001, capacity=100, aux_budget=1000)          # more auxiliary state than budgeted
    j = m.Job(job_id=1, kind="sort", n=5, seed=1, arrival=0.0)
    assert j.status == "pending" and j.cancel_at < 0
