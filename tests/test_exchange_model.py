"""Host model of the write-minimal exchange's pairing (CPU only).

The register engine's exchange form (Section 4's serial step, done by a whole
workgroup at once) decides every move from one number per slot: the count of
predecessors before it.  A successor at slot x below the group's predecessor
count c is the (x - rank)-th misplaced successor from the front; a
predecessor at slot x >= c is the (c - rank - 1)-th misplaced predecessor
from the back; equal indices swap.  This model applies those formulas to
plain arrays and must leave them exactly as the oracle's serial two-pointer
partition does, which swaps the same pairs.  It pins the index formulas, not
the kernel (the GPU tests compare the kernel with the oracle's step)."""
import itertools

import numpy as np

import oracle


def exchange_model(keys: np.ndarray, pivot: int):
    pred = keys < pivot
    c = int(pred.sum())
    rank = np.concatenate(([0], np.cumsum(pred)[:-1])).astype(np.int64)
    slot = np.arange(len(keys), dtype=np.int64)
    succ_mis = ~pred & (slot < c)
    pred_mis = pred & (slot >= c)
    m = int(succ_mis.sum())
    assert m == int(pred_mis.sum())
    k_succ = (slot - rank)[succ_mis]          # front rank among misplaced successors
    k_pred = (c - rank - 1)[pred_mis]         # back rank among misplaced predecessors
    assert sorted(k_succ.tolist()) == list(range(m)) and sorted(k_pred.tolist()) == list(range(m))
    succ_slot = np.empty(m, np.int64)
    succ_slot[k_succ] = slot[succ_mis]
    pred_slot = np.empty(m, np.int64)
    pred_slot[k_pred] = slot[pred_mis]
    out = keys.copy()
    out[succ_slot[k_pred]] = keys[pred_mis]   # each predecessor to its partner's slot
    out[pred_slot[k_succ]] = keys[succ_mis]   # and the partner to the predecessor's
    exchange_model.moved = succ_mis | pred_mis
    return out, c, m


def test_exchange_formulas_equal_serial_two_pointer_random():
    rng = np.random.default_rng(11)
    for n in (1, 2, 3, 16, 17, 100, 1000, 4097):
        for _ in range(4):
            keys = rng.integers(0, 1 << 20, size=n, dtype=np.uint64)
            for q in (0.0, 0.01, 0.3, 0.5, 0.97, 1.0):
                pivot = int(np.quantile(keys, q)) + (1 if q == 1.0 else 0)
                got, c, m = exchange_model(keys, pivot)
                ref = keys.copy()
                split = oracle.partition(ref, pivot)
                assert split == c
                assert np.array_equal(got, ref), (n, q)
                assert int((got != keys).sum()) <= 2 * m   # only the swapped pairs change


def test_exchange_formulas_exhaustive_small():
    for n in range(0, 7):
        for tup in itertools.product(range(4), repeat=n):
            keys = np.array(tup, dtype=np.uint64)
            for pivot in range(0, 5):
                got, c, _ = exchange_model(keys, pivot)
                ref = keys.copy()
                assert oracle.partition(ref, pivot) == c
                assert np.array_equal(got, ref), (tup, pivot)


def test_exchange_formulas_with_virtual_padding():
    """Virtual predecessors in front and virtual successors behind the real slots
    (a group touching a region's ends) are never misplaced, so never moved."""
    rng = np.random.default_rng(12)
    for front, back in ((0, 5), (7, 0), (13, 29)):
        real = rng.integers(1, 1000, size=300, dtype=np.uint64)
        keys = np.concatenate((np.zeros(front, np.uint64), real, np.full(back, 5000, np.uint64)))
        got, c, _ = exchange_model(keys, 500)
        moved = exchange_model.moved
        assert not moved[:front].any() and not moved[len(keys) - back:].any()
        ref = keys.copy()
        assert oracle.partition(ref, 500) == c and np.array_equal(got, ref)
