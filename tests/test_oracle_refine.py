"""Pins of the oracle's further assignment pass (paper Section 4.3): the
invariants that determine a regrouping, a hand-worked pass, and Lloyd's
monotone total distance."""

import numpy as np
import pytest

import oracle
from workloads import dense_mixture


def _check_regroup(a, k):
    off, mem, lab = oracle.regroup(a, k)
    a = np.asarray(a, dtype=np.int64)
    n = a.size
    assert off.dtype == np.uint32 and mem.dtype == np.uint32 and lab.dtype == np.int32
    assert off[0] == 0 and off[-1] == n and len(off) == len(lab) + 1
    sizes = np.diff(off.astype(np.int64))
    assert (sizes > 0).all()                                   # no empty cluster
    assert np.array_equal(np.sort(mem), np.arange(n))          # a partition of [0, n)
    assert (np.diff(lab) > 0).all()                            # previous order kept
    assert set(lab.tolist()) == set(a.tolist())                # every used label, only those
    for r in range(len(lab)):
        m = mem[off[r]:off[r + 1]].astype(np.int64)
        assert (np.diff(m) > 0).all()                          # ascending members
        assert (a[m] == lab[r]).all()                          # cluster r = label lab[r]
        assert sizes[r] == np.count_nonzero(a == lab[r])
    return off, mem, lab


@pytest.mark.parametrize("n,k,used,seed", [(1, 1, 1, 0), (50, 7, 3, 1), (1000, 40, 40, 2), (999, 300, 120, 3)])
def test_regroup_invariants(n, k, used, seed):
    g = np.random.default_rng(seed)
    labels = g.choice(k, size=used, replace=False)
    _check_regroup(g.choice(labels, size=n), k)


def test_regroup_special_cases():
    off, mem, lab = oracle.regroup(np.zeros(0, np.int32), 5)
    assert off.tolist() == [0] and mem.size == 0 and lab.size == 0
    off, mem, lab = _check_regroup(np.full(9, 4), 5)
    assert off.tolist() == [0, 9] and lab.tolist() == [4] and mem.tolist() == list(range(9))
    with pytest.raises(ValueError):
        oracle.regroup(np.array([0, 3]), 3)
    with pytest.raises(ValueError):
        oracle.regroup(np.array([-1, 0]), 3)


def test_pass_hand_worked():
    # 1-D points 0, 1, 2 and 10, 11, 12; the previous assignment put 2 with the
    # far group: centroids 0.5 and 8.75 (exact in binary), so 2 moves back
    X = np.array([[0], [1], [2], [10], [11], [12]], np.float32)
    off, mem, lab, C, a2, d2 = oracle.assignment_pass(X, [0, 0, 1, 1, 1, 1], 2)
    assert off.tolist() == [0, 2, 6] and mem.tolist() == [0, 1, 2, 3, 4, 5]
    assert C[:, 0].tolist() == [0.5, 8.75]
    assert a2.tolist() == [0, 0, 0, 1, 1, 1]
    assert d2.tolist() == [0.25, 0.25, 2.25, 1.5625, 5.0625, 10.5625]
    # an unused label is dropped and the next index closes the gap
    off, mem, lab, C, a3, _ = oracle.assignment_pass(X, [2, 2, 2, 0, 0, 0], 3)
    assert lab.tolist() == [0, 2] and C[:, 0].tolist() == [11.0, 1.0] and a3.tolist() == [1, 1, 1, 0, 0, 0]


def test_passes_never_raise_the_total_distance():
    # Lloyd: the mean minimises the within-cluster sum and the argmin can only
    # lower it again, so sum_i D(x_i, centre of i) never grows from pass to pass
    X, lab, _ = dense_mixture(3000, 8, 12, -3, 3, 1.0, "equal", 5)
    g = np.random.default_rng(5)
    a = g.integers(0, 30, size=len(X)).astype(np.int32)
    k = 30
    prev = None
    for _ in range(4):
        off, mem, lab_of, C, a2, d2 = oracle.assignment_pass(X, a, k)
        total = oracle.sse(d2)
        # the centroid step alone: old clusters against their new means
        own = oracle.euclid_dist_rows(X, C)[np.arange(len(X)), np.searchsorted(lab_of, a)]
        assert total <= own.sum() * (1 + 1e-12)
        if prev is not None:
            assert own.sum() <= prev * (1 + 1e-12)
            assert total <= prev * (1 + 1e-12)
        prev, a, k = total, a2, len(lab_of)


def test_pass_fixed_point():
    X, lab, _ = dense_mixture(600, 4, 5, -50, 50, 1.0, "equal", 7)
    _, _, _, C1, a1, _ = oracle.assignment_pass(X, lab.astype(np.int32), 5)
    _, _, _, C2, a2, _ = oracle.assignment_pass(X, a1, 5)
    assert np.array_equal(a1, a2) and np.array_equal(C1, C2)
    assert np.array_equal(a1, lab)
