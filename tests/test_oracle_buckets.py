"""Pins of the oracle's bucketing against brute force: two objects share a
bucket exactly when their table signatures are equal, every table partitions
the ids, and the output order is the canonical one."""

import numpy as np
import pytest

import oracle


def _check_canonical(members, offsets, bucket_of, n):
    assert offsets[0] == 0 and offsets[-1] == n
    assert np.all(np.diff(offsets.astype(np.int64)) > 0)
    assert np.array_equal(np.sort(members), np.arange(n))
    firsts = []
    for b in range(len(offsets) - 1):
        seg = members[offsets[b]:offsets[b + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)
        assert np.all(bucket_of[seg] == b)
        firsts.append(seg[0])
    assert np.all(np.diff(np.asarray(firsts, dtype=np.int64)) > 0)


@pytest.mark.parametrize("n,m,vals", [(150, 3, 2), (300, 2, 4), (64, 1, 5), (100, 4, 1)])
def test_bucketize_brute_force(n, m, vals):
    g = np.random.default_rng(n + m)
    T = g.integers(-vals, vals + 1, size=(n, m))
    members, offsets, bucket_of = oracle.bucketize(T)
    _check_canonical(members, offsets, bucket_of, n)
    for i in range(n):
        for j in range(n):
            assert (bucket_of[i] == bucket_of[j]) == bool(np.all(T[i] == T[j]))


def test_bucketize_edges():
    m, o, b = oracle.bucketize(np.zeros((1, 3), np.int64))
    assert m.tolist() == [0] and o.tolist() == [0, 1] and b.tolist() == [0]
    m, o, b = oracle.bucketize(np.arange(10).reshape(10, 1)[::-1])
    assert o.tolist() == list(range(11)) and m.tolist() == list(range(10))
    m, o, b = oracle.bucketize(np.full((7, 2), 5))
    assert o.tolist() == [0, 7] and b.tolist() == [0] * 7
    m, o, b = oracle.bucketize(np.zeros((0, 2), np.int64))
    assert o.tolist() == [0] and m.size == 0


def test_bucketize_tables_columns():
    g = np.random.default_rng(5)
    sig = g.integers(0, 3, size=(80, 6))
    tabs = oracle.bucketize_tables(sig, 2, 3)
    for l, (mm, oo, bo) in enumerate(tabs):
        ref = oracle.bucketize(sig[:, 2 * l:2 * l + 2])
        assert all(np.array_equal(x, y) for x, y in zip((mm, oo, bo), ref))
