"""Pins of the oracle's quantile bucketing (paper Algorithm 1): a hand-worked
case with a tie, the defining properties of an even partition of the
(value, id) order on random inputs, the extreme bucket counts, and the QALSH
values against exact integer arithmetic and an exact-rational error bound."""

from fractions import Fraction

import numpy as np
import pytest

import oracle


def test_hand_worked_with_tie():
    # values 3, 1, 2, 1, 5, 0 (ids 1 and 3 tie); t = 2 splits the six ranks 3 + 3
    X = np.array([[3], [1], [2], [1], [5], [0]], np.float32)
    A = np.array([[1], [-1]], np.float32)
    mem, off, bof = oracle.quantile_buckets(X, A, 2)
    assert off.tolist() == [[0, 3, 6], [0, 3, 6]]
    assert mem.tolist() == [[1, 3, 5, 0, 2, 4], [0, 2, 4, 1, 3, 5]]
    assert bof.tolist() == [[1, 0, 1, 0, 1, 0], [0, 1, 0, 1, 0, 1]]
    # the tie: with t = 3 ranks 0-1 | 2-3 | 4-5 put id 1 (rank 1) and id 3 (rank 2) apart
    mem, off, bof = oracle.quantile_buckets(X, A[:1], 3)
    assert mem[0].tolist() == [1, 5, 2, 3, 0, 4] and bof[0, 1] == 0 and bof[0, 3] == 1


@pytest.mark.parametrize("n,d,m,t,seed", [(50, 3, 2, 7, 0), (301, 8, 3, 16, 1), (1000, 16, 4, 999, 2)])
def test_even_partition_of_the_value_order(n, d, m, t, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, d)).astype(np.float32)
    X[::7] = X[3]                                  # exact ties between objects
    A = g.normal(size=(m, d)).astype(np.float32)
    V = oracle.qalsh_values(X, A)
    mem, off, bof = oracle.quantile_buckets(X, A, t)
    for p in range(m):
        sizes = np.diff(off[p].astype(np.int64))
        assert sizes.sum() == n and sizes.max() - sizes.min() <= 1
        # sizes of floor(r t / n) buckets: bucket b holds ranks ceil(b n / t) ..
        cdiv = lambda a, c: -(-a // c)
        assert sizes.tolist() == [cdiv((b + 1) * n, t) - cdiv(b * n, t) for b in range(t)]
        assert np.array_equal(np.sort(mem[p]), np.arange(n))
        for b in range(t):
            ids = mem[p, off[p, b]:off[p, b + 1]].astype(np.int64)
            assert (np.diff(ids) > 0).all() and (bof[p, ids] == b).all()
            if b + 1 < t:
                nxt = mem[p, off[p, b + 1]:off[p, b + 2]].astype(np.int64)
                top = max(zip(V[p, ids], ids))         # largest (value, id) of bucket b
                low = min(zip(V[p, nxt], nxt))         # smallest of bucket b + 1
                assert top < low


def test_extreme_bucket_counts():
    g = np.random.default_rng(3)
    X = g.normal(size=(40, 5)).astype(np.float32)
    A = g.normal(size=(2, 5)).astype(np.float32)
    mem, off, bof = oracle.quantile_buckets(X, A, 1)
    assert off.tolist() == [[0, 40]] * 2 and mem.tolist() == [list(range(40))] * 2
    V = oracle.qalsh_values(X, A)
    mem, off, bof = oracle.quantile_buckets(X, A, 40)
    for p in range(2):
        assert np.array_equal(mem[p], np.lexsort((np.arange(40), V[p])))
    with pytest.raises(ValueError):
        oracle.quantile_buckets(X, A, 41)
    with pytest.raises(ValueError):
        oracle.quantile_buckets(X, A, 0)


def test_qalsh_values_exact_cases():
    g = np.random.default_rng(4)
    Xi = g.integers(-1000, 1000, size=(200, 33))
    Ai = g.integers(-1000, 1000, size=(5, 33))
    V = oracle.qalsh_values(Xi.astype(np.float32), Ai.astype(np.float32))
    assert np.array_equal(V, (Ai @ Xi.T).astype(np.float64))    # integers: exact
    # general floats: within d roundings of the exact rational dot product
    X = g.normal(size=(20, 9)).astype(np.float32)
    A = g.normal(size=(3, 9)).astype(np.float32)
    V = oracle.qalsh_values(X, A)
    for p in range(3):
        for i in range(20):
            ex = sum(Fraction(float(A[p, t])) * Fraction(float(X[i, t])) for t in range(9))
            mag = sum(abs(Fraction(float(A[p, t])) * Fraction(float(X[i, t]))) for t in range(9))
            assert abs(Fraction(V[p, i]) - ex) <= mag * Fraction(9, 2 ** 53)
