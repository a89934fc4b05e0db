"""Pins of the oracle's central vectors and assignment against exact rational
arithmetic, brute force and special cases (Eq. (1), Section 3.3)."""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

U64 = 2.0 ** -53


def _gamma(k, u=U64):
    return k * u / (1 - k * u)


def test_centroids_exact_mean_and_bound():
    g = np.random.default_rng(0)
    X = g.integers(-50, 50, size=(40, 5)).astype(np.float32)
    offs = np.array([0, 4, 12, 13], dtype=np.uint32)
    mem = np.array([0, 3, 7, 9, 1, 2, 4, 5, 6, 8, 10, 11, 20], dtype=np.uint32)
    C = oracle.centroids(X, offs, mem)
    for j in range(3):
        rows = X[mem[offs[j]:offs[j + 1]]]
        assert np.array_equal(C[j], rows.astype(np.float64).mean(axis=0))  # sizes 4, 8, 1
    Y = g.uniform(-40, 40, size=(300, 6)).astype(np.float32)
    offs = np.array([0, 37, 300], dtype=np.uint32)
    mem = np.arange(300, dtype=np.uint32)
    C = oracle.centroids(Y, offs, mem)
    for j in range(2):
        rows = Y[mem[offs[j]:offs[j + 1]]]
        for t in range(6):
            ex = sum(Fraction(float(v)) for v in rows[:, t]) / len(rows)
            bound = _gamma(len(rows) + 1) * float(np.abs(rows[:, t]).astype(np.float64).mean())
            assert abs(C[j, t] - float(ex)) <= bound


def test_centroids_sequential_order_is_the_definition():
    # ascending member order, one rounding per addition: compare with a
    # plain python loop over floats
    X = np.array([[1e8], [1.0], [-1e8], [3.0]], dtype=np.float32)
    C = oracle.centroids(X, np.array([0, 4], np.uint32), np.arange(4, dtype=np.uint32))
    s = 0.0
    for v in X[:, 0]:
        s = s + float(v)
    assert C[0, 0] == s / 4


def _exact_d2(x, c):
    return sum((Fraction(float(a)) - Fraction(float(b))) ** 2 for a, b in zip(x, c))


def test_euclid_dist_error_bound_and_argmin():
    g = np.random.default_rng(2)
    X = g.uniform(-5, 5, size=(30, 9)).astype(np.float32)
    C = g.uniform(-5, 5, size=(7, 9))
    D = oracle.euclid_dist_rows(X, C)
    for i in range(30):
        ex = [_exact_d2(X[i], C[j]) for j in range(7)]
        for j in range(7):
            assert abs(D[i, j] - float(ex[j])) <= _gamma(11) * float(ex[j]) + 1e-300
        a, _ = oracle.assign_euclid(X[i:i + 1], C)
        assert a[0] == min(range(7), key=lambda j: (ex[j], j))


def test_assign_special_cases():
    g = np.random.default_rng(4)
    X = g.standard_normal((50, 4)).astype(np.float32)
    a, dist = oracle.assign_euclid(X, np.zeros((1, 4)))
    assert np.all(a == 0)
    # seeds that are data points map those points to themselves
    idx = [3, 17, 40]
    C = X[idx].astype(np.float64)
    a, dist = oracle.assign_euclid(X, C)
    assert a[idx].tolist() == [0, 1, 2] and np.all(dist[idx] == 0)
    # duplicated centroid: the lower index wins the exact tie
    C2 = np.concatenate([C, C[1:2]])
    a2, _ = oracle.assign_euclid(X, C2)
    assert np.array_equal(a2, a)
    C3 = np.concatenate([C[1:2], C])
    a3, _ = oracle.assign_euclid(X, C3)
    assert np.all(a3 != 2)


def test_sse_matches_exactly_rounded_sum():
    g = np.random.default_rng(6)
    dist = g.exponential(100.0, size=20000) * g.choice([1.0, 1e-6, 1e6], size=20000)
    s = oracle.sse(dist)
    exact = math.fsum(dist.tolist())
    assert abs(s - exact) <= _gamma(4096 + 10) * np.abs(dist).sum()
    small = np.array([1.0, 2.0 ** -60, -1.0 + 2 ** -52])
    assert oracle.sse(small) == ((1.0 + 2.0 ** -60) + (-1.0 + 2 ** -52))
    assert oracle.sse(np.zeros(0)) == 0.0


def test_modes_ties_smallest():
    V = np.array([[5, 1], [3, 1], [5, 2], [3, 2], [9, 2]], dtype=np.uint32)
    M = oracle.modes(V, np.array([0, 4, 5], np.uint32), np.array([0, 1, 2, 3, 4], np.uint32))
    assert M.tolist() == [[3, 1], [9, 2]]


def test_assign_sig_brute_force():
    g = np.random.default_rng(8)
    S = g.integers(0, 3, size=(40, 6)).astype(np.uint32)
    M = g.integers(0, 3, size=(5, 6)).astype(np.uint32)
    a, dist = oracle.assign_sig(S, M)
    for i in range(40):
        cnt = [sum(int(S[i, f] == M[j, f]) for f in range(6)) for j in range(5)]
        best = max(range(5), key=lambda j: (cnt[j], -j))
        assert a[i] == best
        assert dist[i] == 1.0 - cnt[best] / 6.0


def test_assign_hetero_brute_force():
    g = np.random.default_rng(9)
    Xn = g.uniform(-2, 2, size=(25, 3)).astype(np.float32)
    cat = g.integers(0, 2, size=(25, 4)).astype(np.int32)
    Cn = g.uniform(-2, 2, size=(6, 3))
    Mc = g.integers(0, 2, size=(6, 4)).astype(np.int32)
    for gamma in (1.0, 0.5, 0.0):
        a, dist = oracle.assign_hetero(Xn, cat, Cn, Mc, gamma)
        for i in range(25):
            ex = [_exact_d2(Xn[i], Cn[j]) + Fraction(gamma) * int(np.sum(cat[i] != Mc[j]))
                  for j in range(6)]
            j = min(range(6), key=lambda jj: (ex[jj], jj))
            srt = sorted(ex)
            if srt[1] - srt[0] > Fraction(1, 10**9):
                assert a[i] == j
            assert abs(dist[i] - float(ex[a[i]])) < 1e-9


def test_radius():
    dist = np.array([4.0, 9.0, 1.0, 0.0])
    a = np.array([0, 0, 2, 2])
    assert oracle.radius(dist, a, 4).tolist() == [3.0, 0.0, 1.0, 0.0]


def test_dist_pairs_equal_full_rows_and_exact_values():
    # the per-row distance to one given centre is the same number as the full
    # distance matrix's entry (same arithmetic), and within the dot-product
    # rounding bound of the exact rational value
    g = np.random.default_rng(12)
    X = g.uniform(-30, 30, size=(700, 13)).astype(np.float32)
    C = g.uniform(-30, 30, size=(9, 13))
    idx = g.integers(0, 9, size=700)
    D = oracle.euclid_dist_rows(X, C)
    got = oracle.euclid_dist_pairs(X, C, idx, chunk=128)
    assert np.array_equal(got, D[np.arange(700), idx])
    for i in range(0, 700, 97):
        ex = _exact_d2(X[i], C[idx[i]])
        assert abs(got[i] - float(ex)) <= _gamma(15) * float(ex) + 1e-300
    # a 3-4-5 triangle and a zero distance
    X2 = np.array([[3.0, 0.0], [1.5, -2.0]], dtype=np.float32)
    C2 = np.array([[0.0, 4.0], [1.5, -2.0]])
    assert oracle.euclid_dist_pairs(X2, C2, np.array([0, 1])).tolist() == [25.0, 0.0]
    cat = g.integers(0, 3, size=(700, 5)).astype(np.int32)
    Mc = g.integers(0, 3, size=(9, 5)).astype(np.int32)
    for gamma in (1.0, 0.25):
        h = oracle.hetero_dist_pairs(X, cat, C, Mc, idx, gamma)
        a, dist = oracle.assign_hetero(X, cat, C, Mc, gamma)
        assert np.array_equal(oracle.hetero_dist_pairs(X, cat, C, Mc, a, gamma), dist)
        mism = (cat != Mc[idx]).sum(axis=1)
        assert np.array_equal(h, D[np.arange(700), idx] + gamma * mism)
