"""Pins of the oracle's densified one-permutation hashing (Algorithm 3's
first step; Shrivastava and Li, ICML 2014): hand-worked bin assignment and
rotation densification, a plain per-bin loop on small sets, the closed forms
of special sets (a singleton fills every coordinate with its one value; the
smallest coordinate is the set's MinHash under the same permutation;
disjoint sets never agree), and the collision rate of every coordinate =
Jaccard similarity within binomial error."""

import math

import numpy as np
import pytest

import oracle
from oracle.doph import EMPTY, densify_rotation, doph_bin, doph_sets
from oracle.lsh import perm

from .test_oracle_lsh import _unfmix32


def _csr(sets):
    off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int64)
    return off, np.concatenate([np.asarray(s, dtype=np.uint32) for s in sets])


def test_bin_boundaries_hand_worked():
    # 400 equal ranges of [0, 2^32): bin k starts at ceil(k * 2^32 / 400)
    D = 400
    starts = [-(-(k << 32) // D) for k in range(D)]
    v = np.array([0, (1 << 32) - 1] + starts[1:] + [s - 1 for s in starts[1:]], dtype=np.uint64)
    want = [0, D - 1] + list(range(1, D)) + list(range(0, D - 1))
    assert doph_bin(v, D).tolist() == want
    assert doph_bin(np.array([(1 << 31)], dtype=np.uint64), 2).tolist() == [1]
    assert doph_bin(np.array([(1 << 31) - 1], dtype=np.uint64), 2).tolist() == [0]


def test_rotation_densification_hand_worked():
    E = int(EMPTY)
    m = np.array([[E, 5, E, E, 9],     # bins 0, 2, 3 borrow from the right
                  [7, E, E, E, E],     # everything wraps round to bin 0
                  [E, E, E, E, 3],     # bins 0..3 borrow bin 4
                  [1, 2, 3, 4, 5]],    # nothing empty
                 dtype=np.uint64)
    want = [[5, 5, 9, 9, 9],
            [7, 7, 7, 7, 7],
            [3, 3, 3, 3, 3],
            [1, 2, 3, 4, 5]]
    assert densify_rotation(m).tolist() == want
    with pytest.raises(ValueError):
        densify_rotation(np.full((1, 3), EMPTY, dtype=np.uint64))


def test_hand_built_set():
    # identity-like key (a = 1, b = 0): pi = fmix32, so a token with permuted
    # value v is unfmix32(v); place values in bins 1 and 3 of D = 4
    key = np.array([1, 0], dtype=np.uint32)
    q = 1 << 30  # bin width of D = 4
    vals = [q + 17, q + 5, 3 * q + 2, 3 * q + 9]
    toks = [_unfmix32(v) for v in vals]
    assert [int(perm(key, np.uint32(t))) for t in toks] == vals
    off, tk = _csr([toks])
    sig = doph_sets(off, tk, key, 4)
    # bin 1 min q+5, bin 3 min 3q+2; bin 0 borrows bin 1, bin 2 borrows bin 3
    assert sig.tolist() == [[q + 5, q + 5, 3 * q + 2, 3 * q + 2]]


def _doph_loop(tokens, key, D):
    # plain per-bin loop: smallest permuted value per bin, then walk right
    mins = [None] * D
    for t in tokens:
        v = int(perm(key, np.uint32(t)))
        b = (v * D) >> 32
        if mins[b] is None or v < mins[b]:
            mins[b] = v
    out = []
    for j in range(D):
        k = j
        while mins[k % D] is None:
            k += 1
        out.append(mins[k % D])
    return out


@pytest.mark.parametrize("D", [1, 7, 64, 400])
def test_doph_equals_plain_loop(D):
    g = np.random.default_rng(D)
    sets = [g.choice(10**6, size=int(s), replace=False) for s in g.integers(1, 90, size=25)]
    sets.append(np.array([123456789]))
    key = g.integers(0, 2**32, size=2, dtype=np.uint64).astype(np.uint32)
    off, tk = _csr(sets)
    sig = doph_sets(off, tk, key, D)
    for i, s in enumerate(sets):
        assert sig[i].tolist() == _doph_loop(s, key, D)


def test_doph_special_sets():
    g = np.random.default_rng(5)
    key = g.integers(0, 2**32, size=2, dtype=np.uint64).astype(np.uint32)
    A = g.choice(10**6, size=150, replace=False).astype(np.uint32)
    B = A[::-1].copy()
    C = np.setdiff1d(g.choice(10**6, size=300, replace=False), A)[:120].astype(np.uint32)
    S = np.array([98765], dtype=np.uint32)
    off, tk = _csr([A, B, C, S])
    D = 400
    sig = doph_sets(off, tk, key, D)
    assert np.array_equal(sig[0], sig[1])                 # the set, not its order
    assert not np.any(sig[0] == sig[2])                   # disjoint sets never agree
    assert np.all(sig[3] == perm(key, np.uint32(98765)))  # a singleton everywhere
    mh = oracle.minhash_sets(off, tk, key[None, :])
    assert np.array_equal(sig.min(axis=1), mh[:, 0])      # smallest coordinate = MinHash
    with pytest.raises(ValueError):
        doph_sets(np.array([0, 2, 2]), np.array([1, 2], np.uint32), key, D)


@pytest.mark.parametrize("J", [0.1, 0.5, 0.8])
def test_doph_collision_rate_is_jaccard(J):
    # every coordinate collides with probability J (unbiased estimator); the
    # per-permutation mean over D coordinates, averaged over independent
    # permutations, must be within 4.5 standard errors of J
    U, I = 200, int(round(200 * J))
    g = np.random.default_rng(int(J * 1000))
    toks = g.choice(10**6, size=U, replace=False).astype(np.uint32)
    onlyA = (U - I) // 2
    A = np.concatenate([toks[:I], toks[I:I + onlyA]])
    B = np.concatenate([toks[:I], toks[I + onlyA:]])
    Jt = I / len(np.union1d(A, B))
    off, tk = _csr([A, B])
    D, R = 64, 1500
    keys = g.integers(0, 2**32, size=(R, 2), dtype=np.uint64).astype(np.uint32)
    rates = np.array([np.mean(np.equal(*doph_sets(off, tk, k, D))) for k in keys])
    se = rates.std(ddof=1) / math.sqrt(R)
    assert abs(rates.mean() - Jt) < 4.5 * se, (rates.mean(), Jt, se)
    # and the per-coordinate estimator is tighter than one MinHash value
    assert rates.std() < math.sqrt(Jt * (1 - Jt))
