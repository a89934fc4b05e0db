"""Pins of the oracle's LSH families against facts outside the oracle:
published MurmurHash3 vectors, exact rational arithmetic, the E2LSH collision
probability closed form (Datar et al. 2004) and MinHash's collision
probability = Jaccard (Eq. (2))."""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.lsh import fmix32, perm


def _golden_fmix(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "murmur3_fmix32.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            s, h = line.split()
            rows.append((int(s, 16), int(h, 16)))
    return rows


def test_fmix32_published_vectors(golden_dir):
    rows = _golden_fmix(golden_dir)
    assert len(rows) == 3
    got = fmix32(np.array([s for s, _ in rows], dtype=np.uint64))
    assert [int(g) for g in got] == [h for _, h in rows]


def _unfmix32(y):
    """Inverse of the finalizer, built from modular inverses of its odd
    multipliers and the inverse of xor-shift (independent of the forward)."""
    M = (1 << 32) - 1
    inv1 = pow(0x85EBCA6B, -1, 1 << 32)
    inv2 = pow(0xC2B2AE35, -1, 1 << 32)

    def unxorshift(v, s):
        r = v
        for _ in range(32 // s + 1):
            r = v ^ (r >> s)
        return r & M

    y = unxorshift(int(y), 16)
    y = (y * inv2) & M
    y = unxorshift(y, 13)
    y = (y * inv1) & M
    return unxorshift(y, 16)


def test_perm_is_bijection():
    g = np.random.default_rng(11)
    xs = g.integers(0, 2**32, size=2000, dtype=np.uint64)
    for x in xs[:300]:
        assert _unfmix32(int(fmix32(np.uint64(x)))) == int(x)
    key = (0x12345678, 0x9ABCDEF0)
    a = key[0] | 1
    ainv = pow(a, -1, 1 << 32)
    p = perm(key, xs)
    back = [((int(v) - key[1]) * ainv) & 0xFFFFFFFF for v in p]
    assert [_unfmix32(v) for v in back[:300]] == [int(x) for x in xs[:300]]
    # no two of 2**20 consecutive ids collide
    ids = np.arange(1 << 20, dtype=np.uint64)
    assert np.unique(perm(key, ids)).size == ids.size


def _sets_csr(sets):
    off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int64)
    return off, np.concatenate([np.asarray(s, dtype=np.uint32) for s in sets])


@pytest.mark.parametrize("J", [0.1, 0.3, 0.5, 0.7, 0.9])
def test_minhash_collision_rate_is_jaccard(J):
    # |A u B| = 200, |A n B| = 200 J; collision frequency over F functions
    # must be within 4.5 binomial sigma of J (Eq. (2)).
    U, I = 200, int(round(200 * J))
    g = np.random.default_rng(int(J * 100))
    toks = g.choice(10**6, size=U, replace=False).astype(np.uint32)
    onlyA = (U - I) // 2
    A = np.concatenate([toks[:I], toks[I:I + onlyA]])
    B = np.concatenate([toks[:I], toks[I + onlyA:]])
    Jt = I / len(np.union1d(A, B))
    F = 20000
    keys = g.integers(0, 2**32, size=(F, 2), dtype=np.uint64).astype(np.uint32)
    off, tk = _sets_csr([A, B])
    sig = oracle.minhash_sets(off, tk, keys)
    rate = np.mean(sig[0] == sig[1])
    sd = math.sqrt(Jt * (1 - Jt) / F)
    assert abs(rate - Jt) < 4.5 * sd, (rate, Jt)


def test_minhash_special_cases():
    g = np.random.default_rng(3)
    keys = g.integers(0, 2**32, size=(64, 2), dtype=np.uint64).astype(np.uint32)
    A = np.array([5, 9, 1000, 77], dtype=np.uint32)
    B = A[::-1].copy()  # same set, other order
    C = np.array([6, 10, 1001], dtype=np.uint32)  # disjoint from A
    S = np.array([424242], dtype=np.uint32)
    off, tk = _sets_csr([A, B, C, S])
    sig = oracle.minhash_sets(off, tk, keys)
    assert np.array_equal(sig[0], sig[1])
    assert not np.any(sig[0] == sig[2])  # a bijection never maps two tokens alike
    assert np.array_equal(sig[3], [perm(k, np.uint32(424242)) for k in keys])
    # brute force minimum on one set
    for f in range(64):
        assert sig[0, f] == min(int(perm(keys[f], np.uint32(t))) for t in A)
    with pytest.raises(ValueError):
        oracle.minhash_sets(np.array([0, 0]), np.zeros(0, np.uint32), keys)


def _exact_codes(X, A, b, w):
    n, d = X.shape
    out = np.empty((n, A.shape[0]), dtype=np.int64)
    near = 0
    for i in range(n):
        for p in range(A.shape[0]):
            v = sum(Fraction(float(A[p, t])) * Fraction(float(X[i, t])) for t in range(d))
            q = (v + Fraction(float(b[p]))) / Fraction(float(np.float32(w)))
            out[i, p] = math.floor(q)
            frac = q - math.floor(q)
            near += min(frac, 1 - frac) < Fraction(1, 10**9)
    return out, near


@pytest.mark.parametrize("w", [4.0, 8.0, 3.0, 4.0 * math.sqrt(32)])
def test_e2lsh_codes_match_exact_arithmetic(w):
    g = np.random.default_rng(int(w * 1000))
    X = g.uniform(-10, 10, size=(40, 7)).astype(np.float32)
    A = g.standard_normal(size=(9, 7)).astype(np.float32)
    b = g.uniform(0, w, size=9).astype(np.float32)
    ex, near = _exact_codes(X, A, b, w)
    assert near == 0
    assert np.array_equal(oracle.e2lsh_codes(X, A, b, w), ex)


def test_e2lsh_floor_at_bucket_edges():
    A = np.array([[1.0, 0.0]], dtype=np.float32)
    b = np.array([0.0], dtype=np.float32)
    eps = 2.0 ** -20
    X = np.array([[8.0, 3.0], [8.0 - eps, 3.0], [-8.0, 1.0], [-8.0 + eps, 0.0],
                  [-8.0 - eps, 0.0], [0.0, 5.0], [-eps, 0.0]], dtype=np.float32)
    got = oracle.e2lsh_codes(X, A, b, 4.0)[:, 0]
    assert got.tolist() == [2, 1, -2, -2, -3, 0, -1]
    # offset b shifts by exactly b / w
    got = oracle.e2lsh_codes(X, A, np.array([2.0], np.float32), 4.0)[:, 0]
    assert got.tolist() == [2, 2, -2, -2, -2, 0, 0]
    # a huge width puts every point of a bounded set in bucket 0 when b = w/2
    Xr = np.random.default_rng(1).uniform(-5, 5, size=(100, 2)).astype(np.float32)
    got = oracle.e2lsh_codes(Xr, A, np.array([5e29], np.float32), 1e30)
    assert np.all(got == 0)


def _e2lsh_p(r, w):
    """Collision probability of floor((a.x+b)/w) for two points at distance r
    (Datar, Immorlica, Indyk, Mirrokni 2004, Section 3.2)."""
    c = w / r
    Phi = 0.5 * (1 + math.erf(-c / math.sqrt(2)))
    return 1 - 2 * Phi - 2 / (math.sqrt(2 * math.pi) * c) * (1 - math.exp(-c * c / 2))


@pytest.mark.parametrize("r,w", [(1.0, 4.0), (4.0, 4.0), (10.0, 4.0), (3.0, 8.0)])
def test_e2lsh_collision_rate_closed_form(r, w):
    g = np.random.default_rng(int(r * 10 + w))
    d = 16
    x = g.standard_normal(d)
    u = g.standard_normal(d)
    y = x + r * u / np.linalg.norm(u)
    X = np.stack([x, y]).astype(np.float32)
    rr = float(np.linalg.norm(X[0].astype(np.float64) - X[1].astype(np.float64)))
    P = 40000
    A = g.standard_normal(size=(P, d)).astype(np.float32)
    b = g.uniform(0, w, size=P).astype(np.float32)
    c = oracle.e2lsh_codes(X, A, b, w)
    rate = np.mean(c[0] == c[1])
    p = _e2lsh_p(rr, w)
    sd = math.sqrt(p * (1 - p) / P)
    assert abs(rate - p) < 4.5 * sd, (rate, p)


def test_code_range_rule():
    assert oracle.code_bits(8) == 16 and oracle.code_bits(10) == 12 and oracle.code_bits(3) == 32
    assert oracle.codes_in_range(np.array([[-2048, 2047]]), 10)
    assert not oracle.codes_in_range(np.array([[-2049, 0]]), 10)
    assert not oracle.codes_in_range(np.array([[2048]]), 10)
    assert oracle.codes_in_range(np.array([[-(2**31), 2**31 - 1]]), 2)


def test_hetero_tokens_fields():
    cat = np.array([[3, 0, 65535], [7, 1, 2]], dtype=np.int32)
    codes = np.array([[-32768, 0], [32767, -1]], dtype=np.int64)
    tok = oracle.hetero_tokens(cat, codes)
    assert tok.shape == (2, 5)
    for i in range(2):
        assert len(set(tok[i].tolist())) == 5
        for a in range(3):
            assert tok[i, a] >> 16 == a and tok[i, a] & 0xFFFF == cat[i, a]
        for p in range(2):
            t = int(tok[i, 3 + p])
            assert t >> 31 == 1 and (t >> 16) & 0x7FFF == p
            assert (t & 0xFFFF) - 32768 == codes[i, p]
    with pytest.raises(ValueError):
        oracle.hetero_tokens(cat, np.array([[32768, 0], [0, 0]]))
    with pytest.raises(ValueError):
        oracle.hetero_tokens(np.array([[65536]]), np.zeros((1, 1), np.int64))
