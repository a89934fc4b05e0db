"""LSH families of the data transformation (paper Section 2.2 and 3.1).

* E2LSH code ``floor((a.x + b) / w)`` -- the form the Remarks after Example 1
  name, with ``a`` drawn as in Eq. (3) (entries N(0,1)).
* MinHash ``h_pi(A) = min_{a in A} pi(a)`` (Eq. (2)) with ``pi`` a keyed
  bijection of 32-bit words.
* Heterogeneous rows (Algorithm 2): numeric attributes are discretised by
  E2LSH codes into categorical attributes, then every row is a set of
  (attribute, value) tokens hashed by MinHash.
"""

from __future__ import annotations

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)


def fmix32(x):
    """MurmurHash3's 32-bit finalizer (Appleby, public domain): xor-shift 16,
    multiply by 0x85EBCA6B, xor-shift 13, multiply by 0xC2B2AE35, xor-shift 16,
    all modulo 2**32.  Each step is invertible, so this is a bijection."""
    x = np.asarray(x, dtype=np.uint64) & MASK32
    x = x ^ (x >> np.uint64(16))
    x = (x * np.uint64(0x85EBCA6B)) & MASK32
    x = x ^ (x >> np.uint64(13))
    x = (x * np.uint64(0xC2B2AE35)) & MASK32
    x = x ^ (x >> np.uint64(16))
    return x.astype(np.uint32)


def perm(key, x):
    """The random permutation pi of Eq. (2) for one pair of key words
    ``(k0, k1)``: ``pi(x) = (a * fmix32(x) + b) mod 2**32`` with ``a = k0 | 1``
    (odd, hence invertible modulo 2**32) and ``b = k1``.  A composition of
    bijections, so pi is a bijection of the 32-bit universe."""
    a = np.uint64(int(key[0]) | 1)
    b = np.uint64(int(key[1]))
    y = fmix32(x).astype(np.uint64)
    return ((a * y + b) & MASK32).astype(np.uint32)


def minhash_sets(offsets, tokens, keys, chunk=4096):
    """MinHash signatures of sets (Eq. (2), Algorithm 3).

    ``offsets`` int64 [n+1] and ``tokens`` uint32 [nnz] give set i as
    ``tokens[offsets[i]:offsets[i+1]]``; ``keys`` uint32 [F, 2] are the F
    permutations.  Returns ``sig`` uint32 [n, F] with
    ``sig[i, f] = min over tokens t of set i of pi_f(t)``.
    An empty set has no minimum: ValueError.
    """
    offsets = np.asarray(offsets, dtype=np.int64)
    tokens = np.asarray(tokens, dtype=np.uint32)
    keys = np.asarray(keys, dtype=np.uint32)
    n = len(offsets) - 1
    if n > 0 and np.any(np.diff(offsets) <= 0):
        raise ValueError("empty set")
    F = len(keys)
    sig = np.empty((n, F), dtype=np.uint32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        lo, hi = offsets[s], offsets[e]
        toks = tokens[lo:hi]
        starts = offsets[s:e] - lo
        for f in range(F):
            sig[s:e, f] = np.minimum.reduceat(perm(keys[f], toks), starts)
    return sig


def e2lsh_codes(X, A, b, w, chunk=8192):
    """E2LSH codes ``code[i, p] = floor((a_p . x_i + b_p) / w)``.

    Arithmetic (fixed so that a second implementation can reproduce it bit for
    bit): inputs are float32 values widened to float64; the dot product is
    accumulated over t = 0 .. d-1 in that order, ``s <- s + a_pt * x_it``
    (each product is exact in float64, so this equals a fused multiply-add);
    then ``v = s + b_p``, ``q = v / w`` (float64 division, w widened from
    float32) and ``code = floor(q)``.  Returns int64 [n, P].
    """
    X = np.asarray(X, dtype=np.float32)
    A64 = np.asarray(A, dtype=np.float32).astype(np.float64)
    b64 = np.asarray(b, dtype=np.float32).astype(np.float64)
    w64 = np.float64(np.float32(w))
    n, d = X.shape
    P = A64.shape[0]
    out = np.empty((n, P), dtype=np.int64)
    for s0 in range(0, n, chunk):
        e0 = min(n, s0 + chunk)
        X64 = X[s0:e0].astype(np.float64)
        acc = np.zeros((e0 - s0, P), dtype=np.float64)
        for t in range(d):
            acc += X64[:, t:t + 1] * A64[None, :, t]
        v = acc + b64[None, :]
        q = v / w64
        out[s0:e0] = np.floor(q).astype(np.int64)
    return out


def code_bits(m):
    """Bits available per code when the m codes of one table form a 128-bit
    bucket key: ``min(32, 128 // m)``."""
    return min(32, 128 // int(m))


def codes_in_range(codes, m):
    """True when every code fits a signed field of ``code_bits(m)`` bits
    (codes outside it cannot form an exact 128-bit key: a range error)."""
    B = code_bits(m)
    lo, hi = -(1 << (B - 1)), (1 << (B - 1)) - 1
    codes = np.asarray(codes)
    return bool(codes.size == 0 or (codes.min() >= lo and codes.max() <= hi))


def hetero_tokens(cat, codes):
    """Tokens of heterogeneous rows (Algorithm 2, first step): categorical
    attribute a with value v becomes token ``(a << 16) | v``; numeric
    projection p with E2LSH code c becomes ``0x80000000 | (p << 16) |
    (c + 32768)``.  Requires v, c + 32768 in [0, 65536) and a, p < 32768,
    else ValueError (a range error).  Returns uint32 [n, n_cat + P_h]; the
    tokens of one row are distinct by construction."""
    cat = np.asarray(cat, dtype=np.int64)
    codes = np.asarray(codes, dtype=np.int64)
    n, n_cat = cat.shape
    P = codes.shape[1]
    if n_cat >= 32768 or P >= 32768:
        raise ValueError("too many attributes")
    if cat.size and (cat.min() < 0 or cat.max() > 0xFFFF):
        raise ValueError("categorical value out of range")
    if codes.size and (codes.min() < -32768 or codes.max() > 32767):
        raise ValueError("numeric code out of range")
    a = np.arange(n_cat, dtype=np.int64)
    p = np.arange(P, dtype=np.int64)
    tc = (a[None, :] << 16) | cat
    tn = 0x80000000 | (p[None, :] << 16) | (codes + 32768)
    return np.concatenate([tc, tn], axis=1).astype(np.uint32)
