"""Densified one-permutation hashing (DOPH) of sets -- the dimensionality
reduction that the sparse data transformation applies first (paper
Section 3.1, Algorithm 3, its first step; Section 3.3 represents sets by the
reduced dimensions; Section 4.1 reduces the URL sets to 400 dimensions).

Written from the published method (Shrivastava and Li, "Densifying One
Permutation Hashing via Rotation for Fast Near Neighbor Search", ICML 2014):

* One permutation pi of the token universe (here the keyed bijection of
  32-bit words of ``oracle.lsh.perm``) is applied to every token of a set.
* The permuted universe [0, 2**32) is split into D contiguous ranges of equal
  size (up to rounding): a permuted value v falls into bin
  ``floor(v * D / 2**32)``.
* Coordinate j of the signature is the smallest permuted value of the set in
  bin j (one-permutation hashing).
* Densification by rotation: an empty bin takes the value of the first
  non-empty bin to its right, going round cyclically.  The published rule
  adds t*C to a value borrowed from t bins away so that borrowed values never
  equal values of other distances; here values are kept as permuted values
  (not offsets inside their bin), and bins are disjoint ranges, so a value
  already names the bin it came from and the distance is implied.  Two
  signatures therefore agree at a coordinate exactly when the published
  rule's values agree.

The collision probability of every coordinate equals the Jaccard similarity
of the two sets (the estimator of that paper is unbiased).  An empty set has
no value: ValueError.
"""

from __future__ import annotations

import numpy as np

from .lsh import perm

EMPTY = np.uint64(1 << 32)  # marks an empty bin (no 32-bit value equals it)


def doph_bin(v, D):
    """Bin of permuted values ``v`` (uint32) among D equal ranges of
    [0, 2**32): ``floor(v * D / 2**32)``, computed exactly in 64-bit
    integers."""
    return ((np.asarray(v, dtype=np.uint64) * np.uint64(D)) >> np.uint64(32)).astype(np.int64)


def densify_rotation(mins):
    """Rotation densification of one-permutation minima.  ``mins`` uint64
    [n, D] holds each bin's smallest permuted value or ``EMPTY``; every row
    must have a non-empty bin.  Returns uint32 [n, D] where an empty bin holds
    the value of the first non-empty bin to its right, cyclically."""
    mins = np.asarray(mins, dtype=np.uint64)
    n, D = mins.shape
    if n and np.any(np.all(mins == EMPTY, axis=1)):
        raise ValueError("empty set")
    # position of the first non-empty bin at or after j in the doubled row
    # [bins 0..D-1, bins 0..D-1], found as a suffix minimum of the indices of
    # non-empty bins
    big = np.int64(3 * D)
    idx = np.where(mins != EMPTY, np.arange(D, dtype=np.int64)[None, :], big)
    idx2 = np.concatenate([idx, np.where(idx < big, idx + D, big)], axis=1)
    nxt = np.minimum.accumulate(idx2[:, ::-1], axis=1)[:, ::-1][:, :D]
    src = nxt % D
    return np.take_along_axis(mins, src, axis=1).astype(np.uint32)


def doph_sets(offsets, tokens, key, D, chunk=4096):
    """DOPH signatures of sets: ``offsets`` int64 [n+1] and ``tokens`` uint32
    [nnz] (set i is ``tokens[offsets[i]:offsets[i+1]]``), ``key`` the two key
    words of the permutation, D the reduced dimension.  Returns uint32
    [n, D]."""
    offsets = np.asarray(offsets, dtype=np.int64)
    tokens = np.asarray(tokens, dtype=np.uint32)
    n = len(offsets) - 1
    if n > 0 and np.any(np.diff(offsets) <= 0):
        raise ValueError("empty set")
    out = np.empty((n, D), dtype=np.uint32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        lo, hi = offsets[s], offsets[e]
        v = perm(key, tokens[lo:hi]).astype(np.uint64)
        row = np.repeat(np.arange(e - s, dtype=np.int64), np.diff(offsets[s:e + 1]))
        mins = np.full((e - s) * D, EMPTY, dtype=np.uint64)
        np.minimum.at(mins, row * D + doph_bin(v, D), v)
        out[s:e] = densify_rotation(mins.reshape(e - s, D))
    return out
