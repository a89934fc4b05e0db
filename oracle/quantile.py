"""Quantile bucketing of dense data (paper Algorithm 1, Homogeneous Dense
Data Transformation).

For each of m projection vectors a_p the table holds the QALSH value
h_p(x_i) = a_p . x_i of every object; the table is sorted in ascending order
of the values and the sorted ids are partitioned evenly into t buckets.

Readings (the algorithm leaves them open): equal values are ordered by id,
so the rank of object i is its position in the (value, id) order; "evenly"
puts rank r into bucket floor(r * t / n) (bucket sizes differ by at most
one), which needs 1 <= t <= n.  Within a bucket the members are listed in
ascending id.  The values are float32 inputs widened to float64 and summed
over the attributes in order, one rounding per addition (the products are
exact in float64), as for the E2LSH values.
"""

from __future__ import annotations

import numpy as np


def qalsh_values(X, A, chunk=8192):
    """``V[p, i] = a_p . x_i`` in float64: sum over t = 0 .. d-1 in that
    order of the exact products, one rounding per addition.  [m, n]."""
    X = np.asarray(X, dtype=np.float32)
    A64 = np.asarray(A, dtype=np.float32).astype(np.float64)
    n, d = X.shape
    V = np.empty((A64.shape[0], n), dtype=np.float64)
    for s0 in range(0, n, chunk):
        e0 = min(n, s0 + chunk)
        X64 = X[s0:e0].astype(np.float64)
        acc = np.zeros((A64.shape[0], e0 - s0), dtype=np.float64)
        for t in range(d):
            acc += A64[:, t:t + 1] * X64[None, :, t]
        V[:, s0:e0] = acc
    return V


def quantile_buckets(X, A, t):
    """Algorithm 1: ``(members uint32 [m, n], offsets uint32 [m, t + 1],
    bucket_of uint32 [m, n])``; table p's bucket b holds
    ``members[p, offsets[p, b]:offsets[p, b + 1]]``."""
    X = np.asarray(X, dtype=np.float32)
    n = X.shape[0]
    if not 1 <= t <= n:
        raise ValueError("need 1 <= t <= n")
    V = qalsh_values(X, A)
    m = V.shape[0]
    ids = np.arange(n)
    members = np.empty((m, n), dtype=np.uint32)
    offsets = np.empty((m, t + 1), dtype=np.uint32)
    bucket_of = np.empty((m, n), dtype=np.uint32)
    for p in range(m):
        order = np.lexsort((ids, V[p]))          # ascending value, then id
        rank = np.empty(n, dtype=np.int64)
        rank[order] = ids
        b = rank * t // n                        # even partition of the ranks
        bucket_of[p] = b
        members[p] = np.lexsort((ids, b))        # by bucket, ascending id inside
        offsets[p] = np.searchsorted(np.sort(b), np.arange(t + 1), side="left")
    return members, offsets, bucket_of
