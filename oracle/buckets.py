"""Buckets from hash tables (Algorithms 2 and 3: ``T[G(x_j)].push(j)``).

A bucket of a table is the set of object ids whose signature G -- the tuple of
that table's hash values -- is identical.  Output order is canonical so that
two implementations can be compared element by element: within a table,
buckets are ordered by their smallest member and members are ascending.
"""

from __future__ import annotations

import numpy as np


def bucketize(tuples):
    """Group the rows of ``tuples`` ([n, m] integers, the signature of every
    object in one table) by exact equality.

    Returns ``(members uint32 [n], offsets uint32 [nb+1], bucket_of uint32
    [n])``: bucket b holds ``members[offsets[b]:offsets[b+1]]``.
    """
    tuples = np.asarray(tuples)
    n = tuples.shape[0]
    if n == 0:
        return (np.zeros(0, np.uint32), np.zeros(1, np.uint32), np.zeros(0, np.uint32))
    _, group = np.unique(tuples.reshape(n, -1), axis=0, return_inverse=True)
    group = group.reshape(-1)
    ng = int(group.max()) + 1
    first = np.full(ng, n, dtype=np.int64)
    np.minimum.at(first, group, np.arange(n, dtype=np.int64))
    rank = np.empty(ng, dtype=np.int64)
    rank[np.argsort(first, kind="stable")] = np.arange(ng)
    bucket_of = rank[group]
    members = np.argsort(bucket_of, kind="stable")
    counts = np.bincount(bucket_of, minlength=ng)
    offsets = np.concatenate([[0], np.cumsum(counts)])
    return members.astype(np.uint32), offsets.astype(np.uint32), bucket_of.astype(np.uint32)


def bucketize_tables(sig, m, L):
    """Bucketize L tables whose signatures are consecutive column groups of
    ``sig`` ([n, m*L]): table l uses columns l*m .. l*m+m-1 (the m hash
    functions drawn for that table).  Returns a list of L triples."""
    sig = np.asarray(sig)
    return [bucketize(sig[:, l * m:(l + 1) * m]) for l in range(L)]
