"""Further passes of the data assignment (paper Section 4.3, Clustering
Performance: where compactness matters more than speed, GEEK may run
several passes of the data assignment).

A further pass takes the clusters of the previous assignment as its seeds:
the central vector of every cluster is recomputed from its members
(Section 3.3, the centroid of a seed) and every object is assigned again
(Eq. (1)) -- one step of Lloyd's iteration.

Reading (the paper does not say what happens to a cluster that received no
object): such clusters are dropped; the others keep the order of their
previous index, so the new index of cluster j is the number of non-empty
clusters with a smaller index.
"""

from __future__ import annotations

import numpy as np

from .assign import assign_euclid, centroids


def regroup(assign, k):
    """Clusters of an assignment as a seeds CSR.  Cluster j holds the objects
    i with ``assign[i] == j`` in ascending i; clusters with no object are
    dropped.  Returns ``(offsets uint32 [k_out + 1], members uint32 [n],
    label_of int32 [k_out])`` where ``label_of[r]`` is the previous index of
    the r-th cluster.  A stable sort of the objects by their label is the
    grouping step."""
    a = np.asarray(assign, dtype=np.int64)
    if a.size and (a.min() < 0 or a.max() >= k):
        raise ValueError("label outside [0, k)")
    members = np.argsort(a, kind="stable")
    labels, starts = np.unique(a[members], return_index=True)
    offsets = np.append(starts, a.size).astype(np.uint32)
    return offsets, members.astype(np.uint32), labels.astype(np.int32)


def assignment_pass(X, assign, k):
    """One further pass: ``regroup``, the float64 centroids of the clusters,
    and the one-pass assignment to them.  Returns ``(offsets, members,
    label_of, C, assign2, dist2)``."""
    offsets, members, label_of = regroup(assign, k)
    C = centroids(X, offsets, members)
    a2, dist2 = assign_euclid(X, C)
    return offsets, members, label_of, C, a2, dist2
