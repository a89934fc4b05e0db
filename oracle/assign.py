"""Central vectors and the one-pass data assignment (paper Section 3.3).

* Centroid of a seed (homogeneous dense data): the mean of its members.
* Mode (sets, categorical attributes): per position the most frequent value.
* Assignment: ``ID_i = argmin_j Dist(x_i, c_j)`` (Eq. (1)) with the lowest
  index winning ties; for a similarity, Dist = 1 - Sim (Section 2.1).

Floating-point order is fixed and stated in each function so that a second
implementation can reproduce the values bit for bit.
"""

from __future__ import annotations

import numpy as np

SSE_BLOCK = 4096


def centroids(X, seed_offsets, seed_members):
    """Centroid of every seed in float64: ``c_j = (sum over members i of seed
    j, in ascending member order, of x_i) / |C_j|``; the sum is accumulated
    sequentially (one rounding per addition) and then divided once."""
    X = np.asarray(X, dtype=np.float32)
    offs = np.asarray(seed_offsets, dtype=np.int64)
    mem = np.asarray(seed_members, dtype=np.int64)
    k = len(offs) - 1
    d = X.shape[1]
    sizes = np.diff(offs)
    if k and sizes.min() <= 0:
        raise ValueError("empty seed")
    acc = np.zeros((k, d), dtype=np.float64)
    for r in range(int(sizes.max()) if k else 0):
        sel = np.flatnonzero(sizes > r)
        acc[sel] += X[mem[offs[sel] + r]].astype(np.float64)
    return acc / sizes[:, None].astype(np.float64)


def modes(V, seed_offsets, seed_members):
    """Mode of every seed, position by position: ``mode[j, f]`` is the most
    frequent value of ``V[i, f]`` over the members i of seed j, the smallest
    such value on ties.  ``V`` is an integer matrix [n, F]."""
    V = np.asarray(V)
    offs = np.asarray(seed_offsets, dtype=np.int64)
    mem = np.asarray(seed_members, dtype=np.int64)
    k = len(offs) - 1
    out = np.empty((k, V.shape[1]), dtype=V.dtype)
    for j in range(k):
        rows = V[mem[offs[j]:offs[j + 1]]]
        for f in range(V.shape[1]):
            vals, cnt = np.unique(rows[:, f], return_counts=True)
            out[j, f] = vals[np.argmax(cnt)]
    return out


def euclid_dist_rows(X, C):
    """Squared Euclidean distances D[i, j] = sum_t (x_it - c_jt)^2 for float32
    rows X and float64 centres C, in float64 with the order: for t = 0 .. d-1,
    ``delta = x_it - c_jt`` (x widened), ``acc <- acc + delta * delta``, each
    operation rounded (no fused multiply-add).  Returns float64 [n, k]."""
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    C = np.asarray(C, dtype=np.float64)
    acc = np.zeros((X64.shape[0], C.shape[0]), dtype=np.float64)
    for t in range(X64.shape[1]):
        delta = X64[:, t:t + 1] - C[None, :, t]
        acc += delta * delta
    return acc


def euclid_dist_pairs(X, C, idx, chunk=262144):
    """Squared Euclidean distance of every row to one given centre,
    ``D[i] = sum_t (x_it - c_{idx_i, t})^2``, in exactly the arithmetic of
    ``euclid_dist_rows`` (t ascending, ``delta = x_it - c_jt``, ``acc <- acc +
    delta * delta``, each operation rounded), so ``D[i] ==
    euclid_dist_rows(X, C)[i, idx[i]]`` bit for bit.  Returns float64 [n]."""
    X = np.asarray(X, dtype=np.float32)
    C = np.asarray(C, dtype=np.float64)
    idx = np.asarray(idx, dtype=np.int64)
    n = X.shape[0]
    out = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        Xc = np.ascontiguousarray(X[s:e].T).astype(np.float64)
        Cc = np.ascontiguousarray(C[idx[s:e]].T)
        acc = np.zeros(e - s, dtype=np.float64)
        for t in range(X.shape[1]):
            delta = Xc[t] - Cc[t]
            acc += delta * delta
        out[s:e] = acc
    return out


def hetero_dist_pairs(Xn, cat, Cn, Mc, idx, gamma=1.0):
    """The heterogeneous distance of every row to one given seed, in the
    arithmetic of ``assign_hetero``: ``euclid_dist_pairs`` of the numeric
    attributes plus ``gamma * mismatches`` (float64).  Returns float64 [n]."""
    idx = np.asarray(idx, dtype=np.int64)
    dn = euclid_dist_pairs(Xn, Cn, idx)
    mism = (np.asarray(cat) != np.asarray(Mc)[idx]).sum(axis=1).astype(np.float64)
    return dn + np.float64(gamma) * mism


def assign_euclid(X, C, chunk=2048):
    """One-pass assignment to the nearest centroid (Eq. (1)): returns
    ``(assign int32 [n], dist float64 [n])`` where dist is the squared
    distance of ``euclid_dist_rows`` to the chosen centre and ties go to the
    lowest index."""
    X = np.asarray(X, dtype=np.float32)
    n = X.shape[0]
    a = np.empty(n, dtype=np.int32)
    dist = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        D = euclid_dist_rows(X[s:e], C)
        j = np.argmin(D, axis=1)
        a[s:e] = j
        dist[s:e] = D[np.arange(e - s), j]
    return a, dist


def assign_sig(S, M, chunk=1024):
    """Assignment of signature rows S [n, F] to modes M [k, F] by similarity
    ``matches / F`` (the fraction of positions where the values agree):
    ``ID_i = argmax_j matches(i, j)``, lowest index on ties.  Returns
    ``(assign int32, dist float64 = 1 - matches / F)``."""
    S = np.asarray(S)
    M = np.asarray(M)
    n, F = S.shape
    a = np.empty(n, dtype=np.int32)
    dist = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        match = (S[s:e, None, :] == M[None, :, :]).sum(axis=2)
        j = np.argmax(match, axis=1)
        a[s:e] = j
        mm = match[np.arange(e - s), j].astype(np.float64)
        dist[s:e] = 1.0 - mm / np.float64(F)
    return a, dist


def assign_hetero(Xn, cat, Cn, Mc, gamma=1.0, chunk=1024):
    """Assignment of heterogeneous rows: ``D = D_num + gamma * mismatches``
    where D_num is ``euclid_dist_rows`` of the numeric attributes to the
    numeric centroid and mismatches counts categorical attributes that differ
    from the seed's mode; computed as ``D_num + (gamma * mismatches)`` in
    float64.  Returns ``(assign int32, dist float64)``."""
    cat = np.asarray(cat)
    Mc = np.asarray(Mc)
    n = cat.shape[0]
    g = np.float64(gamma)
    a = np.empty(n, dtype=np.int32)
    dist = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        Dn = euclid_dist_rows(Xn[s:e], Cn)
        mism = (cat[s:e, None, :] != Mc[None, :, :]).sum(axis=2).astype(np.float64)
        D = Dn + g * mism
        j = np.argmin(D, axis=1)
        a[s:e] = j
        dist[s:e] = D[np.arange(e - s), j]
    return a, dist


def sse(dist):
    """Total distance of Definition 1 over the chosen centres, summed in
    float64 in a fixed order: sequentially within consecutive blocks of 4096
    rows, then sequentially over the block sums."""
    dist = np.asarray(dist, dtype=np.float64)
    if dist.size == 0:
        return 0.0
    blocks = []
    for s in range(0, dist.size, SSE_BLOCK):
        blocks.append(np.cumsum(dist[s:s + SSE_BLOCK])[-1])
    return float(np.cumsum(np.asarray(blocks))[-1])


def radius(dist, assign, k, euclid=True):
    """Radius of every cluster (Evaluation Metrics): the largest distance of
    a member to its centre -- the square root of the largest squared distance
    for Euclidean data; 0 for a cluster with no member."""
    r = np.zeros(k, dtype=np.float64)
    np.maximum.at(r, np.asarray(assign, dtype=np.int64), np.asarray(dist, dtype=np.float64))
    return np.sqrt(r) if euclid else r
