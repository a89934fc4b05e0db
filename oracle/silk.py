"""SILK: seeding from similar buckets (paper Section 3.2, Algorithm 4).

For each of L SILK tables: draw K MinHash functions over object ids, give each
bucket B the signature G(B) = (min pi_1(B), ..., min pi_K(B)), and put buckets
with identical G into one bin.  A bin holding at most one bucket is ignored.
Otherwise C_shared is the set of ids that appear in more than half of the
bin's buckets (majority voting) and it joins the multiset C when
``|C_shared| >= delta``.  Finally near-duplicates in C are removed by running
the procedure once more over C (the sets of C act as buckets, one table).

Readings where the paper is silent:
* "more than half" is strict: keep an id when 2 * count > |Bin|.
* De-duplication uses one extra table with its own K functions.  A bin there
  that holds a single set passes that set through unchanged -- the only
  reading that reproduces the four seeds of Example 2 -- and bins of several
  sets are majority-voted and delta-filtered.
* Seeds are ordered by the ascending lexicographic K-tuple of their
  de-duplication bin; members are ascending.
"""

from __future__ import annotations

import numpy as np

from .lsh import perm


def majority(sets):
    """Majority voting over a bin: the ids appearing in more than half of the
    given sets (2 * count > number of sets), ascending."""
    if len(sets) == 0:
        return np.zeros(0, dtype=np.uint32)
    ids, cnt = np.unique(np.concatenate([np.asarray(s, dtype=np.int64) for s in sets]),
                         return_counts=True)
    return ids[2 * cnt > len(sets)].astype(np.uint32)


def _vote_table(sets, bins, delta):
    """Algorithm 4's loop over the bins of one table."""
    out = []
    for b in bins:
        if len(b) <= 1:
            continue
        cs = majority([sets[j] for j in b])
        if len(cs) >= delta:
            out.append(cs)
    return out


def _dedup(C, bins, delta):
    """Near-duplicate removal over C, given the bins of the extra table."""
    seeds = []
    for b in bins:
        if len(b) == 1:
            seeds.append(np.asarray(C[b[0]], dtype=np.uint32))
            continue
        cs = majority([C[j] for j in b])
        if len(cs) >= delta:
            seeds.append(cs)
    return seeds


def silk_from_bins(bucket_sets, table_bins, dedup_bins_of, delta):
    """SILK with the bins given explicitly instead of hashed.

    ``bucket_sets``: list of id arrays (the buckets of B); ``table_bins``: for
    each SILK table, a list of bins (lists of bucket indices);
    ``dedup_bins_of``: a function mapping the multiset C (list of sets) to the
    bins of the de-duplication table.  Returns ``(C, seeds)``.
    """
    C = []
    for bins in table_bins:
        C.extend(_vote_table(bucket_sets, bins, delta))
    return C, _dedup(C, dedup_bins_of(C), delta)


def _signatures(offsets, members, keys, tally=None):
    """G(B) for every set of a CSR: column k = min over the set of pi_k.
    ``tally`` (a one-element list, optional) is increased by the number of
    pi evaluations made."""
    offsets = np.asarray(offsets, dtype=np.int64)
    members = np.asarray(members, dtype=np.uint32)
    K = len(keys)
    G = np.empty((len(offsets) - 1, K), dtype=np.uint32)
    for k in range(K):
        h = perm(keys[k], members)
        if tally is not None:
            tally[0] += int(h.size)
        G[:, k] = np.minimum.reduceat(h, offsets[:-1])
    return G


def _bins_of(G):
    """Group the rows of G (identical signature = same bin).  Returns bins as
    lists of row indices (ascending), ordered by the ascending lexicographic
    tuple, and that tuple for each bin."""
    if len(G) == 0:
        return [], G
    order = np.lexsort(tuple(G[:, k] for k in range(G.shape[1] - 1, -1, -1)))
    Gs = G[order]
    brk = np.ones(len(order), dtype=bool)
    brk[1:] = np.any(Gs[1:] != Gs[:-1], axis=1)
    starts = np.flatnonzero(brk)
    ends = np.concatenate([starts[1:], [len(order)]])
    bins = [sorted(order[s:e].tolist()) for s, e in zip(starts, ends)]
    return bins, Gs[starts]


def _vote_table_csr(offsets, members, G, delta):
    """Majority voting of one table for all bins at once (same result as
    ``_vote_table`` on the bins of G; written over arrays for speed)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    members = np.asarray(members, dtype=np.int64)
    nb = len(offsets) - 1
    _, bin_of = np.unique(G, axis=0, return_inverse=True)
    bin_of = bin_of.reshape(-1)
    bsize = np.bincount(bin_of)
    sizes = np.diff(offsets)
    owner = np.repeat(np.arange(nb), sizes)
    keep = bsize[bin_of[owner]] >= 2
    pairs_voted = int(keep.sum())
    pb = bin_of[owner[keep]].astype(np.int64)
    pid = members[keep]
    nid = int(members.max()) + 1 if members.size else 1
    key, cnt = np.unique(pb * nid + pid, return_counts=True)
    kb, kid = key // nid, key % nid
    sel = 2 * cnt > bsize[kb]
    kb, kid = kb[sel], kid[sel]
    out = []
    if kb.size:
        brk = np.flatnonzero(np.concatenate([[True], kb[1:] != kb[:-1]]))
        ends = np.concatenate([brk[1:], [kb.size]])
        for s, e in zip(brk, ends):
            if e - s >= delta:
                out.append(kid[s:e].astype(np.uint32))
    return out, pairs_voted


def silk_seeds(offsets, members, K, L, delta, keys):
    """SILK over the bucket collection B given as one CSR over all tables
    (``offsets`` [NB+1], ``members``).  ``keys`` uint32 [(L+1)*K, 2]: rows
    i*K .. i*K+K-1 draw the K functions of SILK table i, and rows L*K ..
    L*K+K-1 those of the de-duplication table.

    Returns ``(seed_offsets uint32 [k+1], seed_members uint32, info)``;
    ``info`` holds the multiset size |C| before de-duplication and the work
    counters as counted while computing: the pi evaluations of the SILK
    tables (``hash_evals``) and of the de-duplication table
    (``hash_evals_dedup``), and the voted (bin, id) pairs.  Section 3.5 bounds
    the work by the buckets alone (their number times their size times K
    and L), not by the number of clusters.
    """
    keys = np.asarray(keys, dtype=np.uint32)
    offsets = np.asarray(offsets, dtype=np.int64)
    members = np.asarray(members, dtype=np.uint32)
    C = []
    pairs = 0
    evals = [0]
    for i in range(L):
        G = _signatures(offsets, members, keys[i * K:(i + 1) * K], evals)
        got, pv = _vote_table_csr(offsets, members, G, delta)
        C.extend(got)
        pairs += pv
    info = dict(multiset=len(C), hash_evals=evals[0], pairs_voted=pairs)
    if not C:
        info["hash_evals_dedup"] = 0
        return np.zeros(1, np.uint32), np.zeros(0, np.uint32), info
    c_off = np.concatenate([[0], np.cumsum([len(c) for c in C])]).astype(np.int64)
    c_mem = np.concatenate(C).astype(np.uint32)
    dedup_evals = [0]
    Gc = _signatures(c_off, c_mem, keys[L * K:(L + 1) * K], dedup_evals)
    bins, _ = _bins_of(Gc)
    seeds = _dedup(C, bins, delta)
    info["hash_evals_dedup"] = dedup_evals[0]
    seen = {}
    dup = 0
    for s in seeds:
        t = s.tobytes()
        dup += t in seen
        seen[t] = 1
    info["dup_after_dedup"] = dup
    s_off = np.concatenate([[0], np.cumsum([len(s) for s in seeds])]).astype(np.uint32)
    s_mem = (np.concatenate(seeds) if seeds else np.zeros(0)).astype(np.uint32)
    return s_off, s_mem, info
