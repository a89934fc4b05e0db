"""Generators for the five workloads (dense small, dense large, sparse sets,
heterogeneous rows, batched jobs) and for the method's random parameters.

Every stream is derived from ``numpy.random.SeedSequence([seed, stream, ...])``
so that the data, the projection parameters, the MinHash keys and the SILK keys
never share random numbers.  Large dense arrays can be drawn directly on a
torch device (the recipe is the same, the noise stream is torch's generator).
"""

from __future__ import annotations

import math

import numpy as np

STREAM_DATA = 0
STREAM_E2LSH = 1
STREAM_MINHASH = 2
STREAM_SILK = 3
STREAM_PERM = 4
STREAM_JOB = 5

# Workload sizes.  "dense_small" and "dense_large" are the two dense Euclidean
# configurations; "sets", "hetero" and "batched" the sparse, heterogeneous and
# many-job ones.  Sizes mirror the paper's datasets (Table 2): Sift10M-shaped
# dense data, URL-shaped sparse sets, GeoNames-like heterogeneous rows.
CONFIGS = {
    "dense_small": dict(n=20_000, d=32, clusters=50, lo=-10.0, hi=10.0, sigma=1.0,
                        sizes="equal", m=8, L=16, w=4.0, K_S=3, L_S=20, delta=10),
    "dense_large": dict(n=10_000_000, d=128, clusters=10_000, lo=-50.0, hi=50.0,
                        sigma=1.0, sizes="zipf", m=10, L=32, w=8.0, K_S=3, L_S=20,
                        delta=10),
    "sets": dict(n=5_000_000, vocab=1_000_000, clusters=2_000, K=4, L=64,
                 K_S=3, L_S=20, delta=10),
    "hetero": dict(n=2_000_000, d_num=20, n_cat=10, clusters=1_000, P_h=20, w=4.0,
                   K=4, L=32, K_S=3, L_S=20, delta=10),
    "batched": dict(jobs=256),
}


def rng(seed: int, *path: int) -> np.random.Generator:
    """A PCG64 generator for the stream ``(seed, *path)``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), *map(int, path)])))


def largest_remainder(total: int, weights) -> np.ndarray:
    """Integer counts proportional to ``weights`` summing exactly to ``total``
    (Hamilton's largest-remainder rounding, ties to the lower index)."""
    w = np.asarray(weights, dtype=np.float64)
    q = total * w / w.sum()
    base = np.floor(q).astype(np.int64)
    rem = int(total - base.sum())
    if rem > 0:
        frac = q - base
        order = np.lexsort((np.arange(len(w)), -frac))
        base[order[:rem]] += 1
    return base


def dense_mixture(n, d, clusters, lo, hi, sigma=1.0, sizes="equal", seed=0,
                  device=None, zipf_s=1.0):
    """Isotropic Gaussian mixture, rows shuffled so ids carry no cluster order.

    Returns ``(X, labels, centers)``.  ``X`` is float32 ``[n, d]`` row-major:
    a numpy array when ``device`` is None, else a torch tensor on ``device``
    (noise drawn by torch's generator there, so a 5 GB array never passes
    through host memory).  ``sizes`` is "equal" or "zipf" (cluster c of
    ``clusters`` gets a share proportional to 1/c**zipf_s).
    """
    g = rng(seed, STREAM_DATA)
    centers = g.uniform(lo, hi, size=(clusters, d)).astype(np.float32)
    if sizes == "equal":
        counts = largest_remainder(n, np.ones(clusters))
    elif sizes == "zipf":
        counts = largest_remainder(n, 1.0 / np.arange(1, clusters + 1, dtype=np.float64) ** zipf_s)
    else:
        raise ValueError(sizes)
    labels = np.repeat(np.arange(clusters, dtype=np.int64), counts)
    labels = labels[rng(seed, STREAM_PERM).permutation(n)]
    if device is None:
        noise = g.standard_normal(size=(n, d), dtype=np.float32)
        X = centers[labels] + np.float32(sigma) * noise
        return X.astype(np.float32, copy=False), labels, centers
    import torch

    tg = torch.Generator(device=device)
    tg.manual_seed(int(g.integers(0, 2**62)))
    lab_t = torch.from_numpy(labels).to(device)
    cen_t = torch.from_numpy(centers).to(device)
    X = torch.empty((n, d), dtype=torch.float32, device=device)
    step = 1 << 20
    for s in range(0, n, step):
        e = min(n, s + step)
        X[s:e] = cen_t[lab_t[s:e]] + sigma * torch.randn((e - s, d), generator=tg,
                                                        device=device, dtype=torch.float32)
    return X, labels, centers


def e2lsh_params(P, d, w, seed=0):
    """Projection vectors ``A`` float32 [P, d] with N(0,1) entries and offsets
    ``b`` float32 [P] uniform in [0, w) (Eq. (3) of the paper and the E2LSH
    form in the Remarks after Example 1)."""
    g = rng(seed, STREAM_E2LSH, P, d)
    A = g.standard_normal(size=(P, d)).astype(np.float32)
    b = g.uniform(0.0, w, size=P).astype(np.float32)
    wf = np.float32(w)
    b = np.minimum(b, np.nextafter(wf, np.float32(0)))
    return A, b


def key_words(count, seed=0, stream=STREAM_MINHASH):
    """``count`` pairs of uniform uint32 words [count, 2]: the random draws
    behind ``count`` MinHash permutations."""
    g = rng(seed, stream, count)
    return g.integers(0, 2**32, size=(count, 2), dtype=np.uint64).astype(np.uint32)


def planted_seeds(labels, clusters, per_seed=32):
    """Seed j = the first ``min(size_j, per_seed)`` ids (ascending) of planted
    cluster j, as a CSR pair ``(offsets uint32 [k+1], members uint32)``.
    Clusters with no members are dropped."""
    order = np.argsort(labels, kind="stable")
    lab_sorted = labels[order]
    starts = np.searchsorted(lab_sorted, np.arange(clusters))
    ends = np.searchsorted(lab_sorted, np.arange(clusters), side="right")
    mem, offs = [], [0]
    for c in range(clusters):
        ids = order[starts[c]:ends[c]]
        if len(ids) == 0:
            continue
        take = np.sort(ids)[:per_seed]
        mem.append(take)
        offs.append(offs[-1] + len(take))
    return np.asarray(offs, dtype=np.uint32), np.concatenate(mem).astype(np.uint32)


def _zipf_sampler(vocab, s):
    r = np.arange(1, vocab + 1, dtype=np.float64)
    cdf = np.cumsum(r ** (-s))
    cdf /= cdf[-1]
    return cdf


def _first_distinct(rows, toks, quota, nrows):
    """Flat candidates ``(rows, toks)`` in row-major order of appearance:
    per row keep the first ``quota[row]`` distinct tokens in order of first
    appearance; returns the kept flat indices in the same order."""
    key = (rows.astype(np.int64) << 32) | toks.astype(np.int64)
    order = np.argsort(key, kind="stable")          # ties keep appearance order
    ks = key[order]
    first = np.ones(len(ks), dtype=bool)
    first[1:] = ks[1:] != ks[:-1]
    keep = np.sort(order[first])                     # back to appearance order
    kr = rows[keep]
    start = np.searchsorted(kr, np.arange(nrows))    # rows are sorted in ``keep``
    rank = np.arange(len(keep)) - start[kr]
    return keep[rank < quota[kr]]


def _first_distinct_t(rows, toks, quota, nrows):
    """``_first_distinct`` on torch tensors (same rule)."""
    import torch

    key = (rows.to(torch.int64) << 32) | toks.to(torch.int64)
    order = torch.argsort(key, stable=True)
    ks = key[order]
    first = torch.ones(len(ks), dtype=torch.bool, device=ks.device)
    first[1:] = ks[1:] != ks[:-1]
    keep = torch.sort(order[first]).values
    kr = rows[keep]
    start = torch.searchsorted(kr, torch.arange(nrows, device=kr.device))
    rank = torch.arange(len(keep), device=kr.device) - start[kr]
    return keep[rank < quota[kr]]


def _sparse_sets_device(n, labels, s_all, p_toks, p_off, cdf, share, chunk, device, seed):
    """The per-set draws of ``sparse_sets`` on a torch device (torch's
    generator supplies the uniforms; the recipe is the same)."""
    import torch

    tg = torch.Generator(device=device)
    tg.manual_seed(int(seed))
    cdf_t = torch.from_numpy(cdf).to(device)
    p_toks_t = torch.from_numpy(p_toks.astype(np.int64)).to(device)
    p_off_t = torch.from_numpy(p_off).to(device)
    labels_t = torch.from_numpy(labels).to(device)
    s_t = torch.from_numpy(s_all).to(device)
    vocab = len(cdf)

    def zipf(size):
        u = torch.rand(size, generator=tg, device=device, dtype=torch.float64)
        return torch.clamp(torch.searchsorted(cdf_t, u), max=vocab - 1)

    offsets = torch.zeros(n + 1, dtype=torch.int64, device=device)
    toks = []
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        m = c1 - c0
        lab = labels_t[c0:c1]
        s = s_t[c0:c1]
        plen = p_off_t[lab + 1] - p_off_t[lab]
        r = torch.minimum(torch.round(share * s.to(torch.float64)).to(torch.int64), plen)
        npick = torch.where(r > 0, 2 * r + 8, torch.zeros_like(r))
        ar = torch.arange(m, device=device)
        prow = torch.repeat_interleave(ar, npick)
        u = (torch.rand(len(prow), generator=tg, device=device, dtype=torch.float64) * plen[prow]).to(torch.int64)
        ptok = p_toks_t[p_off_t[lab[prow]] + u]
        pk = _first_distinct_t(prow, ptok, r, m)
        prow, ptok = prow[pk], ptok[pk]
        zrow = torch.repeat_interleave(ar, 3 * (s - r) + 16)
        ztok = zipf(len(zrow))
        allrow = torch.cat([prow, zrow])
        alltok = torch.cat([ptok, ztok])
        o = torch.argsort(allrow, stable=True)
        allrow, alltok = allrow[o], alltok[o]
        keep = _first_distinct_t(allrow, alltok, s, m)
        krow, ktok = allrow[keep], alltok[keep]
        o = torch.argsort((krow << 32) | ktok)
        toks.append(ktok[o].to(torch.int32))
        cnt = torch.bincount(krow, minlength=m)
        offsets[c0 + 1:c1 + 1] = offsets[c0] + torch.cumsum(cnt, 0)
    return offsets, torch.cat(toks)


def sparse_sets(n, vocab=1_000_000, clusters=2_000, seed=0, mu=4.5, sig=0.6,
                lo=5, hi=2000, zipf_s=1.1, share=0.6, chunk=50_000, device=None):
    """Sparse sets over ``[0, vocab)``: sizes lognormal(mu, sig) rounded and
    clipped to [lo, hi]; tokens Zipf(zipf_s) (token id = rank - 1); each set
    belongs to a uniformly drawn planted cluster and takes
    ``r = min(round(share*s), |prototype|)`` distinct tokens uniformly from
    the cluster's prototype (draws with replacement, repeats skipped), then
    fresh Zipf tokens, repeats skipped, until the size is reached.  Sets are
    drawn ``chunk`` at a time with vectorized de-duplication.

    Returns ``(offsets int64 [n+1], tokens uint32 [nnz], labels)`` with every
    set sorted ascending and free of repeats; with ``device`` the per-set
    draws run there and offsets / tokens (int32 bit patterns) are torch
    tensors on it.
    """
    g = rng(seed, STREAM_DATA, 3)
    cdf = _zipf_sampler(vocab, zipf_s)

    def zipf(size):
        return np.minimum(np.searchsorted(cdf, g.random(size)), vocab - 1).astype(np.uint32)

    def sizes(k):
        s = np.rint(np.exp(g.normal(mu, sig, size=k))).astype(np.int64)
        return np.clip(s, lo, hi)

    # prototypes: the first distinct Zipf draws
    proto_sizes = sizes(clusters)
    p_toks, p_off = [], [0]
    for c in range(clusters):
        want = int(proto_sizes[c])
        cand = zipf(want * 3 + 32)
        keep = _first_distinct(np.zeros(len(cand), np.int64), cand, np.array([want]), 1)
        row = np.sort(cand[keep])
        p_toks.append(row)
        p_off.append(p_off[-1] + len(row))
    p_toks = np.concatenate(p_toks).astype(np.uint32)
    p_off = np.asarray(p_off, dtype=np.int64)
    labels = g.integers(0, clusters, size=n)
    s_all = sizes(n)
    if device is not None:
        off_t, tok_t = _sparse_sets_device(n, labels, s_all, p_toks, p_off, cdf, share, chunk, device,
                                           g.integers(0, 2**62))
        return off_t, tok_t, labels
    offsets = np.zeros(n + 1, dtype=np.int64)
    toks = []
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        m = c1 - c0
        lab = labels[c0:c1]
        s = s_all[c0:c1]
        plen = p_off[lab + 1] - p_off[lab]
        r = np.minimum(np.rint(share * s).astype(np.int64), plen)
        # prototype part: 2r + 8 uniform draws (with replacement), first r distinct
        npick = np.where(r > 0, 2 * r + 8, 0)
        prow = np.repeat(np.arange(m), npick)
        u = (g.random(len(prow)) * plen[prow]).astype(np.int64)
        ptok = p_toks[p_off[lab[prow]] + u]
        pk = _first_distinct(prow, ptok, r, m)
        prow, ptok = prow[pk], ptok[pk]
        # fresh Zipf part: 3(s - r) + 16 draws; the whole row keeps its first s distinct
        nz = 3 * (s - r) + 16
        zrow = np.repeat(np.arange(m), nz)
        ztok = zipf(len(zrow))
        allrow = np.concatenate([prow, zrow])
        alltok = np.concatenate([ptok, ztok])
        o = np.argsort(allrow, kind="stable")        # row-major, prototype draws first
        allrow, alltok = allrow[o], alltok[o]
        keep = _first_distinct(allrow, alltok, s, m)
        krow, ktok = allrow[keep], alltok[keep]
        o = np.lexsort((ktok, krow))                   # sorted within each set
        toks.append(ktok[o].astype(np.uint32))
        cnt = np.bincount(krow, minlength=m)
        offsets[c0 + 1:c1 + 1] = offsets[c0] + np.cumsum(cnt)
    return offsets, np.concatenate(toks).astype(np.uint32), labels


def hetero_rows(n, d_num=20, n_cat=10, clusters=1_000, seed=0, lo=-10.0, hi=10.0,
                sigma=1.0, zipf_s=1.2):
    """Heterogeneous rows: ``d_num`` float32 numeric attributes from an
    equal-weight Gaussian mixture, and ``n_cat`` categorical attributes with
    cardinality round(10**U(1,3)) whose value is (z - 1 + off[a, c]) mod V_a,
    z ~ Zipf(zipf_s) truncated to V_a and off[a, c] a per-(attribute,
    cluster) offset.  Returns ``(X_num, cat int32 [n, n_cat], labels, card)``.
    """
    X, labels, _ = dense_mixture(n, d_num, clusters, lo, hi, sigma, "equal", seed)
    g = rng(seed, STREAM_DATA, 4)
    card = np.rint(10.0 ** g.uniform(1.0, 3.0, size=n_cat)).astype(np.int64)
    cat = np.zeros((n, n_cat), dtype=np.int32)
    for a in range(n_cat):
        V = int(card[a])
        cdf = _zipf_sampler(V, zipf_s)
        z = np.searchsorted(cdf, g.random(n)) + 1
        off = g.integers(0, V, size=clusters)
        cat[:, a] = ((z - 1 + off[labels]) % V).astype(np.int32)
    return X, cat, labels, card


def batched_jobs(jobs=256, seed=0, n_lo=3.0, n_hi=6.0, dims=(16, 32, 64, 128, 256),
                 k_hi=5000, n_scale=1.0):
    """Descriptors of ``jobs`` independent dense clustering problems:
    n log-uniform in [10**n_lo, 10**n_hi] (times ``n_scale``), d uniform over
    ``dims``, planted cluster count log-uniform in [10, k_hi].  The data of job
    j is ``dense_mixture(**spec, seed=spec['seed'])``."""
    g = rng(seed, STREAM_JOB)
    out = []
    for j in range(jobs):
        n_j = max(16, int(round(10.0 ** g.uniform(n_lo, n_hi) * n_scale)))
        d_j = int(g.choice(dims))
        c_j = int(round(10.0 ** g.uniform(1.0, math.log10(k_hi))))
        c_j = max(1, min(c_j, n_j))
        out.append(dict(n=n_j, d=d_j, clusters=c_j, lo=-10.0, hi=10.0, sigma=1.0,
                        sizes="equal", seed=int(seed) * 100_003 + j + 1))
    return out
