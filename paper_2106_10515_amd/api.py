"""Torch-facing wrappers of the four GEEK calls.

They allocate output tensors and a per-device workspace with torch, pass raw
device pointers and torch's current HIP stream to libgeek.so, and return the
outputs.  No arithmetic of the method happens here.  Unsigned outputs are
returned in int32/int64 tensors holding the same bits (view them as uint32
on the host).
"""

from __future__ import annotations

import torch

from . import _lib as L
from ._lib import GeekError

_WS: dict = {}


def _dev(t: torch.Tensor) -> torch.device:
    if not t.is_cuda:
        raise GeekError(L.GEEK_ERR_ARG, "input must be a GPU tensor")
    return t.device


def workspace(nbytes: int, device) -> torch.Tensor:
    """A cached device buffer of at least ``nbytes`` (grown on demand), one
    per (device, current stream): calls enqueued on different streams may run
    at the same time and must not share scratch memory."""
    key = (str(device), torch.cuda.current_stream(device).cuda_stream)
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes:
        _WS.pop(key, None)
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf


def release_workspace():
    _WS.clear()


def stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def new_status(device) -> torch.Tensor:
    return torch.zeros(1, dtype=torch.int32, device=device)


def check_status(status: torch.Tensor, where: str = "device status") -> None:
    """Synchronizes with the stream and raises on a non-zero status word."""
    v = int(status.item())
    if v != 0:
        raise GeekError(v, where)


def _p(t):
    return None if t is None else t.data_ptr()


def _run(op, fn, jobs, device, status):
    nbytes = L.workspace_size(op, jobs)
    ws = workspace(nbytes, device)
    fn(jobs, ws.data_ptr(), ws.numel(), status.data_ptr(), stream_ptr(device))


# ---------------------------------------------------------------- geek_hash
def hash_dense(X, A, b, m, L_tables, w, want_codes=False, status=None, check=True,
               n_fixup=None, key_fp=None):
    """E2LSH codes of every row of X packed into per-table 128-bit keys.
    Returns ``(keys int32 [L, n, 4], codes int32 [n, m*L] or None)``.
    ``key_fp``: optional int32 [L, n] output, the keys' bucketize
    fingerprints (pass it to ``bucketize``)."""
    dev = _dev(X)
    n, d = X.shape
    assert X.dtype == torch.float32 and X.stride(1) == 1
    A = A.contiguous()
    b = b.contiguous()
    P = m * L_tables
    keys = torch.empty((L_tables, n, 4), dtype=torch.int32, device=dev)
    codes = torch.empty((n, P), dtype=torch.int32, device=dev) if want_codes else None
    status = new_status(dev) if status is None else status
    j = L.HashJob(kind=L.GEEK_HASH_DENSE, d=d, n=n, X=_p(X), ldx=X.stride(0), A=_p(A), b=_p(b),
                  m=m, L=L_tables, w=float(w), F=0, keys=_p(keys), codes=_p(codes),
                  n_fixup=_p(n_fixup), key_fp=_p(key_fp))
    _run(L.GEEK_OP_HASH, L.geek_hash, [j], dev, status)
    if check:
        check_status(status, "geek_hash")
    return keys, codes


def hash_dense_batch(problems, status=None, check=True):
    """One geek_hash call over many dense jobs, ``problems`` a list of
    ``(X, A, b, m, L_tables, w)``.  Returns the list of key tensors."""
    dev = _dev(problems[0][0])
    jobs, keys_out = [], []
    for X, A, b, m, L_tables, w in problems:
        n, d = X.shape
        keys = torch.empty((L_tables, n, 4), dtype=torch.int32, device=dev)
        keys_out.append((keys, A.contiguous(), b.contiguous()))
        jobs.append(L.HashJob(kind=L.GEEK_HASH_DENSE, d=d, n=n, X=_p(X), ldx=X.stride(0),
                              A=_p(keys_out[-1][1]), b=_p(keys_out[-1][2]), m=m, L=L_tables, w=float(w),
                              F=0, keys=_p(keys)))
    status = new_status(dev) if status is None else status
    _run(L.GEEK_OP_HASH, L.geek_hash, jobs, dev, status)
    if check:
        check_status(status, "geek_hash (batch)")
    return [k[0] for k in keys_out]


def hash_sets(offsets, tokens, mh_keys, status=None, check=True):
    """MinHash signatures of sets.  Returns ``sig int32 [n, F]``."""
    dev = _dev(tokens)
    n = offsets.numel() - 1
    F = mh_keys.shape[0]
    sig = torch.empty((n, F), dtype=torch.int32, device=dev)
    status = new_status(dev) if status is None else status
    j = L.HashJob(kind=L.GEEK_HASH_SETS, n=n, F=F, offsets=_p(offsets), tokens=_p(tokens),
                  mh_keys=_p(mh_keys), sig=_p(sig))
    _run(L.GEEK_OP_HASH, L.geek_hash, [j], dev, status)
    if check:
        check_status(status, "geek_hash")
    return sig


def hash_doph(offsets, tokens, key, D, status=None, check=True):
    """Densified one-permutation hashing of sets into D coordinates (one key
    pair ``key`` [1, 2] or [2]).  Returns ``sig int32 [n, D]``."""
    dev = _dev(tokens)
    n = offsets.numel() - 1
    key = key.reshape(-1).contiguous()
    sig = torch.empty((n, D), dtype=torch.int32, device=dev)
    status = new_status(dev) if status is None else status
    j = L.HashJob(kind=L.GEEK_HASH_DOPH, n=n, F=D, offsets=_p(offsets), tokens=_p(tokens),
                  mh_keys=_p(key), sig=_p(sig))
    _run(L.GEEK_OP_HASH, L.geek_hash, [j], dev, status)
    if check:
        check_status(status, "geek_hash (DOPH)")
    return sig


def hash_hetero(X, cat, A, b, m, L_tables, w, mh_keys, status=None, check=True):
    """MinHash signatures of heterogeneous rows (numeric attributes turned
    into E2LSH code tokens).  Returns ``sig int32 [n, F]``."""
    dev = _dev(X)
    n, d = X.shape
    F = mh_keys.shape[0]
    # contiguous copies held in locals until the call has been enqueued (a
    # temporary freed earlier could be handed out again as the workspace)
    A = A.contiguous()
    b = b.contiguous()
    cat = cat.contiguous()
    mh_keys = mh_keys.contiguous()
    sig = torch.empty((n, F), dtype=torch.int32, device=dev)
    status = new_status(dev) if status is None else status
    j = L.HashJob(kind=L.GEEK_HASH_HETERO, d=d, n=n, X=_p(X), ldx=X.stride(0), A=_p(A),
                  b=_p(b), m=m, L=L_tables, w=float(w), F=F, cat=_p(cat),
                  n_cat=cat.shape[1], mh_keys=_p(mh_keys), sig=_p(sig))
    _run(L.GEEK_OP_HASH, L.geek_hash, [j], dev, status)
    if check:
        check_status(status, "geek_hash")
    return sig


# ---------------------------------------------------------------- geek_bucketize
def bucketize(keys, n, T, key_words, table_stride, row_stride, want_bucket_of=True,
              status=None, check=True, key_fp=None):
    """Buckets of T tables.  ``keys`` is any int32 device tensor holding the
    key words at the given strides (in words); ``key_fp`` optionally the
    [T, n] fingerprints ``hash_dense`` wrote for them.  Returns ``(members
    [T, n], offsets [T, n+1], nbuckets [T], bucket_of [T, n] or None)``."""
    dev = _dev(keys)
    members = torch.empty((T, n), dtype=torch.int32, device=dev)
    offsets = torch.empty((T, n + 1), dtype=torch.int32, device=dev)
    nbuckets = torch.empty((T,), dtype=torch.int32, device=dev)
    bucket_of = torch.empty((T, n), dtype=torch.int32, device=dev) if want_bucket_of else None
    status = new_status(dev) if status is None else status
    j = L.BucketizeJob(n=n, T=T, key_words=key_words, keys=_p(keys), table_stride=table_stride,
                       row_stride=row_stride, members=_p(members), offsets=_p(offsets),
                       nbuckets=_p(nbuckets), bucket_of=_p(bucket_of), key_fp=_p(key_fp))
    _run(L.GEEK_OP_BUCKETIZE, L.geek_bucketize, [j], dev, status)
    if check:
        check_status(status, "geek_bucketize")
    return members, offsets, nbuckets, bucket_of


def bucketize_batch(problems, want_bucket_of=True, status=None, check=True):
    """One geek_bucketize call over many jobs, ``problems`` a list of
    ``(keys, n, T, key_words, table_stride, row_stride)``."""
    dev = _dev(problems[0][0])
    jobs, outs = [], []
    for keys, n, T, kw, ts, rs in problems:
        o = (torch.empty((T, n), dtype=torch.int32, device=dev),
             torch.empty((T, n + 1), dtype=torch.int32, device=dev),
             torch.empty((T,), dtype=torch.int32, device=dev),
             torch.empty((T, n), dtype=torch.int32, device=dev) if want_bucket_of else None)
        outs.append(o)
        jobs.append(L.BucketizeJob(n=n, T=T, key_words=kw, keys=_p(keys), table_stride=ts, row_stride=rs,
                                   members=_p(o[0]), offsets=_p(o[1]), nbuckets=_p(o[2]),
                                   bucket_of=_p(o[3])))
    status = new_status(dev) if status is None else status
    _run(L.GEEK_OP_BUCKETIZE, L.geek_bucketize, jobs, dev, status)
    if check:
        check_status(status, "geek_bucketize (batch)")
    return outs


# ---------------------------------------------------------------- geek_silk_seeds
def silk_seeds_async(members, offsets, nbuckets, n, T, K, L_silk, delta, silk_keys, cap_k, cap_members,
                     status, cap_c=0):
    """One geek_silk_seeds call with the given capacities; nothing is read
    back to the host, so it may be recorded in a HIP graph.  Returns the
    untrimmed device outputs ``dict(seed_offsets [cap_k+1], seed_members
    [cap_members], k_out [1], needed [3], counters [4])``."""
    dev = _dev(members)
    out = dict(seed_offsets=torch.empty((cap_k + 1,), dtype=torch.int32, device=dev),
               seed_members=torch.empty((cap_members,), dtype=torch.int32, device=dev),
               k_out=torch.empty((1,), dtype=torch.int32, device=dev),
               needed=torch.empty((3,), dtype=torch.int64, device=dev),
               counters=torch.empty((4,), dtype=torch.int64, device=dev))
    j = L.SilkJob(n=n, T=T, K=K, members=_p(members), offsets=_p(offsets), nbuckets=_p(nbuckets),
                  L=L_silk, delta=delta, silk_keys=_p(silk_keys), cap_k=cap_k,
                  cap_members=cap_members, seed_offsets=_p(out["seed_offsets"]),
                  seed_members=_p(out["seed_members"]), k_out=_p(out["k_out"]), needed=_p(out["needed"]),
                  counters=_p(out["counters"]), cap_c=cap_c)
    _run(L.GEEK_OP_SILK, L.geek_silk_seeds, [j], dev, status)
    return out


def silk_seeds(members, offsets, nbuckets, n, T, K, L_silk, delta, silk_keys,
               cap_k=None, cap_members=None, cap_c=None, status=None, check=True):
    """SILK seeds.  Returns ``(seed_offsets [k+1], seed_members [N_C],
    counters [4])`` trimmed to the k seeds found (reads k back to the host;
    with the default capacities a call that reports too little room is
    repeated with the capacities it asked for)."""
    dev = _dev(members)
    auto = cap_k is None and cap_members is None and cap_c is None
    cap_k = cap_k or max(1024, n // 4)
    cap_members = cap_members or max(4096, 16 * n)
    cap_c = cap_c if cap_c is not None else max(16384, 24 * n)
    status = new_status(dev) if status is None else status
    for attempt in range(4):
        out = silk_seeds_async(members, offsets, nbuckets, n, T, K, L_silk, delta, silk_keys, cap_k,
                               cap_members, status, cap_c)
        # default capacities too small: the call reported what it needs (first
        # for the intermediate multiset, then for the seeds); call again
        if auto and attempt < 3 and int(status.item()) == L.GEEK_ERR_CAPACITY:
            nk, nm, nc = (int(v) for v in out["needed"].cpu().tolist())
            cap_k, cap_members, cap_c = max(cap_k, nk), max(cap_members, nm), max(cap_c, nc)
            status.zero_()
            continue
        break
    if check:
        check_status(status, "geek_silk_seeds")
    so, sm = out["seed_offsets"], out["seed_members"]
    k = int(out["k_out"].item())
    nm = int(so[k].item()) if k > 0 else 0
    return so[:k + 1], sm[:nm], out["counters"]


# ---------------------------------------------------------------- geek_assign
def assign_euclid(X, seed_offsets, seed_members, k, precision=L.GEEK_PREC_FP32,
                  want_dist=True, want_radius=True, status=None, check=True, k_dev=None):
    """Central vectors and one-pass Euclidean assignment.  Returns a dict with
    assign, centroids, dist, sse, radius and counters.  ``k_dev`` (optional,
    a one-element int32 device tensor such as silk_seeds_async's k_out):
    the seed count as the device knows it, k then being the capacity."""
    dev = _dev(X)
    n, d = X.shape
    out = dict(
        assign=torch.empty((n,), dtype=torch.int32, device=dev),
        centroids=torch.empty((k, d), dtype=torch.float64, device=dev),
        dist=torch.empty((n,), dtype=torch.float64, device=dev) if want_dist else None,
        sse=torch.empty((1,), dtype=torch.float64, device=dev),
        radius=torch.empty((k,), dtype=torch.float64, device=dev) if want_radius else None,
        counters=torch.zeros((4,), dtype=torch.int64, device=dev),
    )
    status = new_status(dev) if status is None else status
    j = L.AssignJob(metric=L.GEEK_METRIC_EUCLID, precision=precision, n=n, d=d, k=k, X=_p(X),
                    ldx=X.stride(0), n_members=seed_members.numel(),
                    seed_offsets=_p(seed_offsets), seed_members=_p(seed_members),
                    assign=_p(out["assign"]), centroids=_p(out["centroids"]), dist=_p(out["dist"]),
                    sse=_p(out["sse"]), radius=_p(out["radius"]), counters=_p(out["counters"]),
                    k_dev=_p(k_dev))
    _run(L.GEEK_OP_ASSIGN, L.geek_assign, [j], dev, status)
    if check:
        check_status(status, "geek_assign")
    return out


def quantile_buckets(X, A, t, want_bucket_of=True, status=None, check=True):
    """Algorithm 1's dense transformation (geek_quantile_buckets): for each
    row of A [m, d], the n rows of X ranked by a . x (ties by id) and split
    evenly into t buckets.  Returns ``(members, offsets, bucket_of)`` as
    int32 device tensors [m, n], [m, t + 1], [m, n] (bucket_of None unless
    wanted)."""
    dev = _dev(X)
    n, d = X.shape
    m = A.shape[0]
    A = A.contiguous()  # kept alive in this frame until the call is enqueued
    mem = torch.empty((m, n), dtype=torch.int32, device=dev)
    off = torch.empty((m, t + 1), dtype=torch.int32, device=dev)
    bof = torch.empty((m, n), dtype=torch.int32, device=dev) if want_bucket_of else None
    status = new_status(dev) if status is None else status
    j = L.QuantileJob(n=n, d=d, m=m, t=t, X=_p(X), ldx=X.stride(0), A=_p(A),
                      members=_p(mem), offsets=_p(off), bucket_of=_p(bof))
    _run(L.GEEK_OP_QUANTILE, L.geek_quantile_buckets, [j], dev, status)
    if check:
        check_status(status, "geek_quantile_buckets")
    return mem, off, bof


def regroup(assign, k, want_label_of=True, status=None, check=True):
    """The clusters of an assignment as a seeds CSR for a further pass
    (geek_regroup).  Returns ``(seed_offsets, seed_members, k_out, label_of)``
    as device tensors: offsets int32 [k + 1] (the first k_out + 1 entries are
    written), members int32 [n], k_out int32 [1] and label_of int32 [k]."""
    dev = _dev(assign)
    n = assign.numel()
    so = torch.empty((k + 1,), dtype=torch.int32, device=dev)
    sm = torch.empty((max(n, 1),), dtype=torch.int32, device=dev)
    k_out = torch.zeros((1,), dtype=torch.int32, device=dev)
    lab = torch.empty((k,), dtype=torch.int32, device=dev) if want_label_of else None
    status = new_status(dev) if status is None else status
    j = L.RegroupJob(n=n, k=k, assign=_p(assign), seed_offsets=_p(so), seed_members=_p(sm),
                     k_out=_p(k_out), label_of=_p(lab))
    _run(L.GEEK_OP_REGROUP, L.geek_regroup, [j], dev, status)
    if check:
        check_status(status, "geek_regroup")
    return so, sm[:n], k_out, lab


def assignment_pass(X, assign, k, precision=L.GEEK_PREC_BF16, want_dist=True, want_radius=True,
                    status=None, check=True):
    """A further assignment pass: the clusters of ``assign`` become the seeds
    (geek_regroup), their centroids are recomputed and every row is assigned
    again (geek_assign).  Reads the cluster count back to the host.  Returns
    the ``assign_euclid`` dict plus ``label_of`` (the previous index of each
    new cluster) and ``k``."""
    so, sm, k_out, lab = regroup(assign, k, status=status, check=check)
    k2 = int(k_out.item())
    out = assign_euclid(X, so[:k2 + 1], sm, k2, precision, want_dist=want_dist, want_radius=want_radius,
                        status=status, check=check)
    out["label_of"] = lab[:k2] if lab is not None else None
    out["k"] = k2
    return out


def assign_euclid_batch(problems, precision=L.GEEK_PREC_BF16, want_dist=True, want_radius=True,
                        status=None, check=True):
    """One geek_assign call over many Euclidean jobs.  ``problems`` is a list
    of ``(X, seed_offsets, seed_members, k)``.  Returns ``(outs, t_done)``:
    one output dict per job (as ``assign_euclid``) and an int64 tensor of the
    jobs' completion times in device wall-clock ticks since the call began
    (``wallclock_hz()`` ticks per second)."""
    dev = _dev(problems[0][0])
    outs, jobs = [], []
    t_done = torch.zeros((len(problems),), dtype=torch.int64, device=dev)
    for idx, (X, so, sm, k) in enumerate(problems):
        n, d = X.shape
        out = dict(
            assign=torch.empty((n,), dtype=torch.int32, device=dev),
            centroids=torch.empty((k, d), dtype=torch.float64, device=dev),
            dist=torch.empty((n,), dtype=torch.float64, device=dev) if want_dist else None,
            sse=torch.empty((1,), dtype=torch.float64, device=dev),
            radius=torch.empty((k,), dtype=torch.float64, device=dev) if want_radius else None,
            counters=torch.zeros((4,), dtype=torch.int64, device=dev),
        )
        outs.append(out)
        jobs.append(L.AssignJob(metric=L.GEEK_METRIC_EUCLID, precision=precision, n=n, d=d, k=k, X=_p(X),
                                ldx=X.stride(0), n_members=sm.numel(), seed_offsets=_p(so),
                                seed_members=_p(sm), assign=_p(out["assign"]),
                                centroids=_p(out["centroids"]), dist=_p(out["dist"]), sse=_p(out["sse"]),
                                radius=_p(out["radius"]), counters=_p(out["counters"]),
                                t_done=t_done.data_ptr() + 8 * idx))
    status = new_status(dev) if status is None else status
    _run(L.GEEK_OP_ASSIGN, L.geek_assign, jobs, dev, status)
    if check:
        check_status(status, "geek_assign (batch)")
    return outs, t_done


def wallclock_hz() -> int:
    """Ticks per second of the device clock behind ``t_done``."""
    return L.geek_wallclock_hz()


def assign_sig(sig, seed_offsets, seed_members, k, want_dist=True, status=None, check=True):
    """Modes of the seeds and assignment of signature rows by match count."""
    dev = _dev(sig)
    n, F = sig.shape
    out = dict(
        assign=torch.empty((n,), dtype=torch.int32, device=dev),
        modes=torch.empty((k, F), dtype=torch.int32, device=dev),
        dist=torch.empty((n,), dtype=torch.float64, device=dev) if want_dist else None,
        sse=torch.empty((1,), dtype=torch.float64, device=dev),
        radius=torch.empty((k,), dtype=torch.float64, device=dev),
        counters=torch.zeros((4,), dtype=torch.int64, device=dev),
    )
    status = new_status(dev) if status is None else status
    j = L.AssignJob(metric=L.GEEK_METRIC_SIG, n=n, k=k, sig=_p(sig), F=F,
                    n_members=seed_members.numel(),
                    seed_offsets=_p(seed_offsets), seed_members=_p(seed_members),
                    assign=_p(out["assign"]), modes=_p(out["modes"]), dist=_p(out["dist"]),
                    sse=_p(out["sse"]), radius=_p(out["radius"]), counters=_p(out["counters"]))
    _run(L.GEEK_OP_ASSIGN, L.geek_assign, [j], dev, status)
    if check:
        check_status(status, "geek_assign")
    return out


def assign_hetero(X, cat, seed_offsets, seed_members, k, gamma=1.0, precision=L.GEEK_PREC_FP8,
                  want_dist=True, status=None, check=True):
    """Heterogeneous rows: numeric centroid + categorical modes; distance =
    squared Euclidean over X + gamma * mismatching categorical attributes."""
    dev = _dev(X)
    n, d = X.shape
    n_cat = cat.shape[1]
    out = dict(
        assign=torch.empty((n,), dtype=torch.int32, device=dev),
        centroids=torch.empty((k, d), dtype=torch.float64, device=dev),
        modes=torch.empty((k, n_cat), dtype=torch.int32, device=dev),
        dist=torch.empty((n,), dtype=torch.float64, device=dev) if want_dist else None,
        sse=torch.empty((1,), dtype=torch.float64, device=dev),
        radius=torch.empty((k,), dtype=torch.float64, device=dev),
        counters=torch.zeros((4,), dtype=torch.int64, device=dev),
    )
    status = new_status(dev) if status is None else status
    j = L.AssignJob(metric=L.GEEK_METRIC_HETERO, precision=precision, n=n, d=d, k=k, X=_p(X),
                    ldx=X.stride(0), n_cat=n_cat, cat=_p(cat), gamma=float(gamma),
                    n_members=seed_members.numel(), seed_offsets=_p(seed_offsets),
                    seed_members=_p(seed_members), assign=_p(out["assign"]),
                    centroids=_p(out["centroids"]), modes=_p(out["modes"]), dist=_p(out["dist"]),
                    sse=_p(out["sse"]), radius=_p(out["radius"]), counters=_p(out["counters"]))
    _run(L.GEEK_OP_ASSIGN, L.geek_assign, [j], dev, status)
    if check:
        check_status(status, "geek_assign")
    return out
