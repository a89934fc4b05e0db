"""Parity at the full sizes of the sparse-set and heterogeneous workloads, in
the benchmark's launch configuration: 5e6 sets over a 1e6-token vocabulary
(MinHash K = 4 x L = 64, 2,000 planted clusters) and 2e6 heterogeneous rows
(20 numeric + 10 categorical attributes, 1,000 clusters).  Sampled rows are
checked against the FP64 oracle one by one; bucket CSRs through properties
that hold at any size; central vectors and modes of the planted seeds in
full."""

import numpy as np
import pytest
import torch

import oracle
from workloads import CONFIGS, e2lsh_params, hetero_rows, key_words, planted_seeds, sparse_sets
from workloads.gen import STREAM_MINHASH

from .gpu_util import announce, gpu_api, host_u32

pytestmark = pytest.mark.gpu


def _rows(n, seed):
    g = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, n - 1], g.integers(0, n, 509)]))


def _band_csr_properties(sig, mem, off, nb, band, K):
    n = mem.numel()
    nb = int(nb)
    o = off[:nb + 1].long()
    assert int(o[0]) == 0 and int(o[-1]) == n and bool((o[1:] > o[:-1]).all())
    m64 = mem.long()
    assert torch.equal(torch.sort(m64).values, torch.arange(n, device="cuda"))
    start = torch.zeros(n, dtype=torch.bool, device="cuda")
    start[o[:-1]] = True
    inner = ~start[1:]
    assert bool((m64[1:][inner] > m64[:-1][inner]).all())
    heads = m64[o[:-1]]
    assert bool((heads[1:] > heads[:-1]).all())
    key = sig[:, band * K:(band + 1) * K].long()[m64]
    assert bool((key[1:][inner] == key[:-1][inner]).all())
    assert torch.unique(key[o[:-1]], dim=0).shape[0] == nb


def test_full_sets():
    api = gpu_api()
    cfg = CONFIGS["sets"]
    n, K, L = cfg["n"], cfg["K"], cfg["L"]
    announce(f"full size sets: generating n={n}")
    off, tok, lab = sparse_sets(n, cfg["vocab"], cfg["clusters"], seed=0, device="cuda")
    mh = key_words(K * L, 0, STREAM_MINHASH)
    sig = api.hash_sets(off, tok, torch.from_numpy(mh.view(np.int32)).cuda())
    rows = _rows(n, 21)
    off_h = off.cpu().numpy()
    parts = [tok[int(off_h[i]):int(off_h[i + 1])].cpu().numpy().view(np.uint32) for i in rows]
    sub_off = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    ref = oracle.minhash_sets(sub_off, np.concatenate(parts), mh)
    assert np.array_equal(host_u32(sig[torch.from_numpy(rows).cuda()]), ref)
    announce("full size sets: bucketize")
    mem, boff, nb, _ = api.bucketize(sig, n, L, K, K, K * L, want_bucket_of=False)
    for band in (0, L - 1):
        _band_csr_properties(sig, mem[band], boff[band], nb[band], band, K)
    announce("full size sets: assign")
    so, sm = planted_seeds(lab, cfg["clusters"], 32)
    k = len(so) - 1
    out = api.assign_sig(sig, torch.from_numpy(so.view(np.int32)).cuda(), torch.from_numpy(sm.view(np.int32)).cuda(), k)
    S_members = host_u32(sig[torch.from_numpy(sm.astype(np.int64)).cuda()])
    M = oracle.modes(S_members, so, np.arange(len(sm), dtype=np.uint32))
    assert np.array_equal(host_u32(out["modes"]), M)
    a, dist = oracle.assign_sig(host_u32(sig[torch.from_numpy(rows).cuda()]), M)
    assert np.array_equal(out["assign"].cpu().numpy()[rows], a)
    assert np.array_equal(out["dist"].cpu().numpy()[rows], dist)


def test_full_hetero():
    api = gpu_api()
    cfg = CONFIGS["hetero"]
    n = cfg["n"]
    announce(f"full size hetero: generating n={n}")
    X, cat, lab, _ = hetero_rows(n, cfg["d_num"], cfg["n_cat"], cfg["clusters"], seed=0)
    A, b = e2lsh_params(cfg["P_h"], cfg["d_num"], cfg["w"], 0)
    K, L = cfg["K"], cfg["L"]
    mh = key_words(K * L, 0, STREAM_MINHASH)
    Xg, catg = torch.from_numpy(X).cuda(), torch.from_numpy(cat).cuda()
    sig = api.hash_hetero(Xg, catg, torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda(), cfg["P_h"], 1,
                          cfg["w"], torch.from_numpy(mh.view(np.int32)).cuda())
    rows = _rows(n, 22)
    codes = oracle.e2lsh_codes(X[rows], A, b, cfg["w"])
    tk = oracle.hetero_tokens(cat[rows], codes)
    ref = oracle.minhash_sets(np.arange(0, tk.size + 1, tk.shape[1], dtype=np.int64), tk.reshape(-1), mh)
    assert np.array_equal(host_u32(sig[torch.from_numpy(rows).cuda()]), ref)
    announce("full size hetero: bucketize")
    mem, boff, nb, _ = api.bucketize(sig, n, L, K, K, K * L, want_bucket_of=False)
    _band_csr_properties(sig, mem[0], boff[0], nb[0], 0, K)
    so, sm = planted_seeds(lab, cfg["clusters"], 32)
    k = len(so) - 1
    Cn = oracle.centroids(X, so, sm)
    Mc = oracle.modes(cat, so, sm)
    a, dist = oracle.assign_hetero(X[rows], cat[rows], Cn, Mc, 1.0)
    # FP8 (e4m3) numeric part as the workload states it, then BF16
    for prec in (2, 1):
        announce(f"full size hetero: assign prec={prec}")
        out = api.assign_hetero(Xg, catg, torch.from_numpy(so.view(np.int32)).cuda(),
                                torch.from_numpy(sm.view(np.int32)).cuda(), k, 1.0, prec)
        assert np.array_equal(out["centroids"].cpu().numpy(), Cn)
        assert np.array_equal(out["modes"].cpu().numpy(), Mc)
        got_a = out["assign"].cpu().numpy()
        assert np.array_equal(got_a[rows], a)
        got_d = out["dist"].cpu().numpy()
        assert np.array_equal(got_d[rows], dist)
        # every row's distance to its assigned seed and the SSE from the
        # oracle's arithmetic over all rows
        d_all = oracle.hetero_dist_pairs(X, cat, Cn, Mc, got_a, 1.0)
        assert np.array_equal(got_d, d_all)
        assert out["sse"].item() == oracle.sse(d_all)


def test_full_batched_jobs():
    # the 256-job batched workload: one batched BF16 assignment over all jobs;
    # eight jobs (the largest, the smallest and six drawn) equal their
    # single-job calls bit for bit and match the oracle on sampled rows
    api = gpu_api()
    from workloads import batched_jobs, dense_mixture

    specs = batched_jobs(CONFIGS["batched"]["jobs"], seed=0)
    announce(f"full size batched: generating {len(specs)} jobs")
    probs, host = [], []
    for sp in specs:
        X, lab, _ = dense_mixture(sp["n"], sp["d"], sp["clusters"], sp["lo"], sp["hi"], sp["sigma"],
                                  sp["sizes"], sp["seed"], device="cuda")
        so, sm = planted_seeds(lab, sp["clusters"], 32)
        probs.append((X, torch.from_numpy(so.view(np.int32)).cuda(), torch.from_numpy(sm.view(np.int32)).cuda(),
                      len(so) - 1))
        host.append((so, sm))
    outs, t_done = api.assign_euclid_batch(probs, 1)
    sizes = [sp["n"] for sp in specs]
    g = np.random.default_rng(23)
    pick = sorted(set([int(np.argmax(sizes)), int(np.argmin(sizes))] + g.choice(len(specs), 6, replace=False).tolist()))
    assert bool((t_done > 0).all())
    for j in pick:
        X, sog, smg, k = probs[j]
        announce(f"full size batched: job {j} n={X.shape[0]} d={X.shape[1]} k={k}")
        one = api.assign_euclid(X, sog, smg, k, 1)
        for key in ("assign", "centroids", "dist", "sse", "radius"):
            assert torch.equal(outs[j][key], one[key]), (j, key)
        so, sm = host[j]
        Xm = X[torch.from_numpy(sm.astype(np.int64)).cuda()].cpu().numpy()
        C = oracle.centroids(Xm, so, np.arange(len(sm), dtype=np.uint32))
        assert np.array_equal(one["centroids"].cpu().numpy(), C)
        rows = _rows(X.shape[0], 30 + j)
        a, dist = oracle.assign_euclid(X[torch.from_numpy(rows).cuda()].cpu().numpy(), C)
        assert np.array_equal(one["assign"].cpu().numpy()[rows], a)
        assert np.array_equal(one["dist"].cpu().numpy()[rows], dist)


def test_full_silk_pass_properties():
    # the SILK pass of the benchmark (10^6 points of the dense mixture, scaled
    # width, 32 tables, K_S = 3, L_S = 20, delta = 10): the seed CSR is
    # canonical (members ascending, every seed at least delta members) and a
    # second run gives the same seeds and counters bit for bit
    api = gpu_api()
    from workloads import dense_mixture
    from workloads.gen import STREAM_SILK

    cfg = CONFIGS["dense_large"]
    n, d, m, L = 1_000_000, cfg["d"], cfg["m"], cfg["L"]
    w = cfg["w"] * d ** 0.5
    K, LS, delta = cfg["K_S"], cfg["L_S"], cfg["delta"]
    announce(f"full size silk pass: n={n}")
    X, _, _ = dense_mixture(n, d, cfg["clusters"] * n // cfg["n"], cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"],
                            seed=0, device="cuda")
    A, b = e2lsh_params(m * L, d, w, 0)
    keys = torch.from_numpy(key_words((LS + 1) * K, 0, STREAM_SILK).view(np.int32)).cuda()
    kg, _ = api.hash_dense(X, torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda(), m, L, w)
    bm, bo, bn, _ = api.bucketize(kg, n, L, 4, n * 4, 4, want_bucket_of=False)
    runs = [api.silk_seeds(bm, bo, bn, n, L, K, LS, delta, keys) for _ in range(2)]
    so, sm, ctr = (host_u32(runs[0][0]), host_u32(runs[0][1]), runs[0][2].cpu().numpy())
    assert np.array_equal(so, host_u32(runs[1][0])) and np.array_equal(sm, host_u32(runs[1][1]))
    assert np.array_equal(ctr, runs[1][2].cpu().numpy())
    k = len(so) - 1
    assert k > 1000 and so[0] == 0 and so[-1] == len(sm)
    sizes = np.diff(so.astype(np.int64))
    assert (sizes >= delta).all()
    assert int(sm.max()) < n
    seg = np.repeat(np.arange(k), sizes)
    inner = seg[1:] == seg[:-1]
    assert (sm[1:][inner].astype(np.int64) > sm[:-1][inner].astype(np.int64)).all()


def test_full_silk_pass_matches_oracle_digest(golden_dir):
    # the SILK pass at 10^6 points (numpy-drawn mixture, 32 tables, K_S = 3,
    # L_S = 20, delta = 10) against the oracle's seed CSR, stored as digests
    # by tests/golden/make_silk_dense_1e6.py (oracle only)
    import hashlib
    import json
    import os

    from workloads import dense_mixture
    from workloads.gen import STREAM_SILK

    api = gpu_api()
    with open(os.path.join(golden_dir, "silk_dense_1e6.json")) as f:
        ref = json.load(f)
    cfg = CONFIGS["dense_large"]
    n, d, m, L = ref["n"], cfg["d"], cfg["m"], cfg["L"]
    w = cfg["w"] * d ** 0.5
    K, LS, delta = cfg["K_S"], cfg["L_S"], cfg["delta"]
    announce(f"full size silk vs oracle digest: n={n}")
    X, _, _ = dense_mixture(n, d, cfg["clusters"] * n // cfg["n"], cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"],
                            seed=0)
    A, b = e2lsh_params(m * L, d, w, 0)
    keys = torch.from_numpy(key_words((LS + 1) * K, 0, STREAM_SILK).view(np.int32)).cuda()
    kg, _ = api.hash_dense(torch.from_numpy(X).cuda(), torch.from_numpy(A).cuda(), torch.from_numpy(b).cuda(), m, L, w)
    bm, bo, bn, _ = api.bucketize(kg, n, L, 4, n * 4, 4, want_bucket_of=False)
    assert int(bn.sum()) == ref["buckets_total"]
    so, sm, ctr = api.silk_seeds(bm, bo, bn, n, L, K, LS, delta, keys)
    so, sm, ctr = host_u32(so), host_u32(sm), ctr.cpu().numpy()
    assert len(so) - 1 == ref["k"] and len(sm) == ref["members"]
    assert ctr[0] == ref["hash_evals"] and ctr[1] == ref["pairs_voted"] and ctr[2] == ref["multiset"]
    for j, seed in ref["sample_seeds"].items():
        j = int(j)
        assert int(so[j + 1] - so[j]) == seed["size"], j
        assert sm[so[j]:so[j + 1]][:64].tolist() == seed["first"], j
    assert hashlib.sha256(so.astype("<u4").tobytes()).hexdigest() == ref["sha256_seed_offsets"]
    assert hashlib.sha256(sm.astype("<u4").tobytes()).hexdigest() == ref["sha256_seed_members"]
