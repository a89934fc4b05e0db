"""Parity at the full dense workload size, in the launch configuration the
benchmark times (10^7 points, d = 128, 10,000-cluster Zipf mixture; E2LSH
m = 10 x 32 tables, w = 8; 10,000 planted seeds of up to 32 members): on
sampled outputs the FP64 oracle computes one by one, and on properties that
hold at any size.  Also the further assignment pass and Algorithm 1's
quantile bucketing at that size."""

import numpy as np
import pytest
import torch

import oracle
from workloads import CONFIGS, dense_mixture, e2lsh_params, planted_seeds

from .gpu_util import announce, gpu_api, host_u32, unpack_keys

pytestmark = pytest.mark.gpu

N = 10_000_000


@pytest.fixture(scope="module")
def big():
    api = gpu_api()
    cfg = CONFIGS["dense_large"]
    d, m, L, w = cfg["d"], cfg["m"], cfg["L"], cfg["w"]
    announce(f"full size: generating n={N} d={d}")
    X, labels, _ = dense_mixture(N, d, cfg["clusters"], cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"],
                                 seed=0, device="cuda")
    A, b = e2lsh_params(m * L, d, w, 0)
    so, sm = planted_seeds(labels, cfg["clusters"], 32)
    g = np.random.default_rng(11)
    rows = np.unique(np.concatenate([[0, N - 1], g.integers(0, N, 509)]))
    return dict(api=api, X=X, A=A, b=b, so=so, sm=sm, d=d, m=m, L=L, w=w, rows=rows, g=g)


def _host_rows(X, rows):
    return X[torch.from_numpy(rows).cuda()].cpu().numpy()


def _check_csr(mem, off, nb):
    """Properties of one table's bucket CSR on the device: a partition of
    [0, n) into non-empty buckets, members ascending, buckets ordered by their
    smallest member."""
    n = mem.numel()
    nb = int(nb)
    o = off[:nb + 1].long()
    assert int(o[0]) == 0 and int(o[-1]) == n and bool((o[1:] > o[:-1]).all())
    assert torch.equal(torch.sort(mem.long()).values, torch.arange(n, device=mem.device))
    start = torch.zeros(n, dtype=torch.bool, device=mem.device)
    start[o[:-1]] = True
    m64 = mem.long()
    inner = ~start[1:]
    assert bool((m64[1:][inner] > m64[:-1][inner]).all())        # ascending members
    heads = m64[o[:-1]]
    assert bool((heads[1:] > heads[:-1]).all())                   # ordered by smallest member
    return o, start


def _keys(big):
    if "keys" not in big:
        big["keys"], _ = big["api"].hash_dense(big["X"], torch.from_numpy(big["A"]).cuda(),
                                               torch.from_numpy(big["b"]).cuda(), big["m"], big["L"], big["w"])
    return big["keys"]


def _first_assign(big):
    if "assign" not in big:
        so, sm = big["so"], big["sm"]
        big["assign"] = big["api"].assign_euclid(big["X"], torch.from_numpy(so.view(np.int32)).cuda(),
                                                 torch.from_numpy(sm.view(np.int32)).cuda(), len(so) - 1,
                                                 1)["assign"]
    return big["assign"]


def test_full_hash_sampled_rows(big):
    announce("full size: hash")
    keys = _keys(big)
    rows = big["rows"]
    ref = oracle.e2lsh_codes(_host_rows(big["X"], rows), big["A"], big["b"], big["w"])
    got = unpack_keys(host_u32(keys[:, torch.from_numpy(rows).cuda(), :]), big["m"])
    assert np.array_equal(got, ref)


def test_full_bucketize_properties(big):
    api = big["api"]
    keys = _keys(big)
    announce("full size: bucketize")
    mem, off, nb, bof = api.bucketize(keys, N, big["L"], 4, N * 4, 4)
    for t in (0, big["L"] - 1):
        o, start = _check_csr(mem[t], off[t], nb[t])
        kt = keys[t].long()
        km = kt[mem[t].long()]
        inner = ~start[1:]
        assert bool((km[1:][inner] == km[:-1][inner]).all())     # one key per bucket
        heads = km[o[:-1]]
        assert torch.unique(heads, dim=0).shape[0] == int(nb[t])  # different buckets, different keys
        sizes = o[1:] - o[:-1]
        bucket = torch.repeat_interleave(torch.arange(int(nb[t]), device="cuda"), sizes)
        assert torch.equal(bof[t].long()[mem[t].long()], bucket)


@pytest.mark.parametrize("prec", [1, 0])
def test_full_assign_sampled_rows(big, prec):
    api = big["api"]
    so, sm = big["so"], big["sm"]
    k = len(so) - 1
    announce(f"full size: assign prec={prec} k={k}")
    out = api.assign_euclid(big["X"], torch.from_numpy(so.view(np.int32)).cuda(),
                            torch.from_numpy(sm.view(np.int32)).cuda(), k, prec)
    # centroids: the members' rows, in the same ascending order
    Xm = _host_rows(big["X"], sm.astype(np.int64))
    C = oracle.centroids(Xm, so, np.arange(len(sm), dtype=np.uint32))
    assert np.array_equal(out["centroids"].cpu().numpy(), C)
    rows = big["rows"]
    a, dist = oracle.assign_euclid(_host_rows(big["X"], rows), C)
    assert np.array_equal(out["assign"].cpu().numpy()[rows], a)
    got_dist = out["dist"].cpu().numpy()
    assert np.array_equal(got_dist[rows], dist)
    # every row's distance to its assigned centroid, and the SSE, from the
    # oracle's own arithmetic over all 10^7 rows
    if "Xh" not in big:
        big["Xh"] = big["X"].cpu().numpy()
    announce(f"full size: oracle distances of all rows prec={prec}")
    d_all = oracle.euclid_dist_pairs(big["Xh"], C, out["assign"].cpu().numpy())
    assert np.array_equal(got_dist, d_all)
    assert out["sse"].item() == oracle.sse(d_all)
    if prec == 1:
        big["assign"] = out["assign"]


def test_full_further_pass(big):
    api = big["api"]
    k = len(big["so"]) - 1
    announce("full size: regroup + further pass")
    a = _first_assign(big)
    so2, sm2, k_out, lab = api.regroup(a, k)
    k2 = int(k_out.item())
    counts = torch.bincount(a.long(), minlength=k)
    assert k2 == int((counts > 0).sum())
    assert torch.equal(lab[:k2].long(), torch.nonzero(counts).flatten())
    o = so2[:k2 + 1].long()
    assert int(o[0]) == 0 and int(o[-1]) == N
    assert torch.equal(o[1:] - o[:-1], counts[counts > 0])
    start = torch.zeros(N, dtype=torch.bool, device="cuda")
    start[o[:-1]] = True
    m64 = sm2.long()
    assert bool((m64[1:][~start[1:]] > m64[:-1][~start[1:]]).all())   # ascending members
    assert torch.equal(torch.sort(sm2.long()).values, torch.arange(N, device="cuda"))
    assert torch.equal(a.long()[sm2.long()], torch.repeat_interleave(lab[:k2].long(), o[1:] - o[:-1]))
    out = api.assignment_pass(big["X"], a, k, 1)
    # centroids of the two smallest clusters, and sampled rows against all centroids
    sizes = (o[1:] - o[:-1]).cpu().numpy()
    C = out["centroids"].cpu().numpy()
    for r in np.argsort(sizes, kind="stable")[:2]:
        ids = host_u32(sm2[int(o[r]):int(o[r + 1])]).astype(np.int64)
        Cr = oracle.centroids(_host_rows(big["X"], ids), np.array([0, len(ids)], np.uint32),
                              np.arange(len(ids), dtype=np.uint32))
        assert np.array_equal(C[r], Cr[0])
    rows = big["rows"]
    a2, d2 = oracle.assign_euclid(_host_rows(big["X"], rows), C)
    assert np.array_equal(out["assign"].cpu().numpy()[rows], a2)
    assert np.array_equal(out["dist"].cpu().numpy()[rows], d2)
    assert out["sse"].item() == oracle.sse(out["dist"].cpu().numpy())


def test_full_quantile_properties(big):
    api = big["api"]
    m, t = 2, 10_000
    announce(f"full size: quantile m={m} t={t}")
    A, _ = e2lsh_params(m, big["d"], 1.0, 0)
    mem, off, bof = api.quantile_buckets(big["X"], torch.from_numpy(A).cuda(), t)
    expect = [-(-b * N // t) for b in range(t + 1)]
    for p in range(m):
        assert off[p].cpu().numpy().tolist() == expect
        o = off[p].long()
        assert torch.equal(torch.sort(mem[p].long()).values, torch.arange(N, device="cuda"))
        sizes = o[1:] - o[:-1]
        assert torch.equal(bof[p].long()[mem[p].long()],
                           torch.repeat_interleave(torch.arange(t, device="cuda"), sizes))
        # sampled bucket boundaries: every (value, id) of bucket b below every one of b + 1
        for bb in big["g"].integers(0, t - 1, 6):
            lo = host_u32(mem[p, int(o[bb]):int(o[bb + 1])]).astype(np.int64)
            hi = host_u32(mem[p, int(o[bb + 1]):int(o[bb + 2])]).astype(np.int64)
            assert (np.diff(lo) > 0).all() and (np.diff(hi) > 0).all()
            vl = oracle.qalsh_values(_host_rows(big["X"], lo), A[p:p + 1])[0]
            vh = oracle.qalsh_values(_host_rows(big["X"], hi), A[p:p + 1])[0]
            assert max(zip(vl, lo)) < min(zip(vh, hi))
