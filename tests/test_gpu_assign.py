"""GPU parity of geek_assign (Euclidean) against the FP64 oracle: centroids,
assignments, distances and SSE bit for bit, radius to 1e-13 relative."""

import numpy as np
import pytest

import oracle
from workloads import dense_mixture, e2lsh_params, key_words, planted_seeds
from workloads.gen import STREAM_SILK

from .gpu_util import announce, cuda, gpu_api

pytestmark = pytest.mark.gpu

PRECS = {"fp32": 0, "bf16": 1}


def _check(api, X, so, sm, prec, name):
    k = len(so) - 1
    announce(f"assign {name} n={len(X)} d={X.shape[1]} k={k} prec={prec}")
    C = oracle.centroids(X, so, sm)
    a, dist = oracle.assign_euclid(X, C)
    sse = oracle.sse(dist)
    rad = oracle.radius(dist, a, k)
    out = api.assign_euclid(cuda(X), cuda(so), cuda(sm), k, PRECS[prec])
    assert np.array_equal(out["centroids"].cpu().numpy(), C)
    got = out["assign"].cpu().numpy()
    bad = np.flatnonzero(got != a)
    assert bad.size == 0, (bad[:10], got[bad[:10]], a[bad[:10]])
    assert np.array_equal(out["dist"].cpu().numpy(), dist)
    assert out["sse"].item() == sse
    np.testing.assert_allclose(out["radius"].cpu().numpy(), rad, rtol=1e-13, atol=0)
    ctr = out["counters"].cpu().numpy()
    assert ctr[0] + ctr[1] + ctr[2] >= len(X) and ctr[0] + ctr[2] <= len(X)
    return ctr


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,d,clusters,per,seed", [
    (3000, 32, 50, 32, 0),     # one centroid tile (k=50 padded to 64), ragged rows
    (5000, 128, 300, 8, 1),    # five centroid tiles, 40 row tiles
    (2000, 20, 40, 16, 2),     # d padded to 32
    (1500, 256, 70, 4, 3),     # widest d
    (777, 64, 129, 2, 4),      # k just above two tiles
])
def test_assign_planted(prec, n, d, clusters, per, seed):
    api = gpu_api()
    X, lab, _ = dense_mixture(n, d, clusters, -10, 10, 1.0, "equal", seed)
    so, sm = planted_seeds(lab, clusters, per)
    _check(api, X, so, sm, prec, "planted")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_assign_silk_seeds_many_per_cluster(prec):
    # seeds from the oracle's SILK on the scaled small dense config: several
    # seeds per cluster, so rows have many near-tied candidates
    api = gpu_api()
    n, d, m, L = 4000, 32, 8, 16
    X, lab, _ = dense_mixture(n, d, 20, -10, 10, 1.0, "equal", 5)
    w = 4.0 * np.sqrt(d)
    A, b = e2lsh_params(m * L, d, w, 5)
    codes = oracle.e2lsh_codes(X, A, b, w)
    offs, mem = [0], []
    for mm, oo, _ in oracle.bucketize_tables(codes, m, L):
        mem.append(mm)
        offs.extend((oo[1:].astype(np.int64) + offs[-1]).tolist())
    keys = key_words(21 * 3, 5, STREAM_SILK)
    so, sm, _ = oracle.silk_seeds(np.asarray(offs), np.concatenate(mem), 3, 20, 10, keys)
    assert len(so) - 1 > 40
    ctr = _check(api, X, so, sm, prec, "silk-seeds")
    if prec == "bf16":
        assert ctr[1] > 0  # the bf16 window overflowed for some rows


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_assign_ties_and_degenerate(prec):
    api = gpu_api()
    X, lab, _ = dense_mixture(1000, 16, 10, -10, 10, 1.0, "equal", 6)
    # duplicated seeds (identical centroids): exact ties, lowest index wins;
    # single-point seeds: those points are at distance 0
    so = np.array([0, 5, 10, 11, 12, 17], dtype=np.uint32)
    sm = np.array([1, 2, 3, 4, 5, 1, 2, 3, 4, 5, 40, 41, 1, 2, 3, 4, 5], dtype=np.uint32)
    _check(api, X, so, sm, prec, "ties")
    _check(api, X, np.array([0, 1000], np.uint32), np.arange(1000, dtype=np.uint32), prec, "k=1")
    _check(api, X[:1], np.array([0, 1], np.uint32), np.array([0], np.uint32), prec, "n=1")


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,d,clusters,copies,seed", [
    (3000, 32, 10, 36, 8),     # 47 row groups: seed tiles split over workgroups
    (2000, 100, 40, 36, 9),    # k = 1440 (23 tiles) in 16 uneven splits, d padded
    (70000, 16, 10, 34, 10),   # 1094 row groups: no split, direct writes
])
def test_assign_full_scan_rows(prec, n, d, clusters, copies, seed):
    # every planted seed repeated `copies` (> 32) times: each row keeps more
    # exact ties than any candidate window, so every row takes the float64
    # scan over all seeds and must land on the first copy
    api = gpu_api()
    X, lab, _ = dense_mixture(n, d, clusters, -10, 10, 1.0, "equal", seed)
    so1, sm1 = planted_seeds(lab, clusters, 6)
    offs, mem = [0], []
    for c in range(len(so1) - 1):
        for _ in range(copies):
            mem.append(sm1[so1[c]:so1[c + 1]])
            offs.append(offs[-1] + len(mem[-1]))
    so, sm = np.asarray(offs, np.uint32), np.concatenate(mem).astype(np.uint32)
    ctr = _check(api, X, so, sm, prec, f"full-scan copies={copies}")
    assert ctr[2] == n


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,d,clusters,copies,seed", [
    (3000, 32, 10, 36, 8),    # every row takes the float64 scan (seed tiles split)
    (5000, 128, 300, 1, 1),   # rows settled by the first pass
])
def test_assign_device_seed_count(prec, n, d, clusters, copies, seed):
    # the seed count read by the kernels from device memory (k_dev); the host
    # k is a capacity with 200 further seeds behind the count, each a single
    # row (at distance 0 from that row, were it to take part).  The result is
    # the oracle's on the counted seeds; centroid and radius rows past the
    # count are zero.
    import torch

    api = gpu_api()
    X, lab, _ = dense_mixture(n, d, clusters, -10, 10, 1.0, "equal", seed)
    so1, sm1 = planted_seeds(lab, clusters, 6)
    offs, mem = [0], []
    for c in range(len(so1) - 1):
        for _ in range(copies):
            mem.append(sm1[so1[c]:so1[c + 1]])
            offs.append(offs[-1] + len(mem[-1]))
    k, extra = len(offs) - 1, 200
    for i in range(extra):
        mem.append(np.array([i], np.uint32))
        offs.append(offs[-1] + 1)
    so, sm = np.asarray(offs, np.uint32), np.concatenate(mem).astype(np.uint32)
    announce(f"assign device count n={n} d={d} k={k} capacity={k + extra} prec={prec}")
    C = oracle.centroids(X, so[:k + 1], sm[:so[k]])
    a, dist = oracle.assign_euclid(X, C)
    kd = torch.tensor([k], dtype=torch.int32, device="cuda")
    out = api.assign_euclid(cuda(X), cuda(so), cuda(sm), k + extra, PRECS[prec], k_dev=kd)
    cen = out["centroids"].cpu().numpy()
    assert np.array_equal(cen[:k], C) and not cen[k:].any()
    assert np.array_equal(out["assign"].cpu().numpy(), a)
    assert np.array_equal(out["dist"].cpu().numpy(), dist)
    assert out["sse"].item() == oracle.sse(dist)
    rad = out["radius"].cpu().numpy()
    np.testing.assert_allclose(rad[:k], oracle.radius(dist, a, k), rtol=1e-13, atol=0)
    assert not rad[k:].any()


@pytest.mark.parametrize("n,d,clusters", [
    (12000, 8, 6000),    # k = 6000: per-workgroup radius maxima in a 128 KB LDS table
    (30000, 4, 30000),   # k = 30000: radius by global atomics
])
def test_assign_many_seeds_radius_paths(n, d, clusters):
    api = gpu_api()
    X, lab, _ = dense_mixture(n, d, clusters, -10, 10, 1.0, "equal", 11)
    so, sm = planted_seeds(lab, clusters, 2)
    _check(api, X, so, sm, "bf16", f"radius k={len(so) - 1}")


def test_assign_nonfinite_input_is_reported():
    api = gpu_api()
    from paper_2106_10515_amd import GeekError

    X, lab, _ = dense_mixture(300, 32, 3, -10, 10, 1.0, "equal", 7)
    X[17, 5] = np.nan
    so, sm = planted_seeds(lab, 3, 4)
    sm = sm[~np.isin(sm, [17])] if 17 in sm else sm
    so = np.array([0, len(sm)], np.uint32)
    with pytest.raises(GeekError) as e:
        api.assign_euclid(cuda(X), cuda(so), cuda(sm), 1, 0)
    assert e.value.code == 1
