"""GPU parity of geek_assign for heterogeneous rows (numeric centroid +
categorical modes, D = squared distance + gamma * mismatches) and of the FP8
matrix-core path for Euclidean data, against the oracle, bit for bit."""

import numpy as np
import pytest

import oracle
from workloads import dense_mixture, hetero_rows, planted_seeds

from .gpu_util import announce, cuda, gpu_api, host_u32

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("n,clusters,per,gamma,seed", [(4000, 60, 12, 1.0, 0), (2500, 30, 5, 0.5, 1),
                                                       (1800, 25, 40, 4.0, 2)])
def test_hetero_matches_oracle(prec, n, clusters, per, gamma, seed):
    api = gpu_api()
    X, cat, lab, _ = hetero_rows(n, 20, 10, clusters, seed=seed)
    so, sm = planted_seeds(lab, clusters, per)
    k = len(so) - 1
    announce(f"assign-hetero n={n} k={k} gamma={gamma} prec={prec}")
    Cn = oracle.centroids(X, so, sm)
    Mc = oracle.modes(cat, so, sm)
    a, dist = oracle.assign_hetero(X, cat, Cn, Mc, gamma)
    out = api.assign_hetero(cuda(X), cuda(cat), cuda(so), cuda(sm), k, gamma, prec)
    assert np.array_equal(out["centroids"].cpu().numpy(), Cn)
    assert np.array_equal(out["modes"].cpu().numpy(), Mc)
    got = out["assign"].cpu().numpy()
    bad = np.flatnonzero(got != a)
    assert bad.size == 0, (bad[:10], got[bad[:10]], a[bad[:10]])
    assert np.array_equal(out["dist"].cpu().numpy(), dist)
    assert out["sse"].item() == oracle.sse(dist)
    assert np.array_equal(out["radius"].cpu().numpy(), oracle.radius(dist, a, k, euclid=False))


@pytest.mark.parametrize("n,d,clusters,per,seed", [(3000, 32, 50, 16, 0), (2000, 128, 100, 8, 1),
                                                   (1500, 20, 30, 2, 2)])
def test_fp8_euclid_matches_oracle(n, d, clusters, per, seed):
    api = gpu_api()
    X, lab, _ = dense_mixture(n, d, clusters, -10, 10, 1.0, "equal", seed)
    so, sm = planted_seeds(lab, clusters, per)
    k = len(so) - 1
    announce(f"assign-fp8 n={n} d={d} k={k}")
    C = oracle.centroids(X, so, sm)
    a, dist = oracle.assign_euclid(X, C)
    out = api.assign_euclid(cuda(X), cuda(so), cuda(sm), k, 2)
    assert np.array_equal(out["assign"].cpu().numpy(), a)
    assert np.array_equal(out["dist"].cpu().numpy(), dist)
    assert out["sse"].item() == oracle.sse(dist)


@pytest.mark.parametrize("metric", ["euclid", "hetero"])
def test_bf16_first_pass_settles_well_separated_rows(metric):
    # planted clusters far apart relative to the BF16 error bound: the first
    # pass must settle (almost) every row by itself, with padded centroid
    # slots present (k = 100 is padded to 128) and for both epilogues
    api = gpu_api()
    X, cat, lab, _ = hetero_rows(6000, 20, 10, 100, seed=7)
    so, sm = planted_seeds(lab, 100, 16)
    k = len(so) - 1
    announce(f"bf16 first pass settles {metric} n=6000 k={k}")
    if metric == "euclid":
        out = api.assign_euclid(cuda(X), cuda(so), cuda(sm), k, 1)
        a, _ = oracle.assign_euclid(X, oracle.centroids(X, so, sm))
    else:
        out = api.assign_hetero(cuda(X), cuda(cat), cuda(so), cuda(sm), k, 1.0, 1)
        a, _ = oracle.assign_hetero(X, cat, oracle.centroids(X, so, sm), oracle.modes(cat, so, sm), 1.0)
    assert np.array_equal(out["assign"].cpu().numpy(), a)
    ctr = out["counters"].cpu().numpy()
    assert ctr[0] >= 0.99 * len(X), ctr
