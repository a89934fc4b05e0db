"""The small dense workload end to end at its stated size, element by element
against the oracle: 20,000 points, d = 32, 50 equal Gaussian clusters
(centres uniform in [-10, 10]^32, sigma = 1); E2LSH m = 8 x L = 16 tables;
SILK K = 3, L = 20, delta = 10; then the one-pass assignment to the SILK
seeds.  With the literal width w = 4 almost every point is alone in its
buckets and SILK finds no seed; with the scaled width w * sqrt(d) the whole
pass -- codes, buckets, seeds, centroids, assignment, distances and SSE --
equals the oracle's."""

import math

import numpy as np
import pytest
import torch

import oracle
from workloads import CONFIGS, dense_mixture, e2lsh_params, key_words
from workloads.gen import STREAM_SILK

from .gpu_util import announce, cuda, gpu_api, host_u32, unpack_keys

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    cfg = CONFIGS["dense_small"]
    X, _, _ = dense_mixture(cfg["n"], cfg["d"], cfg["clusters"], cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"],
                            seed=0)
    keys = key_words((cfg["L_S"] + 1) * cfg["K_S"], 0, STREAM_SILK)
    return cfg, X, keys


def _pass(api, cfg, X, keys, w):
    n, d, m, L = cfg["n"], cfg["d"], cfg["m"], cfg["L"]
    K, LS, delta = cfg["K_S"], cfg["L_S"], cfg["delta"]
    A, b = e2lsh_params(m * L, d, w, 0)
    codes = oracle.e2lsh_codes(X, A, b, w)
    tables = oracle.bucketize_tables(codes, m, L)
    offs, mem = [0], []
    for mm, oo, _ in tables:
        mem.append(mm)
        offs.extend((oo[1:].astype(np.int64) + offs[-1]).tolist())
    ref_o, ref_m, info = oracle.silk_seeds(np.asarray(offs), np.concatenate(mem), K, LS, delta, keys)
    announce(f"small pipeline w={w:.3f}: oracle k={len(ref_o) - 1}")
    Xg = cuda(X)
    kg, cg = api.hash_dense(Xg, cuda(A), cuda(b), m, L, w, want_codes=True)
    assert np.array_equal(cg.cpu().numpy().astype(np.int64), codes)
    assert np.array_equal(unpack_keys(host_u32(kg), m), codes)
    bm, bo, bn, bof = api.bucketize(kg, n, L, 4, n * 4, 4)
    for t, (rm, ro, rb) in enumerate(tables):
        assert int(bn[t]) == len(ro) - 1, t
        assert np.array_equal(host_u32(bm[t]), rm), t
        assert np.array_equal(host_u32(bo[t])[:len(ro)], ro), t
        assert np.array_equal(host_u32(bof[t]), rb), t
    status = api.new_status("cuda")
    so, sm, ctr = api.silk_seeds(bm, bo, bn, n, L, K, LS, delta, cuda(keys), status=status, check=False)
    ctr = ctr.cpu().numpy()
    assert ctr[0] == info["hash_evals"] and ctr[1] == info["pairs_voted"] and ctr[2] == info["multiset"]
    return Xg, (ref_o, ref_m), (host_u32(so), host_u32(sm)), int(status.item())


def test_small_literal_width_has_no_seed(small):
    api = gpu_api()
    cfg, X, keys = small
    Xg, (ro, rm), (go, gm), st = _pass(api, cfg, X, keys, cfg["w"])
    assert len(ro) == 1 and len(rm) == 0
    assert st == 4 and len(go) == 1  # GEEK_ERR_NO_SEEDS


@pytest.mark.parametrize("prec", [0, 1])
def test_small_scaled_width_whole_pass(small, prec):
    api = gpu_api()
    cfg, X, keys = small
    w = cfg["w"] * math.sqrt(cfg["d"])
    Xg, (ro, rm), (go, gm), st = _pass(api, cfg, X, keys, w)
    assert st == 0
    assert len(ro) - 1 == 485  # k* of this workload under the scaled width
    assert np.array_equal(go, ro) and np.array_equal(gm, rm)
    k = len(ro) - 1
    C = oracle.centroids(X, ro, rm)
    a, dist = oracle.assign_euclid(X, C)
    announce(f"small pipeline: assign k={k} prec={prec}")
    out = api.assign_euclid(Xg, cuda(go.view(np.int32)), cuda(gm.view(np.int32)), k, prec)
    assert np.array_equal(out["centroids"].cpu().numpy(), C)
    assert np.array_equal(out["assign"].cpu().numpy(), a)
    assert np.array_equal(out["dist"].cpu().numpy(), dist)
    assert out["sse"].item() == oracle.sse(dist)
    assert np.array_equal(out["radius"].cpu().numpy(), oracle.radius(dist, a, k))
