"""GPU parity of geek_assign with GEEK_METRIC_SIG (sets: modes of MinHash
signatures, argmax of matching positions) against the oracle, bit for bit."""

import numpy as np
import pytest

import oracle
from workloads import key_words, sparse_sets

from .gpu_util import announce, cuda, gpu_api, host_u32

pytestmark = pytest.mark.gpu


def _seeds_from_labels(lab, clusters, per, g):
    offs, mem = [0], []
    for c in range(clusters):
        ids = np.flatnonzero(lab == c)
        if len(ids) == 0:
            continue
        take = np.sort(g.choice(ids, size=min(per, len(ids)), replace=False))
        mem.append(take)
        offs.append(offs[-1] + len(take))
    return np.asarray(offs, np.uint32), np.concatenate(mem).astype(np.uint32)


def _check(api, sig, so, sm, name):
    k = len(so) - 1
    announce(f"assign-sig {name} n={len(sig)} F={sig.shape[1]} k={k}")
    M = oracle.modes(sig, so, sm)
    a, dist = oracle.assign_sig(sig, M)
    out = api.assign_sig(cuda(sig), cuda(so), cuda(sm), k)
    assert np.array_equal(host_u32(out["modes"]), M)
    got = out["assign"].cpu().numpy()
    bad = np.flatnonzero(got != a)
    assert bad.size == 0, (bad[:10], got[bad[:10]], a[bad[:10]])
    assert np.array_equal(out["dist"].cpu().numpy(), dist)
    assert out["sse"].item() == oracle.sse(dist)
    assert np.array_equal(out["radius"].cpu().numpy(), oracle.radius(dist, a, k, euclid=False))
    return out["counters"].cpu().numpy()


@pytest.mark.parametrize("n,F,clusters,per,seed", [(3000, 256, 40, 12, 0), (2000, 128, 100, 3, 1),
                                                   (1500, 64, 7, 50, 2)])
def test_sig_assign_matches_oracle(n, F, clusters, per, seed):
    api = gpu_api()
    off, tok, lab = sparse_sets(n, vocab=30_000, clusters=clusters, seed=seed)
    sig = oracle.minhash_sets(off, tok, key_words(F, seed))
    g = np.random.default_rng(seed)
    so, sm = _seeds_from_labels(lab, clusters, per, g)
    ctr = _check(api, sig, so, sm, "sets")
    assert ctr[0] + ctr[2] == n


def test_sig_assign_ties_and_dense_fallback():
    # tiny alphabet: many seeds share mode values, so rows gather long match
    # lists (dense fallback) and equal counts (lowest index wins)
    api = gpu_api()
    g = np.random.default_rng(3)
    n, F, k = 1200, 96, 300
    sig = g.integers(0, 3, size=(n, F)).astype(np.uint32)
    so = np.arange(0, 3 * k + 1, 3, dtype=np.uint32)
    sm = np.sort(g.choice(n, size=3 * k, replace=True).reshape(k, 3), axis=1).reshape(-1).astype(np.uint32)
    ctr = _check(api, sig, so, sm, "ties")
    assert ctr[2] > 0


@pytest.mark.parametrize("alphabet", [100_000, 4])
def test_sig_assign_many_seeds_index_path(alphabet):
    # k * F above the direct-comparison limit: rows go through the inverted
    # index on (position, mode value); with a 4-letter alphabet most rows'
    # match lists overflow and fall back to comparing against every mode
    api = gpu_api()
    g = np.random.default_rng(11 + alphabet)
    n, F, k = 600, 256, 4500
    sig = g.integers(0, alphabet, size=(n, F)).astype(np.uint32)
    sizes = g.integers(1, 4, size=k)
    so = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    sm = np.concatenate([np.sort(g.choice(n, size=s, replace=False)) for s in sizes]).astype(np.uint32)
    ctr = _check(api, sig, so, sm, f"index alphabet={alphabet}")
    assert ctr[0] + ctr[2] == n
    if alphabet > 4:
        assert ctr[0] > 0  # resolved by the index
    else:
        assert ctr[2] > 0  # dense fallback
