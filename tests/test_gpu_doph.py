"""GPU parity of densified one-permutation hashing (geek_hash kind DOPH,
Algorithm 3's first step) against the oracle, bit for bit: planted sparse
sets at the paper's 400 reduced dimensions and at sizes that do not divide
the wavefront or a word of occupancy bits, sets far larger than a wavefront,
sets so small that most bins borrow from the right (including the wrap
round to bin 0), a token universe holding 0 and 2^32 - 1, and the
empty-set error; then the (K, L) band buckets read from the reduced rows."""

import numpy as np
import pytest
import torch

import oracle
from workloads import key_words, sparse_sets

from .gpu_util import announce, cuda, gpu_api, host_u32

pytestmark = pytest.mark.gpu


def _csr(sets):
    off = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int64)
    return off, np.concatenate([np.asarray(s, dtype=np.uint32) for s in sets])


def _case(api, off, tok, key, D, name):
    announce(f"doph {name} n={len(off) - 1} nnz={len(tok)} D={D}")
    ref = oracle.doph_sets(off, tok, key, D)
    got = host_u32(api.hash_doph(cuda(off), cuda(tok), cuda(key.reshape(1, 2)), D))
    bad = np.argwhere(got != ref)
    assert bad.size == 0, (bad[:5], got[tuple(bad[0])], ref[tuple(bad[0])])


@pytest.mark.parametrize("n,D,seed", [(3000, 400, 0), (2500, 1, 1), (2000, 63, 2), (1500, 97, 3),
                                      (1000, 1000, 4), (700, 4096, 5)])
def test_doph_planted_sets_match_oracle(n, D, seed):
    api = gpu_api()
    off, tok, _ = sparse_sets(n, vocab=200_000, clusters=40, seed=seed)
    key = key_words(1, seed)[0]
    _case(api, off, tok, key, D, "planted")


def test_doph_large_tiny_and_extreme_tokens():
    api = gpu_api()
    g = np.random.default_rng(11)
    sets = [np.array([0], np.uint32), np.array([0xFFFFFFFF], np.uint32),
            np.array([0, 0xFFFFFFFF], np.uint32),
            np.sort(g.choice(1 << 32, 5000, replace=False)).astype(np.uint32),
            np.arange(64, dtype=np.uint32), np.arange(65, dtype=np.uint32)]
    for s in range(300):
        sz = int(g.integers(1, 8))
        sets.append(np.sort(g.choice(1 << 20, sz, replace=False)).astype(np.uint32))
    off, tok = _csr(sets)
    for D, seed in ((400, 7), (33, 8), (4096, 9)):
        _case(api, off, tok, key_words(1, seed)[0], D, f"tiny-large D={D}")


def test_doph_empty_set_reports_status():
    api = gpu_api()
    from paper_2106_10515_amd._lib import GEEK_ERR_EMPTY_SET, GeekError

    off = np.array([0, 3, 3, 5], dtype=np.int64)
    tok = np.array([1, 2, 3, 4, 5], dtype=np.uint32)
    with pytest.raises(GeekError) as e:
        api.hash_doph(cuda(off), cuda(tok), cuda(key_words(1, 0)), 400)
    assert e.value.code == GEEK_ERR_EMPTY_SET


def test_doph_band_buckets_match_oracle():
    # Algorithm 3 after the reduction: band b of K rows is coordinates
    # b*K .. b*K+K-1 of the reduced row, bucketed by exact K-tuple
    api = gpu_api()
    n, D, K, L = 4000, 400, 4, 64
    off, tok, _ = sparse_sets(n, vocab=100_000, clusters=30, seed=12)
    key = key_words(1, 12)[0]
    announce(f"doph bands n={n} D={D} K={K} L={L}")
    ref = oracle.doph_sets(off, tok, key, D)
    sig = api.hash_doph(cuda(off), cuda(tok), cuda(key.reshape(1, 2)), D)
    mem, boff, nb, bof = api.bucketize(sig, n, L, K, K, D)
    for t in range(L):
        rm, ro, rb = oracle.bucketize(ref[:, t * K:(t + 1) * K])
        assert int(nb[t]) == len(ro) - 1, t
        assert np.array_equal(host_u32(mem[t]), rm), t
        assert np.array_equal(host_u32(boff[t])[:len(ro)], ro), t
        assert np.array_equal(host_u32(bof[t]), rb), t
