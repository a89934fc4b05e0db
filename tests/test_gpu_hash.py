"""GPU parity of geek_hash against the FP64 oracle: E2LSH codes bit for bit
(including pairs that land exactly on bucket edges), packed keys, MinHash
signatures of sets and heterogeneous rows, and the data-error paths."""

import math

import numpy as np
import pytest
import torch

import oracle
from workloads import dense_mixture, e2lsh_params, hetero_rows, key_words, sparse_sets

from .gpu_util import announce, cuda, gpu_api, host_u32, unpack_keys

pytestmark = pytest.mark.gpu


def _dense_case(api, X, A, b, m, L, w, name):
    announce(f"hash {name} n={len(X)} d={X.shape[1]} m={m} L={L} w={w}")
    ref = oracle.e2lsh_codes(X, A, b, w)
    nfix = torch.zeros(1, dtype=torch.int64, device="cuda")
    keys, codes = api.hash_dense(cuda(X), cuda(A), cuda(b), m, L, w, want_codes=True,
                                 n_fixup=nfix)
    got = codes.cpu().numpy().astype(np.int64)
    bad = np.argwhere(got != ref)
    assert bad.size == 0, (bad[:5], got[tuple(bad[0])], ref[tuple(bad[0])])
    assert np.array_equal(unpack_keys(host_u32(keys), m), ref)
    return int(nfix.item())


@pytest.mark.parametrize("n,d,m,L,w,seed", [
    (5000, 32, 8, 16, 4.0, 0),
    (5000, 32, 8, 16, 4.0 * math.sqrt(32), 0),
    (3001, 128, 10, 32, 8.0, 1),
    (2000, 20, 5, 4, 3.0, 2),
    (700, 256, 12, 3, 8.0 * math.sqrt(256), 3),
    (129, 64, 3, 7, 1.5, 4),
])
def test_e2lsh_codes_match_oracle(n, d, m, L, w, seed):
    api = gpu_api()
    X, _, _ = dense_mixture(n, d, 20, -10, 10, 1.0, "equal", seed)
    A, b = e2lsh_params(m * L, d, w, seed)
    _dense_case(api, X, A, b, m, L, w, "mixture")


def test_e2lsh_exact_bucket_edges_go_through_fixup():
    # integer data and projections: every a.x + b is an integer, so with
    # w = 1 (and w = 2) each quotient sits on or next to a bucket edge
    api = gpu_api()
    g = np.random.default_rng(9)
    X = g.integers(-8, 9, size=(1000, 16)).astype(np.float32)
    A = g.integers(-3, 4, size=(40, 16)).astype(np.float32)
    b = np.zeros(40, np.float32)
    nf = _dense_case(api, X, A, b, 8, 5, 1.0, "edges-w1")
    assert nf >= 1000 * 40 * 0.9
    b = (g.integers(0, 4, size=40) * 0.5).astype(np.float32)
    nf = _dense_case(api, X, A, b, 8, 5, 2.0, "edges-w2")
    assert nf > 0
    # values one float32 ulp away from an edge
    Xe = X + np.float32(2.0 ** -20) * g.choice([-1, 1], size=X.shape).astype(np.float32)
    _dense_case(api, Xe.astype(np.float32), A, np.zeros(40, np.float32), 8, 5, 1.0, "edges-ulp")


def test_e2lsh_large_quotients_take_float64():
    # rows scaled by 1e5 or 2e6 put |a.x + b| / w far above 2^21, where the
    # float32 quotient is no longer certified: every pair of such a row is
    # recomputed in float64; the other rows keep the fast path
    api = gpu_api()
    X, _, _ = dense_mixture(1500, 16, 10, -10, 10, 1.0, "equal", 5)
    X[::3] *= np.float32(1e5)
    X[1::6] *= np.float32(2e6)
    for m, L, w in ((2, 3, 1.0), (1, 5, 0.5), (4, 2, 7.0)):
        A, b = e2lsh_params(m * L, 16, w, 5)
        nf = _dense_case(api, X, A, b, m, L, w, "large-quotients")
        assert nf >= (len(X) // 6) * m * L


def test_e2lsh_errors_reported():
    api = gpu_api()
    from paper_2106_10515_amd import GeekError

    X, _, _ = dense_mixture(300, 8, 3, -10, 10, 1.0, "equal", 1)
    A, b = e2lsh_params(20, 8, 4.0, 1)
    Xn = X.copy()
    Xn[5, 3] = np.inf
    with pytest.raises(GeekError) as e:
        api.hash_dense(cuda(Xn), cuda(A), cuda(b), 10, 2, 4.0)
    assert e.value.code == 1
    # m = 10 leaves 12 bits per code: a tiny width overflows them
    with pytest.raises(GeekError) as e:
        api.hash_dense(cuda(X), cuda(A), cuda(b), 10, 2, 1e-3)
    assert e.value.code == 2
    # m = 4 leaves 32 bits per code, m = 5 25 bits
    A5, b5 = e2lsh_params(20, 8, 4.0, 1)
    with pytest.raises(GeekError) as e:
        api.hash_dense(cuda(X), cuda(A5), cuda(b5), 5, 4, 1e-6)
    assert e.value.code == 2


@pytest.mark.parametrize("F", [256, 64, 100])
def test_minhash_sets_match_oracle(F):
    api = gpu_api()
    off, tok, _ = sparse_sets(3000, vocab=50_000, clusters=40, seed=3)
    keys = key_words(F, 3)
    announce(f"minhash sets n={len(off) - 1} nnz={len(tok)} F={F}")
    ref = oracle.minhash_sets(off, tok, keys)
    sig = api.hash_sets(cuda(off), cuda(tok), cuda(keys))
    assert np.array_equal(host_u32(sig), ref)


def test_minhash_hetero_match_oracle():
    api = gpu_api()
    X, cat, _, _ = hetero_rows(2500, 20, 10, 50, seed=4)
    m, L, w = 20, 1, 4.0 * math.sqrt(20)
    A, b = e2lsh_params(m * L, 20, w, 4)
    keys = key_words(128, 4)
    announce("minhash hetero n=2500 F=128")
    codes = oracle.e2lsh_codes(X, A, b, w)
    tok = oracle.hetero_tokens(cat, codes)
    off = np.arange(0, tok.size + 1, tok.shape[1], dtype=np.int64)
    ref = oracle.minhash_sets(off, tok.reshape(-1), keys)
    sig = api.hash_hetero(cuda(X), cuda(cat), cuda(A), cuda(b), m, L, w, cuda(keys))
    assert np.array_equal(host_u32(sig), ref)
    # A as a transposed (non-contiguous) view gives the same signatures
    At = cuda(np.ascontiguousarray(A.T)).T
    assert not At.is_contiguous()
    sig = api.hash_hetero(cuda(X), cuda(cat), At, cuda(b), m, L, w, cuda(keys))
    assert np.array_equal(host_u32(sig), ref)


def test_minhash_empty_set_reported():
    api = gpu_api()
    from paper_2106_10515_amd import GeekError

    off = np.array([0, 2, 2, 5], np.int64)
    tok = np.array([1, 2, 3, 4, 5], np.uint32)
    with pytest.raises(GeekError) as e:
        api.hash_sets(cuda(off), cuda(tok), cuda(key_words(8, 0)))
    assert e.value.code == 5
