"""GPU parity of geek_bucketize against the oracle's exact-tuple grouping:
members, offsets, bucket counts and bucket_of bit for bit, including bins too
large for LDS and MinHash band layouts."""

import math

import numpy as np
import pytest

import oracle
from workloads import dense_mixture, e2lsh_params

from .gpu_util import announce, cuda, gpu_api, host_u32

pytestmark = pytest.mark.gpu


def _compare(api, keys_np, n, T, kw, tstride, rstride, tuples_per_table, name):
    announce(f"bucketize {name} n={n} T={T} kw={kw}")
    mem, off, nb, bof = api.bucketize(cuda(keys_np), n, T, kw, tstride, rstride)
    mem, off, nb, bof = host_u32(mem), host_u32(off), host_u32(nb), host_u32(bof)
    for t in range(T):
        rm, ro, rb = oracle.bucketize(tuples_per_table[t])
        assert nb[t] == len(ro) - 1, (t, nb[t], len(ro) - 1)
        assert np.array_equal(off[t, :nb[t] + 1], ro), t
        assert np.array_equal(mem[t], rm), t
        assert np.array_equal(bof[t], rb), t


def test_bucketize_dense_keys_from_hash():
    api = gpu_api()
    n, d, m, L = 6000, 32, 8, 16
    X, _, _ = dense_mixture(n, d, 30, -10, 10, 1.0, "equal", 0)
    w = 4.0 * math.sqrt(d)
    A, b = e2lsh_params(m * L, d, w, 0)
    codes = oracle.e2lsh_codes(X, A, b, w)
    keys, _ = api.hash_dense(cuda(X), cuda(A), cuda(b), m, L, w)
    announce("bucketize dense from device keys")
    mem, off, nb, bof = api.bucketize(keys, n, L, 4, n * 4, 4)
    mem, off, nb, bof = host_u32(mem), host_u32(off), host_u32(nb), host_u32(bof)
    for t in range(L):
        rm, ro, rb = oracle.bucketize(codes[:, t * m:(t + 1) * m])
        assert nb[t] == len(ro) - 1
        assert np.array_equal(off[t, :nb[t] + 1], ro)
        assert np.array_equal(mem[t], rm)
        assert np.array_equal(bof[t], rb)


@pytest.mark.parametrize("n,T,kw,alpha,seed", [
    (20000, 3, 2, 3, 0),     # 9 distinct keys: every bin oversized
    (50000, 2, 4, 40, 1),    # many small buckets
    (1, 2, 1, 5, 2),
    (4097, 1, 3, 1000, 3),
    (30000, 2, 1, 3000, 5),  # groups of about 10: member-list ranks
    (30000, 2, 1, 300, 6),   # groups of about 100: in-LDS (slot, id) sort
    (300000, 1, 2, 600, 7),  # mostly buckets of one, some pairs; 256 bins
    (2000000, 2, 4, 1 << 20, 8),  # two partition passes, 2048 bins, 2 chunks per first-pass bin
    (600000, 2, 2, 700, 9),       # two passes, pairs and triples among singletons
    (400000, 1, 4, 3, 10),        # two passes, 81 distinct keys: every bin oversized
])
def test_bucketize_synthetic(n, T, kw, alpha, seed):
    api = gpu_api()
    g = np.random.default_rng(seed)
    keys = g.integers(0, alpha, size=(T, n, kw)).astype(np.uint32)
    _compare(api, keys, n, T, kw, n * kw, kw, [keys[t] for t in range(T)], "synthetic")


def test_bucketize_giant_bucket_plus_singletons():
    api = gpu_api()
    g = np.random.default_rng(4)
    n = 60000
    keys = g.integers(0, 2**32, size=(2, n, 4), dtype=np.uint64).astype(np.uint32)
    keys[0, ::2] = 7          # half of table 0 in one bucket
    keys[1, g.random(n) < 0.9] = [1, 2, 3, 4]
    _compare(api, keys, n, 2, 4, n * 4, 4, [keys[0], keys[1]], "giant")


def test_bucketize_minhash_band_layout():
    api = gpu_api()
    g = np.random.default_rng(5)
    n, K, Lb = 10000, 4, 8
    F = K * Lb
    sig = g.integers(0, 3, size=(n, F)).astype(np.uint32)
    tuples = [sig[:, b * K:(b + 1) * K] for b in range(Lb)]
    _compare(api, sig, n, Lb, K, K, F, tuples, "bands")
