"""GPU parity of geek_bucketize against the oracle's exact-tuple grouping:
members, offsets, bucket counts and bucket_of bit for bit, including bins too
large for LDS and MinHash band layouts."""

import math

import numpy as np
import pytest
import torch

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


def test_bucketize_two_streams_at_once():
    # the two halves of the tables bucketized on two streams at the same time
    # (each stream has its own cached workspace in the binding) equal one
    # call over all tables; entries of offsets past nbuckets are unspecified
    # and not compared
    import torch

    api = gpu_api()
    n, d, m, L = 200_000, 32, 8, 16
    X, _, _ = dense_mixture(n, d, 40, -10, 10, 1.0, "equal", 5)
    w = 4.0 * math.sqrt(d)
    A, b = e2lsh_params(m * L, d, w, 5)
    keys, _ = api.hash_dense(cuda(X), cuda(A), cuda(b), m, L, w)
    announce(f"bucketize two streams n={n} L={L}")
    ref = api.bucketize(keys, n, L, 4, n * 4, 4)
    torch.cuda.synchronize()
    h = L // 2
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    st1, st2 = api.new_status("cuda"), api.new_status("cuda")
    torch.cuda.synchronize()
    for rep in range(2):
        with torch.cuda.stream(s1):
            a = api.bucketize(keys[:h], n, h, 4, n * 4, 4, status=st1, check=False)
        with torch.cuda.stream(s2):
            bb = api.bucketize(keys[h:], n, L - h, 4, n * 4, 4, status=st2, check=False)
        torch.cuda.synchronize()
        assert int(st1.item()) == 0 and int(st2.item()) == 0
        for part, t0 in ((a, 0), (bb, h)):
            for t in range(part[0].shape[0]):
                nb = int(ref[2][t0 + t])
                assert int(part[2][t]) == nb, (rep, t0 + t)
                assert torch.equal(part[0][t], ref[0][t0 + t]), (rep, t0 + t)
                assert torch.equal(part[1][t, :nb + 1], ref[1][t0 + t, :nb + 1]), (rep, t0 + t)
                assert torch.equal(part[3][t], ref[3][t0 + t]), (rep, t0 + t)


def _fmix32(x):
    x = x & 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x85EBCA6B) & 0xFFFFFFFF
    x ^= x >> 13
    x = (x * 0xC2B2AE35) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def _bin_hash(words):
    # the library's bin selector (a 32-bit mix of the four key words, missing
    # words zero); test-side only, to aim keys at one bin
    h = 0x9E3779B9
    for i, w in enumerate(list(words) + [0] * (4 - len(words))):
        h = (_fmix32(h ^ int(w)) + 0x7F4A7C15 * (i + 1)) & 0xFFFFFFFF
    return _fmix32(h)


def test_bucketize_huge_buckets():
    # a few keys shared by tens of thousands of objects, among singletons
    api = gpu_api()
    g = np.random.default_rng(3)
    n = 300_000
    big = g.integers(0, 7, size=n).astype(np.uint32)
    single = g.random(n) < 0.1
    keys = np.stack([np.where(single, np.arange(n, dtype=np.uint32) + 100, big),
                     np.zeros(n, np.uint32)], axis=1)
    _compare(api, keys.reshape(-1), n, 1, 2, 0, 2, [keys], "huge buckets")


def test_bucketize_bin_beyond_the_table():
    # every key aimed at bin 0 (the top bits of the bin selector): more
    # distinct keys in one bin than the grouping table holds, some repeated
    api = gpu_api()
    n = 3600  # 4 bins of about 900 records each
    cand = []
    v = 1
    while len(cand) < 2600:
        if (_bin_hash([v, 7]) >> 30) == 0:
            cand.append(v)
        v += 1
    g = np.random.default_rng(4)
    pick = np.concatenate([np.arange(2600), g.integers(0, 2600, n - 2600)])
    g.shuffle(pick)
    k0 = np.asarray(cand, dtype=np.uint32)[pick]
    keys = np.stack([k0, np.full(n, 7, np.uint32)], axis=1)
    _compare(api, keys.reshape(-1), n, 1, 2, 0, 2, [keys], "one bin over the table")


def test_bucketize_large_bin_few_keys():
    # one bin far above the one-pass size holding three keys
    api = gpu_api()
    n = 20_000
    g = np.random.default_rng(5)
    k0 = g.choice(np.asarray([11, 12, 13], np.uint32), size=n)
    keys = np.stack([k0, k0 ^ 0x55AA55AA, np.arange(n, dtype=np.uint32) % 1], axis=1).astype(np.uint32)
    _compare(api, keys.reshape(-1), n, 1, 3, 0, 3, [keys], "large bin, three keys")


def _bin_hash_np(v, w1):
    # _bin_hash over keys [v, w1] for vectors v, w1 (uint64 arithmetic, masked)
    M = np.uint64(0xFFFFFFFF)

    def fm(x):
        x = x & M
        x ^= x >> np.uint64(16)
        x = (x * np.uint64(0x85EBCA6B)) & M
        x ^= x >> np.uint64(13)
        x = (x * np.uint64(0xC2B2AE35)) & M
        x ^= x >> np.uint64(16)
        return x

    h = np.full(v.shape, 0x9E3779B9, np.uint64)
    for i, wd in enumerate([v.astype(np.uint64), np.asarray(w1, np.uint64) + np.zeros(v.shape, np.uint64),
                            np.zeros(v.shape, np.uint64), np.zeros(v.shape, np.uint64)]):
        h = (fm(h ^ wd) + np.uint64(0x7F4A7C15 * (i + 1))) & M
    return fm(h).astype(np.uint32)


def test_bucketize_full_table_with_fingerprint_collision():
    # One bin on the general path (more than 2,048 records) whose third chunk
    # of 1,024 records overfills the 2,048-slot grouping table (the first two
    # chunks leave it at most 1,792 keys full, so the bin goes on), while one
    # of the third chunk's new keys shares the full 32-bit fingerprint with a
    # key already there: that record must give up (the bin is then split)
    # rather than keep walking the full table.
    # (with one word fixed the selector is a bijection of the other, so the
    # keys [v, v] are searched for a collision instead)
    api = gpu_api()
    v = np.arange(1, 1 << 20, dtype=np.uint32)
    f = _bin_hash_np(v, v)
    keep = (f >> 30) == 0                      # all in bin 0 of 4
    v, f = v[keep], f[keep]
    order = np.argsort(f, kind="stable")
    fs = f[order]
    dup = np.nonzero(fs[1:] == fs[:-1])[0]
    assert len(dup) > 0
    a_key, b_key = int(v[order[dup[0]]]), int(v[order[dup[0] + 1]])
    assert _bin_hash([a_key, a_key]) == _bin_hash([b_key, b_key]) and a_key != b_key
    rest = [int(x) for x in v[:5000] if int(x) not in (a_key, b_key)]
    g = np.random.default_rng(6)
    k1 = np.asarray([a_key] + rest[:999], np.uint32)            # 1,000 keys
    k2 = np.asarray(rest[999:999 + 792], np.uint32)             # 792 new keys
    k3 = np.asarray([b_key] + rest[1791:1791 + 1023], np.uint32)  # 1,024 new keys
    c1 = k1[np.concatenate([np.arange(1000), g.integers(0, 1000, 24)])]
    c2 = k2[np.concatenate([np.arange(792), g.integers(0, 792, 232)])]
    c3 = k3.copy()
    for c in (c1, c2, c3):
        g.shuffle(c)
    tail = k1[g.integers(0, 1000, 60)]
    k0 = np.concatenate([c1, c2, c3, tail]).astype(np.uint32)
    n = len(k0)
    keys = np.stack([k0, k0], axis=1)
    _compare(api, keys.reshape(-1), n, 1, 2, 0, 2, [keys], "full table, fingerprint collision")


@pytest.mark.parametrize("m", [8, 10])
def test_bucketize_with_the_hash_fingerprints(m):
    # geek_hash can write each key's bucketize fingerprint beside it; the
    # buckets formed from those fingerprints equal the ones formed from the
    # keys alone and the oracle's (m = 10 takes the compile-time packing,
    # other m the run-time one)
    api = gpu_api()
    n, d, L = 50_000, 32, 4
    X, _, _ = dense_mixture(n, d, 40, -10, 10, 1.0, "equal", 3)
    w = 4.0 * math.sqrt(d)
    A, b = e2lsh_params(m * L, d, w, 3)
    codes = oracle.e2lsh_codes(X, A, b, w)
    fp = torch.empty((L, n), dtype=torch.int32, device="cuda")
    keys, _ = api.hash_dense(cuda(X), cuda(A), cuda(b), m, L, w, key_fp=fp)
    kh, fh = host_u32(keys), host_u32(fp)
    g = np.random.default_rng(7)
    for t in range(L):
        for i in g.integers(0, n, 64):
            assert int(fh[t, i]) == _bin_hash([int(x) for x in kh[t, i]]), (t, i)
        # equal keys carry equal fingerprints
        _, inv = np.unique(kh[t], axis=0, return_inverse=True)
        inv = inv.ravel()
        first = np.full(inv.max() + 1, -1, np.int64)
        first[inv[::-1]] = np.arange(n)[::-1]
        assert np.array_equal(fh[t], fh[t][first[inv]]), t
    announce("bucketize with and without the hash's fingerprints")
    a = api.bucketize(keys, n, L, 4, n * 4, 4, key_fp=fp)
    c = api.bucketize(keys, n, L, 4, n * 4, 4)
    ma, oa, na, ba = (host_u32(x) for x in a)
    mc, oc, nc, bc = (host_u32(x) for x in c)
    for t in range(L):
        rm, ro, rb = oracle.bucketize(codes[:, t * m:(t + 1) * m])
        assert na[t] == nc[t] == len(ro) - 1
        assert np.array_equal(oa[t, :na[t] + 1], ro) and np.array_equal(oc[t, :nc[t] + 1], ro)
        assert np.array_equal(ma[t], rm) and np.array_equal(mc[t], rm)
        assert np.array_equal(ba[t], rb) and np.array_equal(bc[t], rb)
