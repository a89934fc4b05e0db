"""Pins of the oracle's SILK (Algorithm 4): the paper's worked example
(Examples 2 and 3) with explicit bins, a plain per-bin recount of the
vectorised voting, the singleton / threshold rules, and the independence of
the work from the number of clusters (Section 3.5)."""

import os

import numpy as np
import pytest

import oracle
from oracle.silk import _bins_of, _signatures, _vote_table
from workloads import dense_mixture, e2lsh_params, key_words
from workloads.gen import STREAM_SILK


def _load_example(golden_dir):
    buckets, bins, cs, seeds, t1 = {}, [], [], [], []
    delta = None
    with open(os.path.join(golden_dir, "silk_example2.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            if tok[0] == "bucket":
                buckets[tok[1]] = [int(v) for v in tok[2:]]
            elif tok[0] == "bins":
                bins.append([grp.split(",") for grp in tok[2:]])
            elif tok[0] == "delta":
                delta = int(tok[1])
            elif tok[0] == "cshared":
                cs.append([int(v) for v in tok[2:]])
            elif tok[0] == "seed":
                seeds.append([int(v) for v in tok[1:]])
            elif tok[0] == "seed_t1_only":
                t1.append([int(v) for v in tok[1:]])
    return buckets, bins, delta, cs, seeds, t1


def _dedup_bins_identical_only(C):
    # The example's de-duplication table: identical sets share a bin
    # (they always share every MinHash value); all other sets are alone.
    groups = {}
    for i, c in enumerate(C):
        groups.setdefault(tuple(int(v) for v in c), []).append(i)
    return list(groups.values())


def test_example2_reproduces_printed_seeds(golden_dir):
    buckets, bins, delta, cs, seeds, _ = _load_example(golden_dir)
    names = sorted(buckets, key=lambda s: int(s[1:]))
    sets = [np.array(buckets[nm]) for nm in names]
    idx = {nm: i for i, nm in enumerate(names)}
    table_bins = [[[idx[b] for b in grp] for grp in tb] for tb in bins]
    C, out = oracle.silk_from_bins(sets, table_bins, _dedup_bins_identical_only, delta)
    assert [c.tolist() for c in C] == cs
    assert sorted(s.tolist() for s in out) == sorted(seeds)


def test_example3_single_table(golden_dir):
    buckets, bins, delta, _, _, t1 = _load_example(golden_dir)
    names = sorted(buckets, key=lambda s: int(s[1:]))
    sets = [np.array(buckets[nm]) for nm in names]
    idx = {nm: i for i, nm in enumerate(names)}
    C, out = oracle.silk_from_bins(sets, [[[idx[b] for b in grp] for grp in bins[0]]],
                                   _dedup_bins_identical_only, delta)
    assert sorted(s.tolist() for s in out) == sorted(t1)


def test_majority_is_strict():
    assert oracle.majority([[1, 2], [2, 3]]).tolist() == [2]
    assert oracle.majority([[1, 2], [3, 4]]).tolist() == []
    assert oracle.majority([[1], [1], [2], [2]]).tolist() == []
    assert oracle.majority([[1], [1], [1], [2]]).tolist() == [1]


def _hashed_buckets(n=3000, d=16, clusters=12, m=6, L=8, seed=0):
    X, lab, _ = dense_mixture(n, d, clusters, -10, 10, 1.0, "equal", seed)
    w = 4.0 * np.sqrt(d)
    A, b = e2lsh_params(m * L, d, w, seed)
    codes = oracle.e2lsh_codes(X, A, b, w)
    offs, mem = [0], []
    for mm, oo, _ in oracle.bucketize_tables(codes, m, L):
        mem.append(mm)
        offs.extend((oo[1:].astype(np.int64) + offs[-1]).tolist())
    return np.asarray(offs, np.int64), np.concatenate(mem), X


def test_vectorised_vote_equals_per_bin_recount():
    offs, mem, _ = _hashed_buckets()
    K, L, delta = 3, 5, 3
    keys = key_words((L + 1) * K, 7, STREAM_SILK)
    sets = [mem[offs[i]:offs[i + 1]] for i in range(len(offs) - 1)]
    C_plain = []
    for i in range(L):
        G = _signatures(offs, mem, keys[i * K:(i + 1) * K])
        # brute-force binning: dictionary on the exact tuple
        table = {}
        for j in range(len(sets)):
            table.setdefault(tuple(int(v) for v in G[j]), []).append(j)
        C_plain.extend(_vote_table(sets, list(table.values()), delta))
    so, sm, info = oracle.silk_seeds(offs, mem, K, L, delta, keys)
    assert info["multiset"] == len(C_plain) > 0
    # de-duplicate the plain multiset the same way and compare the seeds
    c_off = np.concatenate([[0], np.cumsum([len(c) for c in C_plain])])
    Gc = _signatures(c_off, np.concatenate(C_plain), keys[L * K:(L + 1) * K])
    bins, _ = _bins_of(Gc)
    seeds = []
    for bn in bins:
        if len(bn) == 1:
            seeds.append(C_plain[bn[0]].tolist())
        else:
            cs = oracle.majority([C_plain[j] for j in bn])
            if len(cs) >= delta:
                seeds.append(cs.tolist())
    got = [sm[so[i]:so[i + 1]].tolist() for i in range(len(so) - 1)]
    assert got == seeds
    # invariants: every seed meets the threshold, members ascending, ordered
    # by the de-duplication tuple
    for s in got:
        assert len(s) >= delta and s == sorted(set(s))


def test_one_table_gives_no_seeds():
    # buckets of a single transform table are disjoint, so no id can be in
    # more than half of the buckets of any bin holding two or more of them
    X, _, _ = dense_mixture(500, 8, 5, -10, 10, 1.0, "equal", 1)
    A, b = e2lsh_params(4, 8, 8.0, 1)
    codes = oracle.e2lsh_codes(X, A, b, 8.0)
    mm, oo, _ = oracle.bucketize(codes)
    keys = key_words(6 * 1, 3, STREAM_SILK)
    so, sm, info = oracle.silk_seeds(oo, mm, 1, 5, 1, keys)
    assert len(so) == 1 and sm.size == 0


def test_work_independent_of_cluster_count():
    n, d, m, L = 2000, 8, 4, 6
    K, LS = 3, 4
    keys = key_words((LS + 1) * K, 2, STREAM_SILK)
    evals = set()
    for kp in (10, 100, 1000):
        X, _, _ = dense_mixture(n, d, kp, -10, 10, 1.0, "equal", 4)
        A, b = e2lsh_params(m * L, d, 4.0 * np.sqrt(d), 4)
        codes = oracle.e2lsh_codes(X, A, b, 4.0 * np.sqrt(d))
        offs, mem = [0], []
        for mm, oo, _ in oracle.bucketize_tables(codes, m, L):
            mem.append(mm)
            offs.extend((oo[1:].astype(np.int64) + offs[-1]).tolist())
        _, _, info = oracle.silk_seeds(np.asarray(offs), np.concatenate(mem), K, LS, 10, keys)
        evals.add(info["hash_evals"])
        assert info["pairs_voted"] <= LS * n * L
    assert evals == {K * LS * n * L}
