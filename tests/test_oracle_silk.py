"""Pins of the oracle's SILK (Algorithm 4): the paper's worked example
(Examples 2 and 3) with explicit bins, bucket signatures against a brute-force
minimum, the seed order against hand-worked tuples, the whole pass against an
independent dictionary-and-counter version, the singleton / threshold rules,
and the independence of the counted work from the number of clusters
(Section 3.5)."""

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


def _pi(key, x):
    # one evaluation of the keyed permutation on one id
    return int(oracle.perm(key, np.array([x], dtype=np.uint32))[0])


def test_signatures_equal_brute_force_minimum():
    # G(B) per bucket, recomputed one id at a time, on a CSR with singleton
    # buckets, a large bucket and ids in no particular order
    rng = np.random.default_rng(11)
    sizes = [1, 3, 1, 40, 2, 1, 7, 1, 1, 15]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    mem = rng.permutation(5000)[: offs[-1]].astype(np.uint32)
    keys = key_words(3, 5, STREAM_SILK)
    tally = [0]
    G = _signatures(offs, mem, keys, tally)
    assert tally[0] == 3 * int(offs[-1])
    for j in range(len(sizes)):
        ids = mem[offs[j]:offs[j + 1]].tolist()
        for k in range(3):
            assert int(G[j, k]) == min(_pi(keys[k], x) for x in ids)


def test_bins_ordered_by_ascending_tuple_hand_worked():
    # rows 1 and 3 share (5, 2); rows 2 and 4 share (3, 7); the tuples tie in
    # word 0 and differ in word 1, so only a word-0-major order gives
    # (0,100) < (3,7) < (5,2) < (5,9)
    G = np.array([[5, 9], [5, 2], [3, 7], [5, 2], [3, 7], [0, 100]], dtype=np.uint32)
    bins, tup = _bins_of(G)
    assert bins == [[5], [2, 4], [1, 3], [0]]
    assert tup.tolist() == [[0, 100], [3, 7], [5, 2], [5, 9]]
    # three words: ties in words 0 and 1, decided by word 2
    G3 = np.array([[1, 1, 9], [1, 1, 2], [1, 0, 50], [1, 1, 2]], dtype=np.uint32)
    bins3, tup3 = _bins_of(G3)
    assert bins3 == [[2], [1, 3], [0]]
    assert tup3.tolist() == [[1, 0, 50], [1, 1, 2], [1, 1, 9]]


def _silk_by_dictionaries(sets, K, L, delta, keys):
    """Algorithm 4 written with dictionaries and counters, one id at a time:
    table s uses key rows s*K .. s*K+K-1 and the de-duplication table rows
    L*K .. L*K+K-1; seeds in ascending order of their de-duplication tuple."""
    from collections import Counter

    C = []
    for s in range(L):
        table = {}
        for j, B in enumerate(sets):
            g = tuple(min(_pi(keys[s * K + k], x) for x in B) for k in range(K))
            table.setdefault(g, []).append(j)
        for g in table:
            grp = table[g]
            if len(grp) < 2:
                continue
            cnt = Counter(x for j in grp for x in sets[j])
            shared = sorted(x for x, c in cnt.items() if 2 * c > len(grp))
            if len(shared) >= delta:
                C.append(shared)
    dedup = {}
    for i, c in enumerate(C):
        g = tuple(min(_pi(keys[L * K + k], x) for x in c) for k in range(K))
        dedup.setdefault(g, []).append(i)
    seeds, multi = [], 0
    for g in sorted(dedup):
        grp = dedup[g]
        if len(grp) == 1:
            seeds.append(C[grp[0]])
            continue
        multi += 1
        cnt = Counter(x for i in grp for x in C[i])
        shared = sorted(x for x, c in cnt.items() if 2 * c > len(grp))
        if len(shared) >= delta:
            seeds.append(shared)
    return C, seeds, multi


def test_silk_equals_dictionary_version():
    # pins the key rows of every table, the binning, the vote, the threshold,
    # the de-duplication and the seed order against an independent version
    offs, mem, _ = _hashed_buckets(n=700, d=12, clusters=6, m=5, L=6, seed=3)
    K, L, delta = 3, 4, 4
    keys = key_words((L + 1) * K, 9, STREAM_SILK)
    sets = [mem[offs[i]:offs[i + 1]].tolist() for i in range(len(offs) - 1)]
    C, seeds, multi = _silk_by_dictionaries(sets, K, L, delta, keys)
    assert len(seeds) >= 3 and multi >= 1  # the case exercises a voted de-duplication bin
    so, sm, info = oracle.silk_seeds(offs, mem, K, L, delta, keys)
    got = [sm[so[i]:so[i + 1]].tolist() for i in range(len(so) - 1)]
    assert got == seeds
    assert info["multiset"] == len(C)
    assert info["hash_evals"] == K * L * len(mem)
    assert info["hash_evals_dedup"] == K * sum(len(c) for c in C)


def test_silk_detects_swapped_key_rows():
    # the same buckets with the SILK tables' key rows in another order give
    # the same multiset C in another order, but a de-duplication table drawn
    # from another row changes the bins; the dictionary version follows the
    # documented rows, so a shifted row in the oracle would fail the test above
    offs, mem, _ = _hashed_buckets(n=700, d=12, clusters=6, m=5, L=6, seed=3)
    K, L, delta = 3, 4, 4
    keys = key_words((L + 1) * K, 9, STREAM_SILK)
    shifted = np.roll(keys, K, axis=0)
    a = oracle.silk_seeds(offs, mem, K, L, delta, keys)
    b = oracle.silk_seeds(offs, mem, K, L, delta, shifted)
    assert not (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]))


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
        # counted while computing: K evaluations per member of every bucket
        # of every transform table, whatever the number of clusters
        evals.add(info["hash_evals"])
        assert info["pairs_voted"] <= LS * n * L
    assert evals == {K * LS * n * L}
