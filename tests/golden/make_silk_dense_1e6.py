"""Writes silk_dense_1e6.json: the oracle's SILK seeds for the benchmark's
SILK pass at 10^6 points, computed on the CPU by ``oracle/`` alone.

Workload: 10^6 points of the dense mixture (d = 128, 1,000 clusters with
Zipf(1.0) sizes, centres uniform in [-50, 50]^128, sigma = 1, seed 0, drawn
with numpy), E2LSH m = 10 x L = 32 tables at the scaled width 8 * sqrt(128),
SILK K = 3, L = 20, delta = 10 (Algorithm 4).  The seed CSR is stored as
SHA-256 digests of its little-endian uint32 arrays plus its sizes, the work
counters and a few whole seeds; the GPU test recomputes the digests from the
library's output.  Run from the repository root:
``python tests/golden/make_silk_dense_1e6.py`` (several minutes).
"""

import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import CONFIGS, dense_mixture, e2lsh_params, key_words  # noqa: E402
from workloads.gen import STREAM_SILK  # noqa: E402

N = 1_000_000


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


def main():
    cfg = CONFIGS["dense_large"]
    d, m, L = cfg["d"], cfg["m"], cfg["L"]
    w = cfg["w"] * math.sqrt(d)
    clusters = cfg["clusters"] * N // cfg["n"]
    K, LS, delta = cfg["K_S"], cfg["L_S"], cfg["delta"]
    t0 = time.time()
    X, _, _ = dense_mixture(N, d, clusters, cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"], seed=0)
    A, b = e2lsh_params(m * L, d, w, 0)
    codes = oracle.e2lsh_codes(X, A, b, w)
    print(f"codes {time.time() - t0:.0f}s", flush=True)
    offs, mem = [0], []
    for mm, oo, _ in oracle.bucketize_tables(codes, m, L):
        mem.append(mm)
        offs.extend((oo[1:].astype(np.int64) + offs[-1]).tolist())
    print(f"buckets {time.time() - t0:.0f}s", flush=True)
    keys = key_words((LS + 1) * K, 0, STREAM_SILK)
    so, sm, info = oracle.silk_seeds(np.asarray(offs), np.concatenate(mem), K, LS, delta, keys)
    print(f"silk {time.time() - t0:.0f}s k={len(so) - 1}", flush=True)
    sizes = np.diff(so.astype(np.int64))
    pick = [0, len(sizes) // 2, len(sizes) - 1]
    out = {
        "workload": f"dense mixture n={N} d={d} {clusters} clusters (Zipf sizes) seed 0 (numpy); "
                    f"E2LSH m={m} L={L} w=8*sqrt(128); SILK K={K} L={LS} delta={delta}",
        "n": N, "k": int(len(so) - 1), "members": int(len(sm)),
        "sha256_seed_offsets": digest(so), "sha256_seed_members": digest(sm),
        "buckets_total": int(len(offs) - 1),
        "hash_evals": int(info["hash_evals"]), "pairs_voted": int(info["pairs_voted"]),
        "multiset": int(info["multiset"]),
        "sample_seeds": {str(j): {"size": int(sizes[j]), "first": sm[so[j]:so[j + 1]][:64].astype(int).tolist()}
                         for j in pick},
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "silk_dense_1e6.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, out["k"], out["members"])


if __name__ == "__main__":
    main()
