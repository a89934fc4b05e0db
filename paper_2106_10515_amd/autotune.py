"""Autotuner for the tile shapes of the batched assignment first pass.

A batched ``geek_assign`` call runs its first pass as one persistent launch
per padded depth (32, 64, 128, 256).  That launch can use several tile
shapes (``geek_set_scan_tiles``): ncb column blocks of 32 rows per wavefront,
nbuf LDS stages of seeds, and a number of persistent workgroups per compute
unit.  Every shape yields the same candidate records, so the shape only sets
the speed.  ``tune_batch_tiles`` times each compiled shape on a list of jobs
(the library's own event timer around the first pass) and installs the
fastest per (precision, padded depth); ``save_table`` writes the result as
JSON, and the binding installs ``tuned_tiles.json`` (beside the library)
whenever it loads the library.

Command line: ``python -m paper_2106_10515_amd.autotune [--out PATH]`` tunes
on synthetic Gaussian-mixture jobs of every padded depth (n log-uniform in
[1e3, 1e6], 10..5000 clusters) for BF16, FP8 and FP32 and saves the table.
"""

from __future__ import annotations

import json
import math
import os
import statistics
import warnings

from . import _lib as L

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_tiles.json")
PREC_NAMES = {L.GEEK_PREC_FP32: "fp32", L.GEEK_PREC_BF16: "bf16", L.GEEK_PREC_FP8: "fp8"}
PREC_BY_NAME = {v: k for k, v in PREC_NAMES.items()}
DEPTHS = (32, 64, 128, 256)
BLOCKS_PER_CU = (2, 4, 8, 16)


def padded_depth(d: int) -> int:
    """The matrix-core depth class of d attributes (the first pass pads d)."""
    for dp in DEPTHS:
        if d <= dp:
            return dp
    raise ValueError(f"d = {d} exceeds {DEPTHS[-1]}")


def candidates(precision: int, dp: int, blocks=BLOCKS_PER_CU):
    """Every (ncb, nbuf, blocks_per_cu) the library accepts for this class."""
    keep = L.geek_get_scan_tiles(precision, dp)
    out = []
    for ncb in (1, 2):
        for nbuf in (1, 2):
            for b in blocks:
                if L.geek_set_scan_tiles(precision, dp, ncb, nbuf, b) == L.GEEK_OK:
                    out.append((ncb, nbuf, b))
    L.geek_set_scan_tiles(precision, dp, *keep)
    return out


def tune_batch_tiles(problems, precision: int, reps: int = 3, blocks=BLOCKS_PER_CU, install: bool = True,
                     status=None):
    """Time every shape on ``problems`` (a list of ``(X, seed_offsets,
    seed_members, k)`` device tensors, as for ``api.assign_euclid_batch``),
    one padded depth at a time.  Returns ``{dp: {"best": shape, "ms": {shape:
    median first-pass milliseconds}}}`` and, with ``install``, leaves the
    fastest shape installed for each depth (else the previous one)."""
    from . import api

    groups = {}
    for p in problems:
        groups.setdefault(padded_depth(int(p[0].shape[1])), []).append(p)
    result = {}
    for dp, probs in sorted(groups.items()):
        if len(probs) < 2:  # a batched call needs two jobs at least
            probs = probs * 2
        keep = L.geek_get_scan_tiles(precision, dp)
        timings = {}
        for shape in candidates(precision, dp, blocks):
            L.geek_set_scan_tiles(precision, dp, *shape)
            api.assign_euclid_batch(probs, precision, status=status, check=False)  # warm-up
            ts = []
            for _ in range(reps):
                L.geek_profile(True)
                api.assign_euclid_batch(probs, precision, status=status, check=False)
                ms, _ = L.geek_profile_read(L.GEEK_PROF_ASSIGN_SCAN)
                ts.append(ms)
            L.geek_profile(False)
            timings[shape] = statistics.median(ts)
        best = min(timings, key=timings.get)
        L.geek_set_scan_tiles(precision, dp, *(best if install else keep))
        result[dp] = {"best": best, "ms": timings}
    if status is not None:
        api.check_status(status, "autotune")
    return result


def save_table(results, path: str = TABLE_PATH, note: str = "") -> None:
    """Write ``{precision: tune_batch_tiles(...) result}`` as the JSON table."""
    tiles, ms = {}, {}
    for prec, res in results.items():
        name = PREC_NAMES[prec]
        tiles[name] = {str(dp): list(r["best"]) for dp, r in res.items()}
        ms[name] = {str(dp): {"x".join(map(str, s)): round(t, 4) for s, t in r["ms"].items()}
                    for dp, r in res.items()}
    doc = {"library": L.version(), "note": note,
           "tiles": tiles, "first_pass_ms": ms,
           "shape": "[ncb, nbuf, blocks_per_cu] per precision and padded depth"}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
        f.write("\n")


def install_table(path: str = TABLE_PATH, missing_ok: bool = False) -> int:
    """Install the shapes of a saved table; returns how many were installed.
    Entries the library rejects are skipped with a warning."""
    if not os.path.exists(path):
        if missing_ok:
            return 0
        raise FileNotFoundError(path)
    with open(path) as f:
        doc = json.load(f)
    done = 0
    for name, per_dp in doc.get("tiles", {}).items():
        prec = PREC_BY_NAME.get(name)
        for dp, shape in per_dp.items():
            rc = L.geek_set_scan_tiles(prec if prec is not None else -1, int(dp), *[int(v) for v in shape])
            if rc == L.GEEK_OK:
                done += 1
            else:
                warnings.warn(f"tile table {path}: {name} dp={dp} {shape} rejected (status {rc})")
    return done


def synthetic_problems(device, seed: int = 0, jobs_per_depth: int = 8):
    """Gaussian-mixture jobs for every padded depth: n log-uniform in
    [1e3, 1e6], 10..5000 clusters (log-uniform), seeds = up to 32 members of
    each cluster."""
    import numpy as np
    import torch

    g = np.random.default_rng(seed)
    probs = []
    for d in (16, 64, 128, 256):
        for _ in range(jobs_per_depth):
            n = int(round(10 ** g.uniform(3.0, 6.0)))
            c = max(1, min(n // 2, int(round(10 ** g.uniform(1.0, math.log10(5000))))))
            centers = torch.from_numpy(g.uniform(-10, 10, (c, d)).astype(np.float32)).to(device)
            lab = torch.from_numpy(g.integers(0, c, n)).to(device)
            X = (centers[lab] + torch.randn(n, d, device=device)).contiguous()
            order = torch.argsort(lab, stable=True)
            counts = torch.bincount(lab, minlength=c)
            starts = torch.cumsum(counts, 0) - counts
            take = torch.clamp(counts, max=32)
            keep = torch.arange(n, device=device) - starts[lab[order]] < take[lab[order]]
            sm = order[keep].to(torch.int32)
            so = torch.zeros(c + 1, dtype=torch.int64, device=device)
            so[1:] = torch.cumsum(take, 0)
            nz = take > 0
            so = torch.cat([so[:1], so[1:][nz]]).to(torch.int32)
            probs.append((X, so, sm, int(nz.sum().item())))
    return probs


def main(argv=None) -> None:
    import argparse

    import torch

    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--precisions", default="bf16,fp8,fp32")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    probs = synthetic_problems(dev)
    results = {}
    for name in a.precisions.split(","):
        prec = PREC_BY_NAME[name]
        # start from the built-in defaults so every shape is measured afresh
        for dp in DEPTHS:
            L.geek_set_scan_tiles(prec, dp, 0, 0, 0)
        default = {dp: L.geek_get_scan_tiles(prec, dp) for dp in DEPTHS}
        results[prec] = tune_batch_tiles(probs, prec, reps=a.reps)
        for dp, r in results[prec].items():
            print(f"{name} dp={dp}: best {r['best']} {r['ms'][r['best']]:.3f} ms "
                  f"(default {default[dp]} {r['ms'].get(default[dp], float('nan')):.3f} ms)", flush=True)
    save_table(results, a.out, note="python -m paper_2106_10515_amd.autotune on synthetic mixtures")
    print(f"saved {a.out}", flush=True)


if __name__ == "__main__":
    main()
