#!/usr/bin/env python3
"""Benchmark of GEEK's data pass on one MI355X.

Metric: points/s of hash + bucketize + assign on the dense large workload
(n = 10,000,000 points, d = 128, a 10,000-cluster Gaussian mixture with Zipf
cluster sizes; E2LSH with m = 10 codes x L = 32 tables, w = 8), with the
assignment on the bfloat16 matrix cores (exact: every candidate within the
rigorous error window is re-evaluated in float64).  The float32 matrix-core
path is timed beside it on the same data.  SILK is not part of the metric's
region; the assignment uses k = 10,000 planted seeds (the first 32 members of
every planted cluster), because the literal hash width gives SILK almost
only singleton buckets.

One "step" = geek_hash + geek_bucketize + geek_assign over the whole input,
which is resident in HBM before timing starts.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_BF16 = 2500.0   # TFLOP/s, MI355X dense bf16 matrix
PEAK_FP32 = 157.3    # TFLOP/s, MI355X fp32 matrix
PEAK_HBM = 8000.0    # GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp32-steps", type=int, default=2)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--clusters", type=int, default=10_000)
    ap.add_argument("--cpu-rows", type=int, default=1024, help="oracle rows per CPU worker")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--pipeline", type=int, default=0,
                    help="dense: bucketize the first half of the tables on a second stream while the second "
                         "half is hashed (0 = hash, bucketize and assign one after another)")
    ap.add_argument("--scaled", action="store_true", help="w * sqrt(d) instead of w")
    ap.add_argument("--no-key-fp", action="store_true",
                    help="dense: bucketize fingerprints the keys itself instead of taking the hash's")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 2 GiB device copy (HBM counter calibration)")
    ap.add_argument("--workload", default="dense_large", choices=["dense_large", "batched", "hetero", "sets", "silk", "refine", "quantile"],
                    help="dense_large: the headline metric; batched: 256 mixed dense jobs in one "
                         "captured HIP graph; hetero: heterogeneous rows; sets: sparse sets "
                         "(MinHash, band buckets, signature assignment); silk: the whole GEEK pass "
                         "with SILK seeds on the dense mixture at the scaled width")
    ap.add_argument("--jobs", type=int, default=256, help="batched: number of jobs")
    ap.add_argument("--no-tune", action="store_true", help="batched: keep the installed tile shapes")
    ap.add_argument("--hetero-prec", default="fp8", choices=["fp8", "bf16"],
                    help="hetero: matrix-core type of the numeric part (the workload states FP8 e4m3)")
    ap.add_argument("--sets-hash", default="minhash", choices=["minhash", "doph"],
                    help="sets: F = K*L MinHash functions per set, or DOPH to --doph-dims coordinates "
                         "(bands and modes over the reduced rows)")
    ap.add_argument("--doph-dims", type=int, default=400, help="sets with DOPH: reduced dimension D")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "assign_scan_bf16_dense_large_pmc.txt")


def measured_traffic(kernel_prefix="k_scan<ModeBF16, 128, false, 2, 2, true, false>"):
    """HBM bytes per launch of the scan kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated against a plain
    copy), or None when there is no summary for the current kernel."""
    try:
        vals = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
        if vals.get("kernel", "").startswith(kernel_prefix) and vals.get("kernel_hash") == kernel_source_hash():
            return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        pass
    return None


def kernel_source_hash():
    """Hash of the sources the assignment scan kernel is built from (its
    tile loop and epilogues, and the shared helpers)."""
    import hashlib

    h = hashlib.sha256()
    for name in ("scan.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_2106_10515_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (the library has no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "hetero":
        return bench_hetero(args)
    if args.workload == "sets":
        return bench_sets(args)
    if args.workload == "silk":
        return bench_silk(args)
    if args.workload == "refine":
        return bench_refine(args)
    if args.workload == "quantile":
        return bench_quantile(args)
    import numpy as np
    import torch

    from paper_2106_10515_amd import _lib as L
    from paper_2106_10515_amd import api
    from workloads import CONFIGS, dense_mixture, e2lsh_params, planted_seeds

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cfg = CONFIGS["dense_large"]
    n, d, m, Lt = args.n, cfg["d"], cfg["m"], cfg["L"]
    w = cfg["w"] * (d ** 0.5 if args.scaled else 1.0)
    clusters = min(args.clusters, n)

    t0 = time.time()
    X, labels, _ = dense_mixture(n, d, clusters, cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"],
                                 seed=0, device=dev)
    A, b = e2lsh_params(m * Lt, d, w, 0)
    so, sm = planted_seeds(labels, clusters, 32)
    k = len(so) - 1
    Ag, bg = torch.from_numpy(A).to(dev), torch.from_numpy(b).to(dev)
    sog = torch.from_numpy(so.view(np.int32)).to(dev)
    smg = torch.from_numpy(sm.view(np.int32)).to(dev)
    torch.cuda.synchronize()
    log(f"workload ready n={n} d={d} k={k} in {time.time() - t0:.1f}s")

    status = api.new_status(dev)
    nfix = torch.zeros(1, dtype=torch.int64, device=dev)

    side = torch.cuda.Stream(device=dev)  # default priority
    half = Lt // 2

    def step(prec):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        if args.pipeline:
            # tables in two halves: the buckets of the first half are formed on
            # a second stream while the second half is hashed
            ka, _ = api.hash_dense(X, Ag[:half * m], bg[:half * m], m, half, w, status=status, check=False,
                                   n_fixup=nfix)
            ready = torch.cuda.Event()
            ready.record()
            side.wait_event(ready)
            with torch.cuda.stream(side):
                bza = api.bucketize(ka, n, half, 4, n * 4, 4, status=status, check=False)
            kb, _ = api.hash_dense(X, Ag[half * m:], bg[half * m:], m, Lt - half, w, status=status, check=False,
                                   n_fixup=nfix)
            ev[1].record()
            bzb = api.bucketize(kb, n, Lt - half, 4, n * 4, 4, status=status, check=False)
            done = torch.cuda.Event()
            done.record(side)
            torch.cuda.current_stream().wait_event(done)
            buckets = (bza, bzb)
        else:
            # the hash writes each key's bucketize fingerprint beside it, so
            # bucketize does not read the keys back to fingerprint them
            fp = torch.empty((Lt, n), dtype=torch.int32, device=dev) if not args.no_key_fp else None
            keys, _ = api.hash_dense(X, Ag, bg, m, Lt, w, status=status, check=False, n_fixup=nfix, key_fp=fp)
            ev[1].record()
            buckets = api.bucketize(keys, n, Lt, 4, n * 4, 4, status=status, check=False, key_fp=fp)
        ev[2].record()
        out = api.assign_euclid(X, sog, smg, k, prec, status=status, check=False)
        ev[3].record()
        return ev, out, buckets

    def run(prec, steps, warmup, profile=False):
        for _ in range(warmup):
            step(prec)
        torch.cuda.synchronize()
        api.check_status(status, "warmup")
        if profile:
            L.geek_profile(True)
        stage = np.zeros(3)
        torch.cuda.synchronize()
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        t_start.record()
        evs = []
        out = None
        for _ in range(steps):
            ev, out, _ = step(prec)
            evs.append(ev)
        t_end.record()
        torch.cuda.synchronize()
        api.check_status(status, "timed steps")
        total = t_start.elapsed_time(t_end)
        for ev in evs:
            stage += [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
        prof = {}
        if profile:
            for name, kid in (("assign_scan", L.GEEK_PROF_ASSIGN_SCAN), ("e2lsh", L.GEEK_PROF_E2LSH),
                              ("bucketize", L.GEEK_PROF_BUCKETIZE), ("assign", L.GEEK_PROF_ASSIGN),
                              ("bz_sort", L.GEEK_PROF_BZ_SORT)):
                ms, cnt = L.geek_profile_read(kid)
                prof[name] = (ms / max(cnt, 1), cnt)
            L.geek_profile(False)
        return total / steps, stage / steps, out, prof

    if args.copy_calibration:
        src = torch.empty(1 << 29, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1.0)
        torch.cuda.synchronize()
        dst.copy_(src)  # 2 GiB read + 2 GiB written
        torch.cuda.synchronize()
        del src, dst
    ms_bf16, st_bf16, out_bf16, prof_bf16 = run(L.GEEK_PREC_BF16, args.steps, args.warmup, True)
    log(f"bf16 path {ms_bf16:.2f} ms/step stages {np.round(st_bf16, 2)}")
    ctr_bf16 = out_bf16["counters"].cpu().numpy().tolist()
    a_bf16 = out_bf16["assign"]
    sse_bf16 = float(out_bf16["sse"].item())
    flops = 2.0 * n * d * k
    scan_ms = prof_bf16["assign_scan"][0]
    ach = flops / (scan_ms * 1e-3) / 1e12
    fp32 = None  # the float32 path for comparison (--fp32-steps 0 skips it)
    same = None
    if args.fp32_steps > 0:
        ms_fp32, st_fp32, out_fp32, prof_fp32 = run(L.GEEK_PREC_FP32, args.fp32_steps, 1, True)
        log(f"fp32 path {ms_fp32:.2f} ms/step stages {np.round(st_fp32, 2)}")
        same = bool(torch.equal(a_bf16, out_fp32["assign"])) and sse_bf16 == float(out_fp32["sse"].item())
        scan32_ms = prof_fp32["assign_scan"][0]
        ach32 = flops / (scan32_ms * 1e-3) / 1e12
        fp32 = (ms_fp32, st_fp32, scan32_ms, ach32)
    # per step: launch average x launches per step (two each when pipelined);
    # the rates use each kernel's own busy time (overlapped work counted once)
    hash_ms = prof_bf16["e2lsh"][0] * prof_bf16["e2lsh"][1] / args.steps
    hash_tf = 2.0 * n * d * m * Lt / (hash_ms * 1e-3) / 1e12
    bz_ms = prof_bf16["bucketize"][0] * prof_bf16["bucketize"][1] / args.steps
    # per (table, object): the 16-byte key read (or a 4-byte fingerprint
    # when the hash wrote them) + members, bucket_of and offsets written
    bz_gbs = (16.0 if args.no_key_fp or args.pipeline else 4.0) + 12.0
    bz_gbs = bz_gbs * n * Lt / (bz_ms * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(X, A, b, w, m, Lt, so, sm, a_bf16, out_bf16["dist"], args.cpu_rows, n, log)

    stage_names = (("hash (bucketize of the first half overlapped)", "bucketize (second half)", "assign")
                   if args.pipeline else ("hash", "bucketize", "assign"))
    value = n / (ms_bf16 * 1e-3)
    res = {
        "metric": "points/s (hash+bucketize+assign), d=128 k≈1e4: BF16-MFMA vs FP32 path",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_bf16,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"dense_large: n={n} d={d} {clusters}-cluster Gaussian mixture "
                               f"(Zipf sizes), E2LSH m={m} L={Lt} w={w:g}, k={k} planted seeds",
                   "n": n, "d": d, "k": k, "m": m, "L": Lt, "w": w, "seeds": "planted"},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16, "unit": "TFLOP/s",
                     "frac": ach / PEAK_BF16, "traffic": measured_traffic(),
                     "kernel": "k_scan<ModeBF16,128>", "avg_launch_ms": scan_ms,
                     "flop_per_launch": flops},
        "fp32_path": None if fp32 is None else {
            "value": n / (fp32[0] * 1e-3), "ms_per_step": fp32[0],
            "stages_ms": dict(zip(stage_names, fp32[1].round(3).tolist())),
            "scan_ms": fp32[2], "scan_tflops": fp32[3], "scan_frac": fp32[3] / PEAK_FP32},
        "speedup_bf16_over_fp32": None if fp32 is None else fp32[0] / ms_bf16,
        "stages_ms": dict(zip(stage_names, st_bf16.round(3).tolist())),
        "pipelined_tables": bool(args.pipeline),
        "kernels": {"e2lsh_ms": hash_ms, "e2lsh_tflops": hash_tf, "e2lsh_frac_fp32": hash_tf / PEAK_FP32,
                    "bucketize_ms": bz_ms, "bucketize_gbs_algorithmic": bz_gbs,
                    "bz_sort_ms": prof_bf16["bz_sort"][0]},
        "assign_counters": {"first_pass_rows": ctr_bf16[0], "rescanned_fp32": ctr_bf16[1],
                            "full_fp64_rows": ctr_bf16[2], "fp64_candidate_evals": ctr_bf16[3]},
        "bf16_equals_fp32": same,
        "sse": sse_bf16,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))


_CPU_CTX = {}


def _cpu_init(path):
    """Pool initializer: the sample's shared inputs (projections, centroids)."""
    import numpy as np

    with np.load(path) as z:
        _CPU_CTX.update({k: z[k] for k in z.files})


def _cpu_task(Xs):
    """One worker's share of the oracle run: E2LSH codes and buckets of its
    rows, then their assignment to all centroids (float64, one thread)."""
    import numpy as np

    import oracle

    c = _CPU_CTX
    t0 = time.perf_counter()
    codes = oracle.e2lsh_codes(Xs, c["A"], c["b"], float(c["w"]))
    oracle.bucketize_tables(codes, int(c["m"]), int(c["L"]))
    a, dist = oracle.assign_euclid(Xs, c["C"])
    return a, dist, time.perf_counter() - t0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, A, b, w, m, Lt, so, sm, a_gpu, d_gpu, rows, n, log):
    """The FP64 oracle on a bounded sample of the same workload, timed on the
    host's cores: one worker process on ``rows`` points, then one worker per
    core of the process's CPU share (at most 16) on ``rows`` points each,
    started together; every worker hashes, buckets and assigns its own rows
    against all k centroids (the centroid cost, measured once, is prorated to
    the sample).  The oracle's arithmetic is unchanged; rows are split across
    processes."""
    import multiprocessing as mp
    import tempfile

    import numpy as np

    import oracle

    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    P = max(1, min(16, share))
    Xh = X[:rows * (P + 1)].cpu().numpy()
    mem_rows = X[np.asarray(sm, dtype=np.int64)].cpu().numpy()
    t0 = time.perf_counter()
    C = oracle.centroids(mem_rows, so.astype(np.int64), np.arange(len(sm), dtype=np.uint32))
    t_c = time.perf_counter() - t0
    fd, path = tempfile.mkstemp(suffix=".npz", dir="/tmp")
    os.close(fd)
    np.savez(path, A=A, b=b, w=np.float64(w), m=np.int64(m), L=np.int64(Lt), C=C)
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(P, initializer=_cpu_init, initargs=(path,)) as pool:
            pool.map(_cpu_task, [Xh[:8]] * P)  # workers started and warm
            t0 = time.perf_counter()
            one = pool.map(_cpu_task, [Xh[:rows]])
            t_one = time.perf_counter() - t0
            parts = [Xh[rows * (q + 1):rows * (q + 2)] for q in range(P)]
            t0 = time.perf_counter()
            res = pool.map(_cpu_task, parts, chunksize=1)
            t_all = time.perf_counter() - t0
    finally:
        os.unlink(path)
    a_all = np.concatenate([one[0][0]] + [r[0] for r in res])
    d_all = np.concatenate([one[0][1]] + [r[1] for r in res])
    agree = bool(np.array_equal(a_all, a_gpu[:rows * (P + 1)].cpu().numpy()))
    d_ref = d_gpu[:rows * (P + 1)].cpu().numpy()
    sse_rel = abs(float(d_ref.sum()) - float(d_all.sum())) / max(float(d_all.sum()), 1e-300)
    per_pt_c = t_c / n
    v1 = rows / (t_one + per_pt_c * rows)
    vP = rows * P / (t_all + per_pt_c * rows * P)
    log(f"cpu oracle: 1 core {rows} rows {t_one:.1f}s; {P} cores {rows * P} rows {t_all:.1f}s; "
        f"centroids {t_c:.1f}s")
    return {"value": vP, "unit": "points/s", "cores": P, "kind": "oracle",
            "sample": f"{rows} points per worker process (points {rows} .. {rows * (P + 1) - 1} of {n}), "
                      f"{P} workers started together, each hashing, bucketing and assigning its rows to all "
                      f"{len(so) - 1} centroids in numpy float64 (one thread each); centroid time prorated "
                      f"by sample size / n",
            "single_core": {"value": v1, "rows": rows, "seconds": t_one},
            "seconds": t_all, "host": {"cpu_share": share, "nproc": os.cpu_count(), "model": _cpu_model()},
            "sample_assign_matches_gpu": agree, "sample_sse_rel_err_vs_oracle": sse_rel}


def _timed_graph(step, steps, warmup):
    """Capture ``step`` in a HIP graph (after one eager warm-up call) and time
    ``steps`` replays; returns (ms per replay, graph outputs)."""
    import torch

    step(True)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step(False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        out = step(False)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps, out


def _oracle_euclid_sample(jobs, rows_per_job):
    """The oracle (numpy float64, one thread) on sampled rows of dense jobs
    already assigned on the GPU: for each (X, seed_offsets, seed_members,
    gpu_out) it computes every centroid, then assigns the first rows to all
    of them.  Returns the cpu_baseline object: points/s with the centroid
    time prorated by sample / n, whether the sampled assignments equal the
    GPU's, and the sampled SSE's relative error against the oracle."""
    import numpy as np

    import oracle

    t_tot, rows_tot, agree, s_gpu, s_ref = 0.0, 0, True, 0.0, 0.0
    for X, so, sm, out in jobs:
        Xh = X.cpu().numpy()
        soh, smh = so.cpu().numpy().view(np.uint32), sm.cpu().numpy().view(np.uint32)
        n = Xh.shape[0]
        rows = min(rows_per_job, n)
        t0 = time.perf_counter()
        C = oracle.centroids(Xh, soh, smh)
        t_c = time.perf_counter() - t0
        t0 = time.perf_counter()
        a_ref, d_ref = oracle.assign_euclid(Xh[:rows], C)
        t_a = time.perf_counter() - t0
        t_tot += t_a + t_c * rows / n
        rows_tot += rows
        agree = agree and bool(np.array_equal(a_ref, out["assign"][:rows].cpu().numpy()))
        s_gpu += float(out["dist"][:rows].double().sum())
        s_ref += float(d_ref.sum())
    return {"value": rows_tot / t_tot, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"first {rows_per_job} rows of each of {len(jobs)} job(s) assigned to all of the job's "
                      "seeds (numpy float64, one thread; centroid time prorated by sample / n); hashing, "
                      "bucketing and seeding not included",
            "sample_assign_matches_gpu": agree,
            "sample_sse_rel_err_vs_oracle": abs(s_gpu - s_ref) / max(s_ref, 1e-300)}


def bench_batched(args):
    """Many independent dense jobs (n log-uniform in [1e3, 1e6], d over
    {16, 32, 64, 128, 256}, 10..5000 planted clusters): one geek_hash, one
    geek_bucketize and one batched geek_assign call over all jobs, captured
    in one HIP graph and replayed."""
    import numpy as np
    import torch

    from paper_2106_10515_amd import _lib as L
    from paper_2106_10515_amd import api
    from workloads import CONFIGS, batched_jobs, dense_mixture, e2lsh_params, planted_seeds

    dev = torch.device("cuda:0")
    hc = CONFIGS["dense_small"]  # the small dense configuration's hash parameters
    m, Lt, w = hc["m"], hc["L"], hc["w"]
    specs = batched_jobs(args.jobs, seed=0)
    t0 = time.time()
    probs, hp, total_n = [], {}, 0
    for sp in specs:
        X, lab, _ = dense_mixture(sp["n"], sp["d"], sp["clusters"], sp["lo"], sp["hi"], sp["sigma"],
                                  sp["sizes"], sp["seed"], device=dev)
        so, sm = planted_seeds(lab, sp["clusters"], 32)
        if sp["d"] not in hp:
            A, b = e2lsh_params(m * Lt, sp["d"], w, 0)
            hp[sp["d"]] = (torch.from_numpy(A).to(dev), torch.from_numpy(b).to(dev))
        probs.append((X, torch.from_numpy(so.view(np.int32)).to(dev),
                      torch.from_numpy(sm.view(np.int32)).to(dev), len(so) - 1))
        total_n += sp["n"]
    torch.cuda.synchronize()
    log(f"batched workload ready: {len(specs)} jobs, sum n = {total_n} in {time.time() - t0:.1f}s")
    status = api.new_status(dev)
    # tile shapes of the batched first pass: measured on these jobs (untimed)
    tiles = None
    if not args.no_tune:
        from paper_2106_10515_amd import autotune

        t0 = time.time()
        tuned = autotune.tune_batch_tiles(probs, L.GEEK_PREC_BF16, reps=2, status=status)
        tiles = {str(dp): {"shape": list(r["best"]), "first_pass_ms": round(r["ms"][r["best"]], 4),
                           "shapes_timed": len(r["ms"])} for dp, r in tuned.items()}
        log(f"autotuned tile shapes in {time.time() - t0:.1f}s: {tiles}")

    def step(check):
        keys = api.hash_dense_batch([(X, *hp[X.shape[1]], m, Lt, w) for X, _, _, _ in probs],
                                    status=status, check=check)
        bz = api.bucketize_batch([(kk, X.shape[0], Lt, 4, X.shape[0] * 4, 4) for kk, (X, _, _, _)
                                  in zip(keys, probs)], status=status, check=check)
        outs, t_done = api.assign_euclid_batch(probs, L.GEEK_PREC_BF16, status=status, check=check)
        return keys, bz, outs, t_done

    ms, (keys, bz, outs, t_done) = _timed_graph(step, args.steps, args.warmup)
    api.check_status(status, "graph replays")
    hz = api.wallclock_hz()
    lat_ms = t_done.cpu().numpy().astype(np.float64) / hz * 1e3
    # the same jobs one call per job (eager), for comparison
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    singles = [api.assign_euclid(X, so, sm, k, L.GEEK_PREC_BF16, status=status, check=False)
               for X, so, sm, k in probs]
    e1.record()
    torch.cuda.synchronize()
    single_ms = e0.elapsed_time(e1)
    same = all(np.array_equal(a["assign"].cpu().numpy(), b["assign"].cpu().numpy())
               for a, b in zip(outs, singles))
    flops = float(sum(2.0 * X.shape[0] * X.shape[1] * k for X, _, _, k in probs))
    line = {
        "metric": "points/s (hash+bucketize+assign), 256 mixed dense jobs in one HIP graph",
        "value": total_n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"batched: {len(specs)} jobs, n log-uniform in [1e3, 1e6] (sum {total_n}), "
                               "d in {16,32,64,128,256}, 10..5000 planted clusters, E2LSH m=8 L=16 w=4",
                   "jobs": len(specs), "sum_n": total_n},
        "assign_job_latency_ms": {"p50": float(np.percentile(lat_ms, 50)),
                                  "p99": float(np.percentile(lat_ms, 99)),
                                  "max": float(lat_ms.max())},
        "tiles": tiles,
        "assign_flops": flops,
        "assign_one_call_per_job_ms": single_ms,
        "batched_equals_single_calls": bool(same),
    }
    line["cpu_baseline"] = _oracle_euclid_sample(
        [(X, so, sm, o) for (X, so, sm, _), o in list(zip(probs, outs))[:4]], 128)
    if tiles:
        # the persistent first pass of every padded depth, timed by the
        # autotuner with its chosen shape: 2 n d k flops per job
        fp_ms = sum(v["first_pass_ms"] for v in tiles.values())
        ach = flops / (fp_ms * 1e-3) / 1e12
        line["roofline"] = {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16, "unit": "TFLOP/s",
                            "frac": ach / PEAK_BF16, "traffic": None,
                            "kernel": "k_scan_batch (persistent BF16 first pass, one launch per padded depth)",
                            "avg_launch_ms": fp_ms, "flop_per_launch": flops}
    print(json.dumps(line), flush=True)


def bench_hetero(args):
    """Heterogeneous rows (2e6 rows, 20 numeric + 10 categorical attributes,
    1000 clusters): MinHash of the combined tokens, bucketize of the bands,
    heterogeneous assignment with the BF16 (or FP8) numeric part."""
    import numpy as np
    import torch

    from paper_2106_10515_amd import _lib as L
    from paper_2106_10515_amd import api
    from workloads import CONFIGS, e2lsh_params, hetero_rows, key_words, planted_seeds
    from workloads.gen import STREAM_MINHASH

    dev = torch.device("cuda:0")
    cfg = CONFIGS["hetero"]
    n = cfg["n"]
    t0 = time.time()
    X, cat, lab, _ = hetero_rows(n, cfg["d_num"], cfg["n_cat"], cfg["clusters"], seed=0)
    A, b = e2lsh_params(cfg["P_h"], cfg["d_num"], cfg["w"], 0)
    K, Lb = cfg["K"], cfg["L"]
    mh = key_words(K * Lb, 0, STREAM_MINHASH)
    so, sm = planted_seeds(lab, cfg["clusters"], 32)
    Xg, catg = torch.from_numpy(X).to(dev), torch.from_numpy(cat).to(dev)
    Ag, bg = torch.from_numpy(A).to(dev), torch.from_numpy(b).to(dev)
    mhg = torch.from_numpy(mh.view(np.int32)).to(dev)
    sog, smg = torch.from_numpy(so.view(np.int32)).to(dev), torch.from_numpy(sm.view(np.int32)).to(dev)
    k = len(so) - 1
    torch.cuda.synchronize()
    log(f"hetero workload ready n={n} k={k} in {time.time() - t0:.1f}s")
    status = api.new_status(dev)
    fp8 = args.hetero_prec == "fp8"
    prec = L.GEEK_PREC_FP8 if fp8 else L.GEEK_PREC_BF16

    def step(check):
        sig = api.hash_hetero(Xg, catg, Ag, bg, cfg["P_h"], 1, cfg["w"], mhg, status=status, check=check)
        bz = api.bucketize(sig, n, Lb, K, K, K * Lb, status=status, check=check)
        out = api.assign_hetero(Xg, catg, sog, smg, k, 1.0, prec, status=status, check=check)
        return sig, bz, out

    ms, (sig, bz, out) = _timed_graph(step, args.steps, args.warmup)
    api.check_status(status, "graph replays")
    # stage times (eager, events) and the scan kernel's launch time
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    L.geek_profile(True)
    ev[0].record()
    sig2 = api.hash_hetero(Xg, catg, Ag, bg, cfg["P_h"], 1, cfg["w"], mhg, status=status, check=False)
    ev[1].record()
    api.bucketize(sig2, n, Lb, K, K, K * Lb, status=status, check=False)
    ev[2].record()
    out2 = api.assign_hetero(Xg, catg, sog, smg, k, 1.0, prec, status=status, check=False)
    ev[3].record()
    torch.cuda.synchronize()
    scan_ms, scan_n = L.geek_profile_read(L.GEEK_PROF_ASSIGN_SCAN)
    L.geek_profile(False)
    api.check_status(status, "stage runs")
    stages = [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    d_num = cfg["d_num"]
    flops = 2.0 * n * d_num * k
    peak = 5000.0 if fp8 else PEAK_BF16
    ach = flops / (scan_ms / max(scan_n, 1) * 1e-3) / 1e12
    # oracle on a bounded sample: the assignment of the first rows to every
    # seed's centroid and mode, one thread
    import oracle

    rows = min(512, n)
    t0 = time.perf_counter()
    Cn = oracle.centroids(X, so, sm)
    Mc = oracle.modes(cat, so, sm)
    t_c = time.perf_counter() - t0
    t0 = time.perf_counter()
    a_ref, d_ref = oracle.assign_hetero(X[:rows], cat[:rows], Cn, Mc, 1.0)
    t_a = time.perf_counter() - t0
    a_gpu = out2["assign"][:rows].cpu().numpy()
    d_gpu = out2["dist"][:rows].cpu().numpy()
    line = {
        "metric": "points/s (hash+bucketize+assign), heterogeneous rows",
        "value": n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp8" if fp8 else "bf16", "data": "synthetic",
        "config": {"workload": f"hetero: n={n}, 20 numeric + 10 categorical attributes, "
                               f"{cfg['clusters']} clusters, MinHash K={K} x L={Lb}, k={k} planted seeds",
                   "n": n, "k": k},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                     "traffic": None, "kernel": "k_scan (heterogeneous first pass)",
                     "avg_launch_ms": scan_ms / max(scan_n, 1), "flop_per_launch": flops,
                     "note": "d = 20 numeric attributes pad to the 64-deep FP8 (32-deep BF16) matrix step and "
                             "every (row, seed) pair also counts 10 categorical mismatches on the VALU"},
        "stages_ms": {"hash": stages[0], "bucketize": stages[1], "assign": stages[2]},
        "assign_counters": out2["counters"].cpu().numpy().tolist(),
        "cpu_baseline": {"value": rows / (t_a + t_c * rows / n), "unit": "points/s", "cores": 1,
                         "kind": "oracle",
                         "sample": f"first {rows} of {n} rows assigned to all {k} seeds (numpy float64, one "
                                   "thread; centroid and mode time prorated by rows / n); hashing not included",
                         "sample_assign_matches_gpu": bool(np.array_equal(a_ref, a_gpu)),
                         "sample_sse_rel_err_vs_oracle": abs(float(d_gpu.sum()) - float(d_ref.sum()))
                         / max(float(d_ref.sum()), 1e-300)},
    }
    print(json.dumps(line), flush=True)


def bench_sets(args):
    """Sparse sets (5e6 sets over a 1e6-token vocabulary, 2000 planted
    clusters): MinHash signatures (K=4 x L=64 = 256 functions), buckets of
    the 64 bands, and assignment of the signatures to the modes of the
    planted seeds."""
    import numpy as np
    import torch

    from paper_2106_10515_amd import api
    from workloads import CONFIGS, key_words, planted_seeds, sparse_sets
    from workloads.gen import STREAM_MINHASH

    dev = torch.device("cuda:0")
    cfg = CONFIGS["sets"]
    n = cfg["n"] if args.n == 10_000_000 else args.n
    K, Lb = cfg["K"], cfg["L"]
    doph = args.sets_hash == "doph"
    F = args.doph_dims if doph else K * Lb
    assert F >= K * Lb, "the bands need K*L coordinates"
    t0 = time.time()
    off, tok, lab = sparse_sets(n, cfg["vocab"], cfg["clusters"], seed=0, device=dev)
    mh = torch.from_numpy(key_words(1 if doph else K * Lb, 0, STREAM_MINHASH).view(np.int32)).to(dev)

    def hash_fn(check):
        if doph:
            return api.hash_doph(off, tok, mh, F, status=status, check=check)
        return api.hash_sets(off, tok, mh, status=status, check=check)
    so, sm = planted_seeds(lab, cfg["clusters"], 32)
    sog, smg = torch.from_numpy(so.view(np.int32)).to(dev), torch.from_numpy(sm.view(np.int32)).to(dev)
    k = len(so) - 1
    nnz = int(off[-1].item())
    torch.cuda.synchronize()
    log(f"sets workload ready n={n} nnz={nnz} k={k} in {time.time() - t0:.1f}s")
    status = api.new_status(dev)

    def step(check):
        sig = hash_fn(check)
        bz = api.bucketize(sig, n, Lb, K, K, F, status=status, check=check)
        out = api.assign_sig(sig, sog, smg, k, status=status, check=check)
        return sig, bz, out

    ms, (sig, bz, out) = _timed_graph(step, args.steps, args.warmup)
    api.check_status(status, "graph replays")
    # stage times (eager, events; the hash and the assignment over a few
    # launches each)
    reps = 5
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    ev[0].record()
    for _ in range(reps):
        sig2 = hash_fn(False)
    ev[1].record()
    api.bucketize(sig2, n, Lb, K, K, F, status=status, check=False)
    ev[2].record()
    ev[3].record()
    for _ in range(2):
        api.assign_sig(sig2, sog, smg, k, status=status, check=False)
    ev[4].record()
    torch.cuda.synchronize()
    t_hash = ev[0].elapsed_time(ev[1]) / reps
    t_bz = ev[1].elapsed_time(ev[2])
    t_as = ev[3].elapsed_time(ev[4]) / 2
    api.check_status(status, "stage runs")
    # roofline of the dominant kernel, the signature assignment: one exact
    # 32-bit compare-and-count per (set, seed, coordinate), two VALU lane
    # operations each, against the chip's integer VALU rate
    peak_alu = 256 * 64 * 2.4e9 / 2 / 1e12  # Tcompares/s
    compares = float(n) * k * F
    hash_bytes = nnz * 4 + (n + 1) * 8 + n * F * 4  # tokens + offsets read, rows written
    name = f"DOPH D={F}" if doph else f"MinHash K={K} x L={Lb}"
    line = {
        "metric": f"sets/s ({'DOPH' if doph else 'MinHash'}+bucketize+assign), sparse sets",
        "value": n / (ms * 1e-3), "unit": "sets/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"sets: n={n} sets, {nnz} tokens over a {cfg['vocab']}-token vocabulary, "
                               f"{cfg['clusters']} planted clusters, {name}, bands K={K} x L={Lb}, "
                               f"k={k} planted seeds",
                   "n": n, "nnz": nnz, "k": k, "F": F, "hash": args.sets_hash},
        "roofline": {"bound": "alu", "achieved": compares / (t_as * 1e-3) / 1e12, "peak": peak_alu,
                     "unit": "Tcompare/s", "frac": compares / (t_as * 1e-3) / 1e12 / peak_alu, "traffic": None,
                     "kernel": "signature assignment (k_sig_dense)", "avg_launch_ms": t_as},
        "stages_ms": {("doph" if doph else "minhash"): t_hash, "bucketize": t_bz, "assign": t_as},
        "hash_hbm_gbs": hash_bytes / (t_hash * 1e-3) / 1e9,
        "hash_hbm_frac": hash_bytes / (t_hash * 1e-3) / 8e12,
        "assign_counters": out["counters"].cpu().numpy().tolist(),
    }
    if not doph:
        line["minhash_evals_per_s"] = nnz * K * Lb / (t_hash * 1e-3)
    if not args.no_cpu:
        line["cpu_baseline"] = _oracle_sets_sample(off, tok, mh, so, sm, F if doph else None, sig, out, 512)
    print(json.dumps(line), flush=True)


def _oracle_sets_sample(off, tok, mh, so, sm, doph_dims, sig, out, rows):
    """The oracle (numpy, one thread) on a sample of the sets workload: the
    signatures (MinHash, or DOPH when doph_dims is given) of every planted
    seed member and of the first rows, the seeds' modes, and the assignment
    of those rows.  Returns the cpu_baseline object (sets/s, seed work
    prorated by rows / n) with the sampled checks against the GPU."""
    import numpy as np

    import oracle

    offh, tokh = off.cpu().numpy().astype(np.int64), tok.cpu().numpy().view(np.uint32)
    keys = mh.cpu().numpy().view(np.uint32)
    n = len(offh) - 1
    rows = min(rows, n)

    def sub(ids):  # the CSR of the sets ids, in that order
        lens = offh[ids + 1] - offh[ids]
        o = np.zeros(len(ids) + 1, np.int64)
        np.cumsum(lens, out=o[1:])
        idx = np.repeat(offh[ids] - o[:-1], lens) + np.arange(o[-1])
        return o, tokh[idx]

    def sigs(ids):
        o, t = sub(ids)
        if doph_dims:
            return oracle.doph_sets(o, t, keys.reshape(-1, 2)[0], doph_dims)
        return oracle.minhash_sets(o, t, keys)

    t0 = time.perf_counter()
    S_mem = sigs(np.asarray(sm, dtype=np.int64))
    M = oracle.modes(S_mem, so, np.arange(len(sm), dtype=np.uint32))
    t_seed = time.perf_counter() - t0
    t0 = time.perf_counter()
    S_rows = sigs(np.arange(rows, dtype=np.int64))
    a_ref, d_ref = oracle.assign_sig(S_rows, M)
    t_rows = time.perf_counter() - t0
    s_gpu = float(out["dist"][:rows].double().sum())
    return {"value": rows / (t_rows + t_seed * rows / n), "unit": "sets/s", "cores": 1, "kind": "oracle",
            "sample": f"signatures of the first {rows} of {n} sets and of all {len(sm)} planted seed members, "
                      "the seeds' modes and the rows' assignment (numpy, one thread; seed work prorated by "
                      "rows / n); bucketing not included",
            "sample_signatures_match_gpu": bool(np.array_equal(S_rows.astype(np.uint32),
                                                               sig[:rows].cpu().numpy().view(np.uint32))),
            "sample_assign_matches_gpu": bool(np.array_equal(a_ref, out["assign"][:rows].cpu().numpy())),
            "sample_sse_rel_err_vs_oracle": abs(s_gpu - float(d_ref.sum())) / max(float(d_ref.sum()), 1e-300)}


def bench_silk(args):
    """The whole GEEK pass on the dense mixture (d = 128, Zipf cluster sizes,
    clusters scaled with n) at the scaled E2LSH width w * sqrt(d): hash,
    buckets of 32 tables, SILK seeds (K_S = 3, L_S = 20, delta = 10), then the
    BF16 assignment to the SILK seeds.  The pass is timed eagerly with
    events per stage.  The binding reads the seed count k back to the host
    between SILK and the assignment, so the assignment costs what k seeds
    cost rather than SILK's capacity (geek_assign's k_dev avoids the
    read-back, at the capacity's cost)."""
    import numpy as np
    import torch

    from paper_2106_10515_amd import _lib as L
    from paper_2106_10515_amd import api
    from workloads import CONFIGS, dense_mixture, e2lsh_params, key_words
    from workloads.gen import STREAM_SILK

    dev = torch.device("cuda:0")
    cfg = CONFIGS["dense_large"]
    n = 1_000_000 if args.n == 10_000_000 else args.n
    d, m, Lt = cfg["d"], cfg["m"], cfg["L"]
    w = cfg["w"] * d ** 0.5
    clusters = max(1, cfg["clusters"] * n // cfg["n"])
    X, _, _ = dense_mixture(n, d, clusters, cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"], seed=0, device=dev)
    A, b = e2lsh_params(m * Lt, d, w, 0)
    Ag, bg = torch.from_numpy(A).to(dev), torch.from_numpy(b).to(dev)
    K, LS, delta = cfg["K_S"], cfg["L_S"], cfg["delta"]
    keys = torch.from_numpy(key_words((LS + 1) * K, 0, STREAM_SILK).view(np.int32)).to(dev)
    status = api.new_status(dev)

    def one():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        kg, _ = api.hash_dense(X, Ag, bg, m, Lt, w, status=status, check=False)
        ev[1].record()
        bm, bo, bn, _ = api.bucketize(kg, n, Lt, 4, n * 4, 4, want_bucket_of=False, status=status, check=False)
        ev[2].record()
        so, sm, ctr = api.silk_seeds(bm, bo, bn, n, Lt, K, LS, delta, keys, status=status, check=False)
        ev[3].record()
        k = len(so) - 1
        out = api.assign_euclid(X, so, sm, k, L.GEEK_PREC_BF16, status=status, check=False) if k > 0 else None
        ev[4].record()
        torch.cuda.synchronize()
        return [ev[i].elapsed_time(ev[i + 1]) for i in range(4)], k, ctr, out, (so, sm)

    for _ in range(args.warmup):
        one()
    api.check_status(status, "warmup")
    runs = [one() for _ in range(args.steps)]
    api.check_status(status, "timed")
    st = np.median(np.array([r[0] for r in runs]), axis=0)
    _, k, ctr, out, _ = runs[-1]
    total = float(st.sum())
    line = {
        "metric": "points/s (hash+bucketize+SILK+assign), whole GEEK pass",
        "value": n / (total * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"silk: n={n} d={d} {clusters}-cluster Gaussian mixture (Zipf sizes), "
                               f"E2LSH m={m} L={Lt} w={w:.2f} (scaled), SILK K={K} L={LS} delta={delta}",
                   "n": n, "k_found": k},
        "stages_ms": {"hash": float(st[0]), "bucketize": float(st[1]), "silk": float(st[2]),
                      "assign": float(st[3])},
        "silk_counters": ctr.cpu().numpy().tolist(),
        # SILK's algorithmic work: K hash evaluations per (table, object) and
        # SILK table (the counters' first entry), about 6 integer VALU
        # operations each (the member's finalizer mix shared by its K
        # evaluations, then multiply, add and min per evaluation)
        "roofline": {"bound": "alu", "achieved": float(ctr[0]) * 6 / (st[2] * 1e-3) / 1e12,
                     "peak": 256 * 64 * 2.4e9 / 1e12, "unit": "Tops/s",
                     "frac": float(ctr[0]) * 6 / (st[2] * 1e-3) / (256 * 64 * 2.4e9), "traffic": None,
                     "kernel": "geek_silk_seeds (all kernels of the call)", "avg_launch_ms": float(st[2])},
        "assign_counters": out["counters"].cpu().numpy().tolist() if out is not None else None,
        "sse": float(out["sse"].item()) if out is not None else None,
    }
    if out is not None and not args.no_cpu:
        so, sm = runs[-1][4]
        line["cpu_baseline"] = _oracle_euclid_sample([(X, so, sm, out)], 64)
    print(json.dumps(line), flush=True)


def bench_refine(args):
    """A further assignment pass (Section 4.3) on the dense large workload:
    the clusters of the BF16 assignment to the 10,000 planted seeds become the
    seeds (geek_regroup), their centroids are recomputed and all 10^7 points
    are assigned again on the BF16 matrix cores (geek_assign).  One step =
    one such pass from the same first assignment; the cluster count is read
    back to the host between the two calls, so steps are timed eagerly with
    events."""
    import numpy as np
    import torch

    from paper_2106_10515_amd import _lib as L
    from paper_2106_10515_amd import api
    from workloads import CONFIGS, dense_mixture, planted_seeds

    dev = torch.device("cuda:0")
    cfg = CONFIGS["dense_large"]
    n, d = args.n, cfg["d"]
    clusters = min(args.clusters, n)
    X, labels, _ = dense_mixture(n, d, clusters, cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"],
                                 seed=0, device=dev)
    so, sm = planted_seeds(labels, clusters, 32)
    k = len(so) - 1
    sog = torch.from_numpy(so.view(np.int32)).to(dev)
    smg = torch.from_numpy(sm.view(np.int32)).to(dev)
    status = api.new_status(dev)
    first = api.assign_euclid(X, sog, smg, k, L.GEEK_PREC_BF16, status=status)
    a0 = first["assign"]

    def one():
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        so2, sm2, k_out, lab = api.regroup(a0, k, status=status, check=False)
        ev[1].record()
        k2 = int(k_out.item())
        out = api.assign_euclid(X, so2[:k2 + 1], sm2, k2, L.GEEK_PREC_BF16, status=status, check=False)
        ev[2].record()
        torch.cuda.synchronize()
        return [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])], k2, out

    for _ in range(args.warmup):
        one()
    api.check_status(status, "warmup")
    L.geek_profile(True)
    runs = [one() for _ in range(args.steps)]
    scan_ms, scan_n = L.geek_profile_read(L.GEEK_PROF_ASSIGN_SCAN)
    L.geek_profile(False)
    api.check_status(status, "timed")
    st = np.median(np.array([r[0] for r in runs]), axis=0)
    _, k2, out = runs[-1]
    total = float(st.sum())
    scan_avg = scan_ms / max(scan_n, 1)
    flops = 2.0 * n * d * k2
    ach = flops / (scan_avg * 1e-3) / 1e12
    line = {
        "metric": "points/s of one further assignment pass (regroup + centroids + BF16 assignment)",
        "value": n / (total * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"refine: dense_large n={n} d={d} {clusters}-cluster Gaussian mixture "
                               f"(Zipf sizes); pass from the assignment to k={k} planted seeds",
                   "n": n, "k_in": k, "k_out": k2},
        "stages_ms": {"regroup": float(st[0]), "assign": float(st[1])},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_BF16, "unit": "TFLOP/s",
                     "frac": ach / PEAK_BF16, "traffic": None, "kernel": "k_scan<ModeBF16,128>",
                     "avg_launch_ms": scan_avg, "flop_per_launch": flops},
        "assign_counters": out["counters"].cpu().numpy().tolist(),
        "sse_first": float(first["sse"].item()),
        "sse_after_pass": float(out["sse"].item()),
    }
    print(json.dumps(line), flush=True)


def bench_quantile(args):
    """Algorithm 1's dense transformation on the dense large mixture: m = 40
    projections a ~ N(0, I), each table ranked by a . x in float64 and split
    evenly into t = 10,000 buckets (the paper's parameter study fixes m = 40
    and varies t from 5,000 to 30,000).  One step = one geek_quantile_buckets
    call over all 10^7 points."""
    import numpy as np
    import torch

    from paper_2106_10515_amd import api
    from workloads import CONFIGS, dense_mixture, e2lsh_params

    dev = torch.device("cuda:0")
    cfg = CONFIGS["dense_large"]
    n, d = args.n, cfg["d"]
    m, t = 40, 10_000
    clusters = min(args.clusters, n)
    X, _, _ = dense_mixture(n, d, clusters, cfg["lo"], cfg["hi"], cfg["sigma"], cfg["sizes"], seed=0, device=dev)
    A, _ = e2lsh_params(m, d, 1.0, 0)
    Ag = torch.from_numpy(A).to(dev)
    status = api.new_status(dev)
    for _ in range(args.warmup):
        api.quantile_buckets(X, Ag, t, status=status, check=False)
    torch.cuda.synchronize()
    api.check_status(status, "warmup")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        mem, off, bof = api.quantile_buckets(X, Ag, t, status=status, check=False)
    e1.record()
    torch.cuda.synchronize()
    api.check_status(status, "timed")
    ms = e0.elapsed_time(e1) / args.steps
    algo = 4.0 * n * d + 2 * 4.0 * m * n + 4.0 * m * (t + 1)  # X once; members + bucket_of; offsets
    gbs = algo / (ms * 1e-3) / 1e9
    sizes = np.diff(off.cpu().numpy().astype(np.int64), axis=1)
    line = {
        "metric": "points/s of Algorithm 1's quantile bucketing (m tables, t buckets each)",
        "value": n / (ms * 1e-3), "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"quantile: dense_large n={n} d={d} {clusters}-cluster Gaussian mixture "
                               f"(Zipf sizes), m={m} projections a~N(0,I), t={t}",
                   "n": n, "d": d, "m": m, "t": t},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM, "unit": "GB/s", "frac": gbs / PEAK_HBM,
                     "traffic": None, "kernel": "geek_quantile_buckets (whole call)",
                     "bytes_per_launch": algo},
        "bucket_sizes": [int(sizes.min()), int(sizes.max())],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
