"""Batched geek_assign (many Euclidean jobs in one call, persistent
first-pass launches): every job's outputs equal those of a call with that job
alone bit for bit, and the oracle's for a sample of jobs; a captured HIP graph
of the batched call replays to the same results; completion times are
recorded per job."""

import numpy as np
import pytest

import oracle
from workloads import batched_jobs, dense_mixture, planted_seeds

from .gpu_util import announce, cuda, gpu_api

pytestmark = pytest.mark.gpu

PRECS = {"fp32": 0, "bf16": 1, "fp8": 2}


def _problems(njobs, seed):
    # the many-job recipe at small sizes: n log-uniform in [300, 20000],
    # d over {16 .. 256}, up to 300 planted clusters, 8-member seeds
    specs = batched_jobs(njobs, seed=seed, n_lo=2.5, n_hi=4.3, k_hi=300)
    probs, host = [], []
    for sp in specs:
        X, lab, _ = dense_mixture(sp["n"], sp["d"], sp["clusters"], sp["lo"], sp["hi"], sp["sigma"],
                                  sp["sizes"], sp["seed"])
        so, sm = planted_seeds(lab, sp["clusters"], 8)
        probs.append((cuda(X), cuda(so), cuda(sm), len(so) - 1))
        host.append((X, so, sm))
    return probs, host


def _same(a, b, j):
    for key in ("assign", "centroids", "dist", "sse", "radius", "counters"):
        x, y = a[key].cpu().numpy(), b[key].cpu().numpy()
        assert np.array_equal(x, y), (j, key)


@pytest.mark.parametrize("prec,njobs,seed", [("bf16", 24, 0), ("fp8", 12, 1), ("fp32", 10, 2)])
def test_batch_equals_single_calls(prec, njobs, seed):
    api = gpu_api()
    probs, host = _problems(njobs, seed)
    announce(f"batch {prec} jobs={njobs} n={[p[0].shape[0] for p in probs]}")
    outs, t_done = api.assign_euclid_batch(probs, PRECS[prec])
    for j, (X, so, sm, k) in enumerate(probs):
        single = api.assign_euclid(X, so, sm, k, PRECS[prec])
        _same(outs[j], single, j)
    # oracle on the three smallest jobs
    for j in np.argsort([h[0].shape[0] for h in host])[:3]:
        X, so, sm = host[j]
        C = oracle.centroids(X, so, sm)
        a, dist = oracle.assign_euclid(X, C)
        assert np.array_equal(outs[j]["assign"].cpu().numpy(), a), j
        assert np.array_equal(outs[j]["dist"].cpu().numpy(), dist), j
        assert outs[j]["sse"].item() == oracle.sse(dist), j
    t = t_done.cpu().numpy()
    # jobs finish on several streams at once: any order, all after the start
    assert (t > 0).all(), t
    assert api.wallclock_hz() > 0


def test_batch_graph_replays():
    import torch

    api = gpu_api()
    probs, _ = _problems(16, 3)
    announce("batch graph capture, 16 jobs bf16")
    ref, _ = api.assign_euclid_batch(probs, PRECS["bf16"])
    status = api.new_status(torch.device("cuda"))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm the workspace cache outside capture
        api.assign_euclid_batch(probs, PRECS["bf16"], status=status, check=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs, t_done = api.assign_euclid_batch(probs, PRECS["bf16"], status=status, check=False)
    for rep in range(3):
        for o in outs:  # scribble over the outputs between replays
            o["assign"].fill_(-7)
            o["sse"].fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        api.check_status(status, f"replay {rep}")
        for j in range(len(probs)):
            _same(outs[j], ref[j], (rep, j))


@pytest.fixture
def default_tiles():
    from paper_2106_10515_amd import _lib as L

    saved = {(p, dp): L.geek_get_scan_tiles(p, dp) for p in (0, 1, 2) for dp in (32, 64, 128, 256)}
    yield L
    for (p, dp), shape in saved.items():
        L.geek_set_scan_tiles(p, dp, *shape)


@pytest.mark.parametrize("prec,seed", [("bf16", 4), ("fp8", 5), ("fp32", 6)])
def test_batch_every_tile_shape_same_records(prec, seed, default_tiles):
    # every compiled tile shape of the batched first pass gives the same
    # outputs as the single-job calls
    from paper_2106_10515_amd import autotune

    L = default_tiles
    api = gpu_api()
    probs, _ = _problems(10, seed)
    singles = [api.assign_euclid(X, so, sm, k, PRECS[prec]) for X, so, sm, k in probs]
    dps = sorted({autotune.padded_depth(p[0].shape[1]) for p in probs})
    shapes = set()
    for dp in dps:
        shapes.update(autotune.candidates(PRECS[prec], dp, blocks=(1, 3)))
    for shape in sorted(shapes):
        for dp in dps:
            if L.geek_set_scan_tiles(PRECS[prec], dp, *shape) != L.GEEK_OK:
                L.geek_set_scan_tiles(PRECS[prec], dp, 0, 0, 0)
        announce(f"batch {prec} tile shape {shape}")
        outs, _ = api.assign_euclid_batch(probs, PRECS[prec])
        for j, single in enumerate(singles):
            _same(outs[j], single, (shape, j))


def test_autotune_installs_fastest(default_tiles):
    from paper_2106_10515_amd import autotune

    L = default_tiles
    api = gpu_api()
    probs, _ = _problems(8, 7)
    announce("autotune bf16 on 8 small jobs")
    res = autotune.tune_batch_tiles(probs, PRECS["bf16"], reps=1, blocks=(2, 8))
    assert res
    for dp, r in res.items():
        assert r["best"] == min(r["ms"], key=r["ms"].get)
        assert L.geek_get_scan_tiles(PRECS["bf16"], dp) == r["best"]
        assert len(r["ms"]) == len(autotune.candidates(PRECS["bf16"], dp, blocks=(2, 8)))
    outs, _ = api.assign_euclid_batch(probs, PRECS["bf16"])
    for j, (X, so, sm, k) in enumerate(probs):
        _same(outs[j], api.assign_euclid(X, so, sm, k, PRECS["bf16"]), j)


def test_hash_and_bucketize_batches_equal_single_calls():
    # multi-job geek_hash / geek_bucketize run their jobs on several streams,
    # each with its own workspace slice: every job's keys and buckets equal
    # those of a call with that job alone (also when replayed from a graph)
    import torch

    from workloads import e2lsh_params

    api = gpu_api()
    probs, _ = _problems(9, 9)
    m, Lt, w = 8, 16, 4.0 * 4
    hp = {}
    for X, _, _, _ in probs:
        d = X.shape[1]
        if d not in hp:
            A, b = e2lsh_params(m * Lt, d, w, 3)
            hp[d] = (cuda(A), cuda(b))
    hjobs = [(X, *hp[X.shape[1]], m, Lt, w) for X, _, _, _ in probs]
    announce(f"hash/bucketize batch of {len(hjobs)} jobs")
    keys_b = api.hash_dense_batch(hjobs)
    singles = [api.hash_dense(*job)[0] for job in hjobs]
    for j, (kb, ks) in enumerate(zip(keys_b, singles)):
        assert torch.equal(kb, ks), j
    bjobs = [(k, X.shape[0], Lt, 4, X.shape[0] * 4, 4) for k, (X, _, _, _) in zip(keys_b, probs)]

    def same_buckets(outs):
        for j, (ob, job) in enumerate(zip(outs, bjobs)):
            os_ = api.bucketize(*job)
            nb = ob[2].cpu().numpy()
            assert np.array_equal(nb, os_[2].cpu().numpy()), j
            assert torch.equal(ob[0], os_[0]) and torch.equal(ob[3], os_[3]), j
            for t in range(Lt):
                assert torch.equal(ob[1][t, :nb[t] + 1], os_[1][t, :nb[t] + 1]), (j, t)

    same_buckets(api.bucketize_batch(bjobs))
    status = api.new_status(torch.device("cuda"))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm the workspace cache outside capture
        api.bucketize_batch(bjobs, status=status, check=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = api.bucketize_batch(bjobs, status=status, check=False)
    for rep in range(2):
        for o in outs:
            o[0].fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        api.check_status(status, f"replay {rep}")
        same_buckets(outs)
