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
    assert (t > 0).all() and (np.diff(t) >= 0).all(), t
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
