"""GPU parity of geek_regroup and of a further assignment pass (paper
Section 4.3) against the FP64 oracle: clusters bit for bit (offsets, members,
labels), then centroids, assignments, distances and SSE of the next pass."""

import numpy as np
import pytest

import oracle
from workloads import dense_mixture, planted_seeds

from .gpu_util import announce, cuda, gpu_api, host_u32

pytestmark = pytest.mark.gpu


def _regroup_case(api, a, k, name):
    announce(f"regroup {name} n={len(a)} k={k}")
    off, mem, lab = oracle.regroup(a, k)
    so, sm, k_out, lab_g = api.regroup(cuda(np.asarray(a, np.int32)), k)
    ko = int(k_out.item())
    assert ko == len(lab)
    assert np.array_equal(host_u32(so)[:ko + 1], off)
    assert np.array_equal(host_u32(sm), mem)
    assert np.array_equal(lab_g.cpu().numpy()[:ko], lab)


@pytest.mark.parametrize("n,k,used,seed", [
    (1, 1, 1, 0),             # one object
    (1001, 1, 1, 1),          # k = 1: no sort digits at all
    (5000, 7, 3, 2),          # most labels unused
    (20000, 300, 300, 3),     # two 8-bit digits, every label used
    (33333, 70000, 9000, 4),  # three digits, ragged n, most labels unused
])
def test_regroup_matches_oracle(n, k, used, seed):
    api = gpu_api()
    g = np.random.default_rng(seed)
    labels = g.choice(k, size=used, replace=False)
    _regroup_case(api, g.choice(labels, size=n).astype(np.int32), k, "random")


def test_regroup_special_cases():
    api = gpu_api()
    import torch
    from paper_2106_10515_amd import GeekError

    _regroup_case(api, np.full(3000, 6, np.int32), 7, "one-label")
    _regroup_case(api, np.arange(4097, dtype=np.int32)[::-1].copy(), 4097, "all-singletons")
    so, sm, k_out, _ = api.regroup(torch.zeros(0, dtype=torch.int32, device="cuda"), 5)
    assert int(k_out.item()) == 0 and int(so[0].item()) == 0
    with pytest.raises(GeekError) as e:
        api.regroup(cuda(np.array([0, 1, 5, 2], np.int32)), 5)
    assert e.value.code == 2
    with pytest.raises(GeekError) as e:
        api.regroup(cuda(np.array([0, -1], np.int32)), 5)
    assert e.value.code == 2


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("n,d,clusters,per,seed", [
    (4000, 32, 40, 4, 0),     # few seed members: the first pass is rough
    (3001, 128, 150, 2, 1),   # ragged rows, several centroid tiles
])
def test_assignment_passes_match_oracle(prec, n, d, clusters, per, seed):
    api = gpu_api()
    X, lab, _ = dense_mixture(n, d, clusters, -5, 5, 1.5, "zipf", seed)
    so, sm = planted_seeds(lab, clusters, per)
    k = len(so) - 1
    a, _ = oracle.assign_euclid(X, oracle.centroids(X, so, sm))
    Xg = cuda(X)
    cur = api.assign_euclid(Xg, cuda(so), cuda(sm), k, prec)
    assert np.array_equal(cur["assign"].cpu().numpy(), a)
    for p in range(3):
        announce(f"assignment pass {p + 1} n={n} d={d} k={k} prec={prec}")
        off, mem, lab_of, C, a2, d2 = oracle.assignment_pass(X, a, k)
        out = api.assignment_pass(Xg, cur["assign"], k, prec)
        assert out["k"] == len(lab_of)
        assert np.array_equal(out["label_of"].cpu().numpy(), lab_of)
        assert np.array_equal(out["centroids"].cpu().numpy(), C)
        got = out["assign"].cpu().numpy()
        bad = np.flatnonzero(got != a2)
        assert bad.size == 0, (bad[:10], got[bad[:10]], a2[bad[:10]])
        assert np.array_equal(out["dist"].cpu().numpy(), d2)
        assert out["sse"].item() == oracle.sse(d2)
        a, k, cur = a2, len(lab_of), out


@pytest.mark.parametrize("n,d,clusters,per,spare,seed", [
    (3001, 20, 9, 400, 0, 5),     # narrow rows (one dimension tile, ragged)
    (2500, 256, 12, 250, 7, 6),   # four dimension tiles; members buffer 7 entries longer than used
    (5003, 128, 3, 5000, 0, 7),   # three huge seeds, member count not a multiple of 4
])
def test_centroids_of_large_seeds(n, d, clusters, per, spare, seed):
    # seeds averaging 64 members or more take the dimension-major centroid path
    api = gpu_api()
    X, lab, _ = dense_mixture(n, d, clusters, -10, 10, 1.0, "zipf", seed)
    so, sm = planted_seeds(lab, clusters, per)
    k = len(so) - 1
    assert len(sm) >= 64 * k
    announce(f"large seeds n={n} d={d} k={k} members={len(sm)} spare={spare}")
    C = oracle.centroids(X, so, sm)
    a, dist = oracle.assign_euclid(X, C)
    smg = cuda(np.concatenate([sm, np.zeros(spare, np.uint32)]))
    out = api.assign_euclid(cuda(X), cuda(so), smg, k, 1)
    assert np.array_equal(out["centroids"].cpu().numpy(), C)
    assert np.array_equal(out["assign"].cpu().numpy(), a)
    assert np.array_equal(out["dist"].cpu().numpy(), dist)


def test_regroup_two_jobs_one_call():
    # two jobs in one geek_regroup call (through the C ABI) equal the oracle
    api = gpu_api()
    import torch
    from paper_2106_10515_amd import _lib as L

    g = np.random.default_rng(8)
    cases = [(g.integers(0, 9, 5000).astype(np.int32), 12), (g.integers(0, 300, 777).astype(np.int32), 300)]
    jobs, outs = [], []
    for a, k in cases:
        ag = cuda(a)
        so = torch.empty(k + 1, dtype=torch.int32, device="cuda")
        sm = torch.empty(len(a), dtype=torch.int32, device="cuda")
        ko = torch.zeros(1, dtype=torch.int32, device="cuda")
        lab = torch.empty(k, dtype=torch.int32, device="cuda")
        outs.append((ag, so, sm, ko, lab))
        jobs.append(L.RegroupJob(n=len(a), k=k, assign=ag.data_ptr(), seed_offsets=so.data_ptr(),
                                 seed_members=sm.data_ptr(), k_out=ko.data_ptr(), label_of=lab.data_ptr()))
    announce("regroup two jobs in one call")
    status = api.new_status("cuda")
    api._run(L.GEEK_OP_REGROUP, L.geek_regroup, jobs, torch.device("cuda:0"), status)
    api.check_status(status, "geek_regroup (two jobs)")
    for (a, k), (_, so, sm, ko, lab) in zip(cases, outs):
        off, mem, lo = oracle.regroup(a, k)
        kk = int(ko.item())
        assert kk == len(lo)
        assert np.array_equal(host_u32(so)[:kk + 1], off) and np.array_equal(host_u32(sm), mem)
        assert np.array_equal(lab.cpu().numpy()[:kk], lo)
