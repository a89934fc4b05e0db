"""GPU parity of geek_silk_seeds against the oracle's SILK (Algorithm 4):
the seed sets, their order and the work counters, bit for bit."""

import math

import numpy as np
import pytest
import torch

import oracle
from workloads import dense_mixture, e2lsh_params, key_words, sparse_sets
from workloads.gen import STREAM_SILK

from .gpu_util import announce, cuda, gpu_api, host_u32

pytestmark = pytest.mark.gpu


def _oracle_buckets(codes, m, L):
    offs, mem = [0], []
    for mm, oo, _ in oracle.bucketize_tables(codes, m, L):
        mem.append(mm)
        offs.extend((oo[1:].astype(np.int64) + offs[-1]).tolist())
    return np.asarray(offs, np.int64), np.concatenate(mem)


def _run_dense(api, n, d, clusters, m, L, w, K, LS, delta, seed, check=True):
    X, _, _ = dense_mixture(n, d, clusters, -10, 10, 1.0, "equal", seed)
    A, b = e2lsh_params(m * L, d, w, seed)
    keys = key_words((LS + 1) * K, seed, STREAM_SILK)
    codes = oracle.e2lsh_codes(X, A, b, w)
    offs, mem = _oracle_buckets(codes, m, L)
    ref_o, ref_m, info = oracle.silk_seeds(offs, mem, K, LS, delta, keys)
    announce(f"silk n={n} d={d} m={m} L={L} K={K} LS={LS} delta={delta} ref k={len(ref_o) - 1}")
    kg, _ = api.hash_dense(cuda(X), cuda(A), cuda(b), m, L, w)
    bm, bo, bn, _ = api.bucketize(kg, n, L, 4, n * 4, 4, want_bucket_of=False)
    status = api.new_status("cuda")
    so, sm, ctr = api.silk_seeds(bm, bo, bn, n, L, K, LS, delta, cuda(keys), status=status,
                                 check=False)
    return (ref_o, ref_m, info), (host_u32(so), host_u32(sm), ctr.cpu().numpy()), int(status.item())


@pytest.mark.parametrize("n,d,clusters,m,L,K,LS,delta,seed", [
    (4000, 32, 20, 8, 16, 3, 20, 10, 0),
    (6000, 16, 40, 6, 10, 2, 8, 5, 1),
    (3000, 32, 10, 8, 8, 4, 12, 3, 2),
])
def test_silk_matches_oracle(n, d, clusters, m, L, K, LS, delta, seed):
    api = gpu_api()
    w = 4.0 * math.sqrt(d)
    (ro, rm, info), (go, gm, ctr), st = _run_dense(api, n, d, clusters, m, L, w, K, LS, delta, seed)
    assert st == 0
    assert len(ro) > 2
    assert np.array_equal(go, ro)
    assert np.array_equal(gm, rm)
    assert ctr[0] == info["hash_evals"]
    assert ctr[1] == info["pairs_voted"]
    assert ctr[2] == info["multiset"]


def test_silk_no_seeds_literal_width():
    # the literal width puts almost every point alone in its bucket: no seed
    api = gpu_api()
    (ro, rm, info), (go, gm, ctr), st = _run_dense(api, 3000, 32, 10, 8, 16, 4.0, 3, 6, 10, 3)
    assert len(ro) == 1
    assert st == 4 and len(go) == 1


def test_silk_capacity_reported():
    api = gpu_api()
    from paper_2106_10515_amd import GeekError

    n, d, m, L, w = 3000, 32, 8, 16, 4.0 * math.sqrt(32)
    X, _, _ = dense_mixture(n, d, 10, -10, 10, 1.0, "equal", 4)
    A, b = e2lsh_params(m * L, d, w, 4)
    keys = key_words(21 * 3, 4, STREAM_SILK)
    kg, _ = api.hash_dense(cuda(X), cuda(A), cuda(b), m, L, w)
    bm, bo, bn, _ = api.bucketize(kg, n, L, 4, n * 4, 4, want_bucket_of=False)
    with pytest.raises(GeekError) as e:
        api.silk_seeds(bm, bo, bn, n, L, 3, 20, 10, cuda(keys), cap_k=2, cap_members=4000)
    assert e.value.code == 3


def test_silk_over_minhash_bands():
    # sets -> MinHash -> band buckets -> SILK, compared with the oracle chain
    api = gpu_api()
    off, tok, _ = sparse_sets(4000, vocab=20_000, clusters=30, seed=5)
    K, Lb = 4, 16
    mk = key_words(K * Lb, 5)
    sig = oracle.minhash_sets(off, tok, mk)
    offs, mem = [0], []
    for mm, oo, _ in oracle.bucketize_tables(sig, K, Lb):
        mem.append(mm)
        offs.extend((oo[1:].astype(np.int64) + offs[-1]).tolist())
    sk = key_words(21 * 3, 5, STREAM_SILK)
    ro, rm, info = oracle.silk_seeds(np.asarray(offs), np.concatenate(mem), 3, 20, 10, sk)
    announce(f"silk bands n=4000 ref k={len(ro) - 1}")
    sg = api.hash_sets(cuda(off), cuda(tok), cuda(mk))
    n = len(off) - 1
    bm, bo, bn, _ = api.bucketize(sg, n, Lb, K, K, K * Lb, want_bucket_of=False)
    so, sm, ctr = api.silk_seeds(bm, bo, bn, n, Lb, 3, 20, 10, cuda(sk), check=len(ro) > 1)
    assert np.array_equal(host_u32(so), ro)
    assert np.array_equal(host_u32(sm), rm)


def test_silk_pass_captured_in_one_graph():
    # hash -> bucketize -> SILK -> assignment recorded in one HIP graph: the
    # SILK call reads nothing back to the host and the assignment takes the
    # seed count from the device (k = the seed capacity).  Every replay,
    # with eager work and synchronizations between replays, gives the eager
    # seeds and assignment bit for bit, and that assignment equals a call
    # with the count given on the host.
    from paper_2106_10515_amd import _lib as L

    api = gpu_api()
    n, d, m, Lt, K, LS, delta = 4000, 32, 8, 16, 3, 20, 10
    w = 4.0 * math.sqrt(d)
    X, _, _ = dense_mixture(n, d, 20, -10, 10, 1.0, "equal", 0)
    A, b = e2lsh_params(m * Lt, d, w, 0)
    keys = cuda(key_words((LS + 1) * K, 0, STREAM_SILK))
    Xg, Ag, bg = cuda(X), cuda(A), cuda(b)
    cap_k, cap_m = 4096, 16000
    announce(f"silk + assign graph capture n={n}")

    def chain(status):
        kg, _ = api.hash_dense(Xg, Ag, bg, m, Lt, w, status=status, check=False)
        bm, bo, bn, _ = api.bucketize(kg, n, Lt, 4, n * 4, 4, want_bucket_of=False, status=status, check=False)
        out = api.silk_seeds_async(bm, bo, bn, n, Lt, K, LS, delta, keys, cap_k, cap_m, status)
        asg = api.assign_euclid(Xg, out["seed_offsets"], out["seed_members"], cap_k, L.GEEK_PREC_BF16,
                                status=status, check=False, k_dev=out["k_out"])
        return out, asg

    def result(res):
        out, asg = res
        k = int(out["k_out"].item())
        so = host_u32(out["seed_offsets"][:k + 1])
        return (so, host_u32(out["seed_members"][:int(so[-1])]), out["counters"].cpu().numpy(),
                asg["assign"].cpu().numpy(), asg["dist"].cpu().numpy(), asg["sse"].cpu().numpy(),
                asg["centroids"].cpu().numpy(), asg["radius"].cpu().numpy())

    st_e = api.new_status("cuda")
    eager = chain(st_e)
    ref = result(eager)
    assert int(st_e.item()) == 0 and len(ref[0]) > 2
    # the device count against the host count, on the same seeds
    k = len(ref[0]) - 1
    host = api.assign_euclid(Xg, eager[0]["seed_offsets"][:k + 1].clone(),
                             eager[0]["seed_members"][:int(ref[0][-1])].clone(), k, L.GEEK_PREC_BF16)
    assert np.array_equal(ref[3], host["assign"].cpu().numpy())
    assert np.array_equal(ref[4], host["dist"].cpu().numpy())
    assert np.array_equal(ref[5], host["sse"].cpu().numpy())
    assert np.array_equal(ref[6][:k], host["centroids"].cpu().numpy())
    assert not ref[6][k:].any()
    assert np.array_equal(ref[7][:k], host["radius"].cpu().numpy())
    assert not ref[7][k:].any()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    st_g = api.new_status("cuda")
    with torch.cuda.stream(side):
        chain(st_g)  # warm-up on the side stream (workspace for that stream)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        res = chain(st_g)
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        got = result(res)
        assert int(st_g.item()) == 0, rep
        for a, r in zip(got, ref):
            assert np.array_equal(a, r), rep
        chain(api.new_status("cuda"))  # eager work between replays
        torch.cuda.synchronize()


def test_silk_multiset_capacity_reported_then_fits():
    # too little room for the intermediate multiset C: the call reports the
    # room C needs (needed[2]); called again with it, the seeds equal those of
    # a call with ample room
    api = gpu_api()
    from paper_2106_10515_amd import _lib as L

    n, d, m, Lt, w = 4000, 32, 8, 16, 4.0 * math.sqrt(32)
    X, _, _ = dense_mixture(n, d, 20, -10, 10, 1.0, "equal", 0)
    A, b = e2lsh_params(m * Lt, d, w, 0)
    keys = cuda(key_words(21 * 3, 0, STREAM_SILK))
    kg, _ = api.hash_dense(cuda(X), cuda(A), cuda(b), m, Lt, w)
    bm, bo, bn, _ = api.bucketize(kg, n, Lt, 4, n * 4, 4, want_bucket_of=False)
    announce("silk multiset capacity")
    st = api.new_status("cuda")
    out = api.silk_seeds_async(bm, bo, bn, n, Lt, 3, 20, 10, keys, 4096, 64000, st, cap_c=100)
    torch.cuda.synchronize()
    assert int(st.item()) == L.GEEK_ERR_CAPACITY
    need = out["needed"].cpu().numpy()
    assert need[0] == 0 and need[1] == 0 and need[2] > 100
    st.zero_()
    out2 = api.silk_seeds_async(bm, bo, bn, n, Lt, 3, 20, 10, keys, 4096, 64000, st, cap_c=int(need[2]))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    ref_o, ref_m, _ = api.silk_seeds(bm, bo, bn, n, Lt, 3, 20, 10, keys)
    k = int(out2["k_out"].item())
    assert torch.equal(out2["seed_offsets"][:k + 1], ref_o)
    assert torch.equal(out2["seed_members"][:int(ref_o[-1])], ref_m)
    assert int(out2["needed"][2]) == int(need[2])
