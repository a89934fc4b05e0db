"""GPU parity of geek_quantile_buckets (paper Algorithm 1) against the FP64
oracle: members, offsets and bucket_of of every table bit for bit."""

import numpy as np
import pytest

import oracle
from workloads import dense_mixture, e2lsh_params

from .gpu_util import announce, cuda, gpu_api, host_u32

pytestmark = pytest.mark.gpu


def _case(api, X, A, t, name):
    announce(f"quantile {name} n={len(X)} d={X.shape[1]} m={len(A)} t={t}")
    mem, off, bof = oracle.quantile_buckets(X, A, t)
    gm, go, gb = api.quantile_buckets(cuda(X), cuda(A), t)
    assert np.array_equal(host_u32(go), off)
    assert np.array_equal(host_u32(gb), bof)
    assert np.array_equal(host_u32(gm), mem)


@pytest.mark.parametrize("n,d,m,t,seed", [
    (5000, 32, 4, 8, 0),       # several radix tiles, t a power of two
    (3001, 128, 3, 97, 1),     # ragged n, t not dividing n
    (777, 20, 2, 777, 2),      # t = n: one object per bucket
    (1000, 256, 2, 1, 3),      # t = 1: one bucket per table
    (70001, 16, 2, 300, 4),    # buckets of 233-234 sorted in LDS
    (20000, 8, 2, 3, 5),       # buckets of 6,667: the second radix sort by bucket
    (12288, 8, 2, 3, 6),       # buckets of exactly 4,096: the largest sorted in LDS
])
def test_quantile_buckets_match_oracle(n, d, m, t, seed):
    api = gpu_api()
    X, _, _ = dense_mixture(n, d, 20, -10, 10, 1.0, "equal", seed)
    A, _ = e2lsh_params(m, d, 1.0, seed)
    _case(api, X, A, t, "mixture")


def test_quantile_buckets_ties_and_signed_zero():
    api = gpu_api()
    g = np.random.default_rng(5)
    # small integers: many objects share a value, exactly; zero values from
    # both signs of the products
    X = g.integers(-2, 3, size=(4000, 6)).astype(np.float32)
    A = np.array([[1, 0, 0, 0, 0, 0], [1, -1, 1, -1, 1, -1], [0, 0, 0, 0, 0, -1]], np.float32)
    _case(api, X, A, 37, "ties")
    Xn = X.copy()
    Xn[17, 2] = np.nan
    from paper_2106_10515_amd import GeekError
    with pytest.raises(GeekError) as e:
        api.quantile_buckets(cuda(Xn), cuda(A), 5)
    assert e.value.code == 1


def test_quantile_buckets_strided_rows():
    # X as the first d columns of a wider row-major matrix (ldx > d)
    api = gpu_api()
    import torch

    g = np.random.default_rng(7)
    W = g.normal(size=(3000, 40)).astype(np.float32)
    A = g.normal(size=(3, 33)).astype(np.float32)
    announce("quantile strided n=3000 d=33 ldx=40")
    mem, off, bof = oracle.quantile_buckets(W[:, :33], A, 50)
    Wg = torch.from_numpy(W).cuda()
    gm, go, gb = api.quantile_buckets(Wg[:, :33], torch.from_numpy(A).cuda(), 50)
    assert np.array_equal(host_u32(gm), mem) and np.array_equal(host_u32(go), off)
    assert np.array_equal(host_u32(gb), bof)


def test_quantile_buckets_transposed_projection_view():
    # A handed over as a transposed (non-contiguous) view: the binding's
    # contiguous copy must stay alive until the call has been enqueued
    api = gpu_api()
    X = dense_mixture(4000, 24, 5, -10, 10, 1.0, "equal", 7)[0]
    A = np.random.default_rng(7).standard_normal((3, 24)).astype(np.float32)
    At = cuda(np.ascontiguousarray(A.T)).T
    assert not At.is_contiguous()
    announce("quantile transposed A view n=4000 d=24 m=3 t=40")
    mem, off, bof = oracle.quantile_buckets(X, A, 40)
    gm, go, gb = api.quantile_buckets(cuda(X), At, 40)
    assert np.array_equal(host_u32(go), off)
    assert np.array_equal(host_u32(gb), bof)
    assert np.array_equal(host_u32(gm), mem)
