"""Helpers shared by the GPU parity tests."""

import sys

import numpy as np
import pytest


def gpu_api():
    """The torch-facing API; skips when there is no GPU."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2106_10515_amd import api

    return api


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def cuda(a):
    import torch

    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32)


def unpack_keys(keys_u32, m):
    """Codes from packed 128-bit table keys: code j at bits j*B .. j*B+B-1
    (little-endian over four words), stored as code + 2**(B-1)."""
    B = min(32, 128 // m)
    L, n, _ = keys_u32.shape
    w = keys_u32.astype(np.uint64)
    big = [(w[..., 0] | (w[..., 1] << np.uint64(32))), (w[..., 2] | (w[..., 3] << np.uint64(32)))]
    out = np.empty((n, L * m), dtype=np.int64)
    for j in range(m):
        bit = j * B
        lo_word = bit // 64
        sh = bit % 64
        v = big[lo_word] >> np.uint64(sh)
        if sh + B > 64:
            v = v | (big[lo_word + 1] << np.uint64(64 - sh))
        v = (v & np.uint64((1 << B) - 1)).astype(np.int64) - (1 << (B - 1))
        out[:, j::m] = v.T
    return out
