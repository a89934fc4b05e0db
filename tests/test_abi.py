"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point that include/geek.h declares, and the ctypes job structs
have the header's layout; argument errors are reported without a GPU."""

import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2106_10515_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "geek.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\S.*?\b(geek_[a-z_]+)\s*\(", txt, flags=re.M)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libgeek.so is not built (run __graft_entry__.build())")
    lib = C.CDLL(L.LIB_PATH)
    names = _declared()
    assert set(names) >= set(L.EXPORTS)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert L.version().startswith("geek")


def test_struct_layouts_match_header(tmp_path):
    exe = tmp_path / "abi_layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "abi_layout.c"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    structs = {"geek_hash_job": L.HashJob, "geek_bucketize_job": L.BucketizeJob,
               "geek_silk_job": L.SilkJob, "geek_assign_job": L.AssignJob,
               "geek_regroup_job": L.RegroupJob, "geek_quantile_job": L.QuantileJob}
    n = 0
    for line in out.splitlines():
        sname, field, val = line.split()
        cls = structs[sname]
        if field == "sizeof":
            assert C.sizeof(cls) == int(val), sname
        else:
            assert getattr(cls, field).offset == int(val), (sname, field)
        n += 1
    assert n > 60


def test_argument_errors_need_no_gpu():
    lib = L.lib()
    nb = C.c_size_t(0)
    bad = L.BucketizeJob(n=0, T=1, key_words=4)
    assert lib.geek_workspace_size(L.GEEK_OP_BUCKETIZE, C.byref(bad), 1, C.byref(nb)) == L.GEEK_ERR_ARG
    bad = L.AssignJob(metric=L.GEEK_METRIC_EUCLID, n=10, d=300, k=1, X=16, ldx=300,
                      seed_offsets=16, seed_members=16, assign=16, sse=16, centroids=16)
    assert lib.geek_workspace_size(L.GEEK_OP_ASSIGN, C.byref(bad), 1, C.byref(nb)) == L.GEEK_ERR_UNSUPPORTED
    bad = L.HashJob(kind=L.GEEK_HASH_DENSE, n=10, d=4, X=16, ldx=4, A=16, b=16, m=33, L=1, w=1.0, keys=16)
    assert lib.geek_workspace_size(L.GEEK_OP_HASH, C.byref(bad), 1, C.byref(nb)) == L.GEEK_ERR_UNSUPPORTED
    bad = L.HashJob(kind=L.GEEK_HASH_DENSE, n=10, d=4, X=16, ldx=4, A=16, b=16, m=4, L=1, w=0.0, keys=16)
    assert lib.geek_hash(C.byref(bad), 1, None, 0, None, None) == L.GEEK_ERR_ARG
    bad = L.HashJob(kind=L.GEEK_HASH_DOPH, n=10, F=4097, offsets=16, tokens=16, mh_keys=16, sig=16)
    assert lib.geek_workspace_size(L.GEEK_OP_HASH, C.byref(bad), 1, C.byref(nb)) == L.GEEK_ERR_UNSUPPORTED
    bad = L.HashJob(kind=L.GEEK_HASH_DOPH, n=10, F=400, offsets=16, tokens=16, mh_keys=None, sig=16)
    assert lib.geek_hash(C.byref(bad), 1, None, 0, None, None) == L.GEEK_ERR_ARG
    bad = L.HashJob(kind=7, n=10, F=400, offsets=16, tokens=16, mh_keys=16, sig=16)
    assert lib.geek_hash(C.byref(bad), 1, None, 0, None, None) == L.GEEK_ERR_ARG
    # a device-side seed count: Euclidean jobs only, one job per call
    bad = L.AssignJob(metric=L.GEEK_METRIC_SIG, n=10, k=2, sig=16, F=8, modes=16, n_members=2,
                      seed_offsets=16, seed_members=16, assign=16, sse=16, k_dev=16)
    assert lib.geek_assign(C.byref(bad), 1, C.c_void_p(256), 1 << 20, None, None) == L.GEEK_ERR_ARG
    two = (L.AssignJob * 2)(*[L.AssignJob(metric=L.GEEK_METRIC_EUCLID, n=10, d=4, k=2, X=16, ldx=4,
                                          seed_offsets=16, seed_members=16, assign=16, sse=16,
                                          centroids=16, k_dev=16) for _ in range(2)])
    assert lib.geek_assign(two, 2, C.c_void_p(256), 1 << 20, None, None) == L.GEEK_ERR_ARG
    assert lib.geek_status_string(L.GEEK_ERR_RANGE).decode() == "value outside the packable range"
    ok = L.BucketizeJob(n=1000, T=3, key_words=4, keys=16, table_stride=4000, row_stride=4,
                        members=16, offsets=16, nbuckets=16)
    assert lib.geek_workspace_size(L.GEEK_OP_BUCKETIZE, C.byref(ok), 1, C.byref(nb)) == 0
    assert nb.value > 3 * 1000 * 20
    # a too-small workspace is refused before any launch
    assert lib.geek_bucketize(C.byref(ok), 1, C.c_void_p(256), 16, None, None) == L.GEEK_ERR_WORKSPACE
    bad = L.RegroupJob(n=10, k=0, assign=16, seed_offsets=16, seed_members=16, k_out=16)
    assert lib.geek_workspace_size(L.GEEK_OP_REGROUP, C.byref(bad), 1, C.byref(nb)) == L.GEEK_ERR_ARG
    bad = L.RegroupJob(n=10, k=3, assign=None, seed_offsets=16, seed_members=16, k_out=16)
    assert lib.geek_regroup(C.byref(bad), 1, C.c_void_p(256), 1 << 20, None, None) == L.GEEK_ERR_ARG
    ok = L.RegroupJob(n=1000, k=3, assign=16, seed_offsets=16, seed_members=16, k_out=16)
    assert lib.geek_workspace_size(L.GEEK_OP_REGROUP, C.byref(ok), 1, C.byref(nb)) == 0
    assert nb.value >= 5 * 1000 * 4
    assert lib.geek_regroup(C.byref(ok), 1, C.c_void_p(256), 16, None, None) == L.GEEK_ERR_WORKSPACE
    bad = L.QuantileJob(n=10, d=4, m=2, t=11, X=16, ldx=4, A=16, members=16, offsets=16)
    assert lib.geek_workspace_size(L.GEEK_OP_QUANTILE, C.byref(bad), 1, C.byref(nb)) == L.GEEK_ERR_ARG
    bad = L.QuantileJob(n=10, d=300, m=2, t=3, X=16, ldx=300, A=16, members=16, offsets=16)
    assert lib.geek_workspace_size(L.GEEK_OP_QUANTILE, C.byref(bad), 1, C.byref(nb)) == L.GEEK_ERR_UNSUPPORTED
    ok = L.QuantileJob(n=10, d=4, m=2, t=3, X=16, ldx=4, A=16, members=16, offsets=16)
    assert lib.geek_quantile_buckets(C.byref(ok), 1, C.c_void_p(256), 16, None, None) == L.GEEK_ERR_WORKSPACE


def test_scan_tile_table_host_only(tmp_path):
    # the tile table of the batched first pass is host state: validated and
    # installed without touching a GPU; saved tables round-trip
    from paper_2106_10515_amd import autotune

    saved = {(p, dp): L.geek_get_scan_tiles(p, dp) for p in (0, 1, 2) for dp in (32, 64, 128, 256)}
    try:
        for p in (0, 1, 2):
            assert L.geek_set_scan_tiles(p, 128, 0, 0, 0) == L.GEEK_OK
        assert L.geek_get_scan_tiles(L.GEEK_PREC_BF16, 128) == (2, 2, 8)
        assert L.geek_get_scan_tiles(L.GEEK_PREC_FP32, 128) == (1, 1, 8)
        assert L.geek_set_scan_tiles(L.GEEK_PREC_BF16, 128, 1, 2, 4) == L.GEEK_OK
        assert L.geek_get_scan_tiles(L.GEEK_PREC_BF16, 128) == (1, 2, 4)
        assert L.geek_set_scan_tiles(L.GEEK_PREC_BF16, 48, 1, 1, 4) == L.GEEK_ERR_ARG
        assert L.geek_set_scan_tiles(L.GEEK_PREC_BF16, 128, 1, 1, 65) == L.GEEK_ERR_ARG
        assert L.geek_set_scan_tiles(7, 128, 1, 1, 4) == L.GEEK_ERR_ARG
        assert L.geek_set_scan_tiles(L.GEEK_PREC_BF16, 128, 3, 1, 4) == L.GEEK_ERR_UNSUPPORTED
        assert L.geek_set_scan_tiles(L.GEEK_PREC_FP32, 128, 2, 1, 4) == L.GEEK_ERR_UNSUPPORTED
        assert L.geek_set_scan_tiles(L.GEEK_PREC_FP32, 64, 2, 1, 4) == L.GEEK_OK
        assert len(autotune.candidates(L.GEEK_PREC_BF16, 256)) == 16
        assert len(autotune.candidates(L.GEEK_PREC_FP32, 256)) == 8
        assert [autotune.padded_depth(d) for d in (1, 32, 33, 100, 256)] == [32, 32, 64, 128, 256]
        res = {L.GEEK_PREC_FP8: {64: {"best": (1, 2, 16), "ms": {(1, 2, 16): 0.5, (2, 2, 8): 0.7}}}}
        path = str(tmp_path / "tiles.json")
        autotune.save_table(res, path)
        assert autotune.install_table(path) == 1
        assert L.geek_get_scan_tiles(L.GEEK_PREC_FP8, 64) == (1, 2, 16)
    finally:
        for (p, dp), shape in saved.items():
            L.geek_set_scan_tiles(p, dp, *shape)
