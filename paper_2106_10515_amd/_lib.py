"""ctypes binding of libgeek.so (see include/geek.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the data pass runs in the library's kernels.  There is
no CPU fallback: if the shared library is missing or fails to load, every
call raises ``GeekError``.
"""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgeek.so")

GEEK_OK = 0
GEEK_ERR_ARG = -1
GEEK_ERR_WORKSPACE = -2
GEEK_ERR_UNSUPPORTED = -3
GEEK_ERR_HIP = -4
GEEK_ERR_NONFINITE = 1
GEEK_ERR_RANGE = 2
GEEK_ERR_CAPACITY = 3
GEEK_ERR_NO_SEEDS = 4
GEEK_ERR_EMPTY_SET = 5
GEEK_ERR_KEYS = 6

GEEK_HASH_DENSE, GEEK_HASH_SETS, GEEK_HASH_HETERO, GEEK_HASH_DOPH = 0, 1, 2, 3
GEEK_METRIC_EUCLID, GEEK_METRIC_SIG, GEEK_METRIC_HETERO = 0, 1, 2
GEEK_PREC_FP32, GEEK_PREC_BF16, GEEK_PREC_FP8 = 0, 1, 2
GEEK_OP_HASH, GEEK_OP_BUCKETIZE, GEEK_OP_SILK, GEEK_OP_ASSIGN, GEEK_OP_REGROUP = 0, 1, 2, 3, 4
GEEK_OP_QUANTILE = 5

P = C.c_void_p


class GeekError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        msg = f"{where}: geek status {code}"
        try:
            msg += f" ({_load().geek_status_string(code).decode()})"
            if code == GEEK_ERR_HIP:
                msg += f": {_load().geek_last_hip_error().decode()}"
        except Exception:  # library missing: keep the bare code
            pass
        super().__init__(msg)


class HashJob(C.Structure):
    _fields_ = [
        ("kind", C.c_int32), ("d", C.c_int32), ("n", C.c_int64),
        ("X", P), ("ldx", C.c_int64), ("A", P), ("b", P),
        ("m", C.c_int32), ("L", C.c_int32), ("w", C.c_float), ("F", C.c_int32),
        ("keys", P), ("codes", P), ("offsets", P), ("tokens", P),
        ("cat", P), ("n_cat", C.c_int32), ("pad0", C.c_int32),
        ("mh_keys", P), ("sig", P), ("n_fixup", P), ("key_fp", P),
    ]


class BucketizeJob(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("T", C.c_int32), ("key_words", C.c_int32),
        ("keys", P), ("table_stride", C.c_int64), ("row_stride", C.c_int64),
        ("members", P), ("offsets", P), ("nbuckets", P), ("bucket_of", P), ("key_fp", P),
    ]


class SilkJob(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("T", C.c_int32), ("K", C.c_int32),
        ("members", P), ("offsets", P), ("nbuckets", P),
        ("L", C.c_int32), ("delta", C.c_int32), ("silk_keys", P),
        ("cap_k", C.c_int64), ("cap_members", C.c_int64),
        ("seed_offsets", P), ("seed_members", P), ("k_out", P), ("needed", P), ("counters", P),
        ("cap_c", C.c_int64),
    ]


class AssignJob(C.Structure):
    _fields_ = [
        ("metric", C.c_int32), ("precision", C.c_int32), ("n", C.c_int64),
        ("d", C.c_int32), ("k", C.c_int32), ("X", P), ("ldx", C.c_int64),
        ("sig", P), ("F", C.c_int32), ("n_cat", C.c_int32), ("cat", P), ("gamma", C.c_double),
        ("seed_offsets", P), ("seed_members", P), ("assign", P), ("centroids", P),
        ("modes", P), ("dist", P), ("sse", P), ("radius", P), ("counters", P),
        ("n_members", C.c_int64), ("t_done", P), ("k_dev", P),
    ]


class RegroupJob(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("k", C.c_int32), ("pad0", C.c_int32), ("assign", P),
        ("seed_offsets", P), ("seed_members", P), ("k_out", P), ("label_of", P),
    ]


class QuantileJob(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("d", C.c_int32), ("m", C.c_int32), ("t", C.c_int32), ("pad0", C.c_int32),
        ("X", P), ("ldx", C.c_int64), ("A", P),
        ("members", P), ("offsets", P), ("bucket_of", P),
    ]


EXPORTS = ("geek_workspace_size", "geek_hash", "geek_bucketize", "geek_silk_seeds",
           "geek_assign", "geek_regroup", "geek_quantile_buckets", "geek_status_string", "geek_version", "geek_last_hip_error",
           "geek_profile", "geek_profile_read", "geek_wallclock_hz", "geek_set_scan_tiles",
           "geek_get_scan_tiles", "geek_hash_noalloc")

GEEK_PROF_E2LSH, GEEK_PROF_BUCKETIZE, GEEK_PROF_ASSIGN_SCAN, GEEK_PROF_ASSIGN = 0, 1, 2, 3
GEEK_PROF_MINHASH, GEEK_PROF_SILK, GEEK_PROF_BZ_SORT = 4, 5, 6

_LIB = None


def _load():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise GeekError(GEEK_ERR_HIP, f"libgeek.so not built at {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    lib.geek_workspace_size.argtypes = [C.c_int32, P, C.c_int32, C.POINTER(C.c_size_t)]
    lib.geek_workspace_size.restype = C.c_int32
    for name, jt in (("geek_hash", HashJob), ("geek_bucketize", BucketizeJob),
                     ("geek_silk_seeds", SilkJob), ("geek_assign", AssignJob),
                     ("geek_regroup", RegroupJob), ("geek_quantile_buckets", QuantileJob)):
        f = getattr(lib, name)
        f.argtypes = [C.POINTER(jt), C.c_int32, P, C.c_size_t, P, P]
        f.restype = C.c_int32
    lib.geek_hash_noalloc.argtypes = [C.POINTER(HashJob), C.c_int32, P, P]
    lib.geek_hash_noalloc.restype = C.c_int32
    lib.geek_status_string.argtypes = [C.c_int32]
    lib.geek_status_string.restype = C.c_char_p
    lib.geek_version.restype = C.c_char_p
    lib.geek_last_hip_error.restype = C.c_char_p
    lib.geek_profile.argtypes = [C.c_int32]
    lib.geek_profile.restype = C.c_int32
    lib.geek_profile_read.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    lib.geek_profile_read.restype = C.c_int32
    lib.geek_wallclock_hz.restype = C.c_int64
    lib.geek_set_scan_tiles.argtypes = [C.c_int32] * 5
    lib.geek_set_scan_tiles.restype = C.c_int32
    lib.geek_get_scan_tiles.argtypes = [C.c_int32, C.c_int32] + [C.POINTER(C.c_int32)] * 3
    lib.geek_get_scan_tiles.restype = C.c_int32
    _LIB = lib
    # tile shapes measured by the autotuner, if a table was saved
    from . import autotune
    autotune.install_table(autotune.TABLE_PATH, missing_ok=True)
    return lib


def lib():
    """The loaded library (raises GeekError when it is not built)."""
    return _load()


def version() -> str:
    return _load().geek_version().decode()


def geek_profile(enable: bool) -> None:
    _load().geek_profile(1 if enable else 0)


def geek_profile_read(kernel_id: int):
    """(total milliseconds, number of launches) recorded for ``kernel_id``."""
    ms = C.c_double(0.0)
    cnt = C.c_int64(0)
    rc = _load().geek_profile_read(kernel_id, C.byref(ms), C.byref(cnt))
    if rc != GEEK_OK:
        raise GeekError(rc, "geek_profile_read")
    return float(ms.value), int(cnt.value)


def geek_wallclock_hz() -> int:
    """Ticks per second of the device wall clock (t_done units)."""
    return int(_load().geek_wallclock_hz())


def geek_set_scan_tiles(precision: int, dp: int, ncb: int, nbuf: int, blocks_per_cu: int) -> int:
    """Install a tile shape of the batched first pass; returns the status."""
    return int(_load().geek_set_scan_tiles(precision, dp, ncb, nbuf, blocks_per_cu))


def geek_get_scan_tiles(precision: int, dp: int):
    """(ncb, nbuf, blocks_per_cu) currently used for (precision, dp)."""
    v = [C.c_int32(0) for _ in range(3)]
    rc = _load().geek_get_scan_tiles(precision, dp, *[C.byref(x) for x in v])
    if rc != GEEK_OK:
        raise GeekError(rc, "geek_get_scan_tiles")
    return tuple(int(x.value) for x in v)


def workspace_size(op: int, jobs) -> int:
    arr = (type(jobs[0]) * len(jobs))(*jobs)
    out = C.c_size_t(0)
    rc = _load().geek_workspace_size(op, C.cast(arr, P), len(jobs), C.byref(out))
    if rc != GEEK_OK:
        raise GeekError(rc, "geek_workspace_size")
    return int(out.value)


def _call(name, jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr):
    arr = (type(jobs[0]) * len(jobs))(*jobs)
    rc = getattr(_load(), name)(arr, len(jobs), ws_ptr, ws_bytes, status_ptr, stream_ptr)
    if rc != GEEK_OK:
        raise GeekError(rc, name)
    return rc


def geek_hash(jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr):
    return _call("geek_hash", jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr)


def geek_bucketize(jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr):
    return _call("geek_bucketize", jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr)


def geek_silk_seeds(jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr):
    return _call("geek_silk_seeds", jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr)


def geek_assign(jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr):
    return _call("geek_assign", jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr)


def geek_regroup(jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr):
    return _call("geek_regroup", jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr)


def geek_quantile_buckets(jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr):
    return _call("geek_quantile_buckets", jobs, ws_ptr, ws_bytes, status_ptr, stream_ptr)
