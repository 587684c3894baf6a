"""ctypes declarations of the libbsort C ABI (include/bsort.h).

torch is imported before the library is opened so that the process holds a
single HIP runtime: torch ships its own libamdhip64.so.7, and libbsort's
dependency on that soname then resolves to the copy torch already loaded.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded first, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsort.so")

BSORT_MAX_LEN = 64
STATUS = {0: "BSORT_OK", 1: "BSORT_E_INVALID", 2: "BSORT_E_TOO_LONG", 3: "BSORT_E_NO_MEMORY",
          4: "BSORT_E_WORKSPACE", 5: "BSORT_E_HIP", 6: "BSORT_E_CAPACITY"}
FLAG_PER_BUCKET_LAUNCH = 1
FLAG_TILES_ONLY = 2
FLAG_SERIAL_STAGES = 4
FLAG_STALL_TEST = 8
FLAG_LDS_TILE = 16
KEY_BYTES, KEY_LENGTH, KEY_LENGTH_BYTES = 0, 1, 2
LAYOUT_PACKED, LAYOUT_TEXT = 0, 1

EXPORTS = [
    "bsort_workspace_bytes", "bsort_bucketize", "bsort_sort_buckets", "bsort_sort_batch",
    "bsort_plan_create", "bsort_plan_workspace_bytes", "bsort_plan_execute",
    "bsort_plan_destroy", "bsort_stage_count", "bsort_stage_name", "bsort_sort_batch_staged",
    "bsort_get_device_status", "bsort_status_string",
    "bsort_last_error", "bsort_version", "bsort_tokenize_workspace_bytes", "bsort_tokenize",
    "bsort_fixed_width", "bsort_oets_buckets", "bsort_sort_batch_static",
]
STATIC_SCRATCH_BYTES = 64 << 20


class Words(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_void_p), ("n_bytes", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("n_words", ctypes.c_int32),
                ("max_len", ctypes.c_int32)]


class Buckets(ctypes.Structure):
    _fields_ = [("counts", ctypes.c_void_p), ("starts", ctypes.c_void_p),
                ("order", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_keys", ctypes.c_int32), ("merge_threads", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("hbm_tile_keys", ctypes.c_int32)]


class Batch(ctypes.Structure):
    _fields_ = [("bytes", ctypes.c_void_p), ("n_bytes", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("req_start", ctypes.c_void_p),
                ("h_req_start", ctypes.c_void_p), ("n_requests", ctypes.c_int32),
                ("max_len", ctypes.c_int32)]


class BsortError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Open libbsort.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_1407_6603_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(path)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.bsort_workspace_bytes.argtypes = [i64, i32, i32]
    L.bsort_workspace_bytes.restype = sz
    L.bsort_bucketize.argtypes = [ctypes.POINTER(Words), ctypes.POINTER(Buckets), P, sz, P]
    L.bsort_sort_buckets.argtypes = [ctypes.POINTER(Words), ctypes.POINTER(Buckets), P,
                                     ctypes.POINTER(Tuning), P, sz, P]
    L.bsort_sort_batch.argtypes = [ctypes.POINTER(Batch), P, ctypes.POINTER(Tuning), P, sz, P]
    L.bsort_plan_create.argtypes = [ctypes.POINTER(P), i64, i32, i64, i32,
                                    ctypes.POINTER(Tuning), P]
    L.bsort_plan_workspace_bytes.argtypes = [P]
    L.bsort_plan_workspace_bytes.restype = sz
    L.bsort_plan_execute.argtypes = [P, ctypes.POINTER(Batch), P, P, sz, P]
    L.bsort_plan_destroy.argtypes = [P]
    L.bsort_plan_destroy.restype = None
    L.bsort_stage_count.argtypes = [i32]
    L.bsort_stage_count.restype = ctypes.c_int
    L.bsort_stage_name.argtypes = [i32, ctypes.c_int]
    L.bsort_stage_name.restype = ctypes.c_char_p
    L.bsort_sort_batch_staged.argtypes = [ctypes.POINTER(Batch), P, ctypes.POINTER(Tuning), P,
                                          sz, P, ctypes.POINTER(P), ctypes.c_int]
    L.bsort_sort_batch_staged.restype = ctypes.c_int
    L.bsort_get_device_status.argtypes = [P, P]
    L.bsort_tokenize_workspace_bytes.argtypes = [i64]
    L.bsort_tokenize_workspace_bytes.restype = sz
    L.bsort_tokenize.argtypes = [P, i64, P, P, i64, P, P, sz, P]
    L.bsort_tokenize.restype = ctypes.c_int
    L.bsort_fixed_width.argtypes = [P, i64, P, i64, i32, i32, P, P, P, P]
    L.bsort_fixed_width.restype = ctypes.c_int
    L.bsort_oets_buckets.argtypes = [ctypes.POINTER(Words), ctypes.POINTER(Buckets), P, i32, P, P]
    L.bsort_oets_buckets.restype = ctypes.c_int
    L.bsort_sort_batch_static.argtypes = [ctypes.POINTER(Batch), P, ctypes.POINTER(Tuning), P, P]
    L.bsort_sort_batch_static.restype = ctypes.c_int
    for f in (L.bsort_bucketize, L.bsort_sort_buckets, L.bsort_sort_batch,
              L.bsort_plan_create, L.bsort_plan_execute, L.bsort_get_device_status):
        f.restype = ctypes.c_int
    L.bsort_status_string.argtypes = [ctypes.c_int]
    L.bsort_status_string.restype = ctypes.c_char_p
    L.bsort_last_error.argtypes = []
    L.bsort_last_error.restype = ctypes.c_char_p
    L.bsort_version.argtypes = []
    L.bsort_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int):
    if status != 0:
        detail = load().bsort_last_error().decode(errors="replace")
        raise BsortError(status, detail)
