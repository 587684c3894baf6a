"""Length-bucketed odd-even transposition sort of words on AMD MI355X.

The GPU work lives in libbsort.so (HIP, gfx950; C ABI in include/bsort.h).
This package is its Python binding: torch supplies device memory and
streams, and every step of the sort runs in the library's kernels.
"""
from .api import (BsortError, FLAG_LDS_TILE, FLAG_PER_BUCKET_LAUNCH, FLAG_SERIAL_STAGES,
                  FLAG_STALL_TEST, FLAG_TILES_ONLY,
                  KEY_BYTES, KEY_LENGTH, KEY_LENGTH_BYTES, LAYOUT_PACKED, LAYOUT_TEXT, MAX_LEN,
                  STATIC_SCRATCH_BYTES,
                  fixed_width, oets_buckets, StageTimer, Plan, Tuning,
                  Workspace, bucketize, check_device_status, device_status, sort, sort_batch,
                  sort_batch_static, sort_batch_staged, sort_buckets, sort_text, stage_names,
                  to_device, tokenize,
                  tuning, workspace_bytes)

__all__ = ["BsortError", "FLAG_LDS_TILE", "FLAG_PER_BUCKET_LAUNCH", "FLAG_SERIAL_STAGES",
           "FLAG_STALL_TEST", "FLAG_TILES_ONLY",
           "KEY_BYTES", "KEY_LENGTH", "KEY_LENGTH_BYTES", "LAYOUT_PACKED", "LAYOUT_TEXT",
           "STATIC_SCRATCH_BYTES",
           "fixed_width", "oets_buckets", "StageTimer", "MAX_LEN", "Plan", "Tuning",
           "Workspace", "bucketize", "check_device_status", "device_status", "sort", "sort_batch",
           "sort_batch_static", "sort_batch_staged", "sort_buckets", "sort_text", "stage_names", "to_device",
           "tokenize", "tuning", "workspace_bytes"]
