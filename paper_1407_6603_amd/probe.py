"""Roofline probes (libbsort_probe.so, include/bsort_probe.h): the issue
rates of the vector forms of a compare-exchange, the cross-lane row move,
and LDS and HBM bandwidth, measured on every CU of the current GPU.

``peaks()`` runs each probe a few times and returns the best rate of each;
the benchmark prices its kernels against these measured ceilings beside the
published ones."""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime first, as for libbsort)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbsort_probe.so")

F64_MINMAX, U32_MINMAX, U64_CMP_SELECT, DPP_MOVE, U32_ADD = 0, 1, 2, 3, 4
LDS_READ, LDS_WRITE, HBM_READ, HBM_COPY = 5, 6, 7, 8
EXPORTS = ["bsort_probe_run"]

# (name, probe, iterations, unit of the rate)
PROBES = [
    ("f64_minmax", F64_MINMAX, 4000, "lane instructions/s (v_min_f64, v_max_f64)"),
    ("u32_minmax", U32_MINMAX, 4000, "lane instructions/s (v_min_u32, v_max_u32)"),
    ("u32_add", U32_ADD, 4000, "lane instructions/s (v_add_u32)"),
    ("u64_cmp_select", U64_CMP_SELECT, 4000, "compare-exchanges/s (64-bit compares, 4 selects)"),
    ("dpp_move", DPP_MOVE, 4000, "lane instructions/s (v_mov_b32 row moves)"),
    ("lds_read", LDS_READ, 200, "bytes/s (ds_read_b128)"),
    ("lds_write", LDS_WRITE, 200, "bytes/s (ds_write_b128)"),
    ("hbm_read", HBM_READ, 4, "bytes/s (global_load_dwordx4 stream, 2 GiB)"),
    ("hbm_copy", HBM_COPY, 4, "bytes/s read plus written (2 x 1 GiB)"),
]

_lib = None


def load(path: str = LIB_PATH):
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_1407_6603_amd.build`")
        L = ctypes.CDLL(path)
        L.bsort_probe_run.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_size_t, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
        L.bsort_probe_run.restype = ctypes.c_int
        _lib = L
    return _lib


def run(probe: int, iters: int, scratch: "torch.Tensor"):
    """(milliseconds, units) of one run of a probe on the current stream."""
    ms, units = ctypes.c_double(), ctypes.c_double()
    rc = load().bsort_probe_run(probe, int(iters), scratch.data_ptr(), scratch.numel(),
                                ctypes.byref(ms), ctypes.byref(units),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise RuntimeError(f"probe {probe} failed ({rc})")
    return ms.value, units.value


def peaks(reps: int = 3, scratch_bytes: int = (2 << 30) + (32 << 20)):
    """Best rate of each probe over reps runs (after one warm-up run)."""
    if not torch.cuda.is_available():
        raise RuntimeError("the probes need a GPU")
    scratch = torch.zeros(scratch_bytes, dtype=torch.uint8, device="cuda")
    out = {}
    for name, p, iters, unit in PROBES:
        run(p, 1, scratch)
        best = 0.0
        for _ in range(reps):
            ms, units = run(p, iters, scratch)
            best = max(best, units / (ms * 1e-3))
        out[name] = {"rate": best, "unit": unit}
    del scratch
    return out


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="roofline probes on the current GPU")
    ap.add_argument("--only", default="", help="run one probe (by name) --reps times and "
                    "print each run's rate; default: the best rate of every probe")
    ap.add_argument("--iters", type=int, default=0, help="iterations (default: the table's)")
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    if not a.only:
        print(json.dumps(peaks(reps=a.reps), indent=1))
    else:
        row = [r for r in PROBES if r[0] == a.only]
        if not row:
            raise SystemExit(f"unknown probe {a.only}; one of {[r[0] for r in PROBES]}")
        name, p, iters, unit = row[0]
        scratch = torch.zeros((2 << 30) + (32 << 20) if name.startswith("hbm") else 64 << 20,
                              dtype=torch.uint8, device="cuda")
        for _ in range(a.reps):
            ms, units = run(p, a.iters or iters, scratch)
            print(json.dumps({"probe": name, "ms": ms, "rate": units / (ms * 1e-3),
                              "unit": unit}), flush=True)
