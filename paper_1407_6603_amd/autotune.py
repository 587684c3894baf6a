"""Launch-shape autotuner for the batched sort.

Two knobs decide speed, never the result: the odd-even transposition tile
size (words per tile; sorting a tile costs ~T/2 compare-exchanges per word,
while a sub-array of n words needs ceil(n/T) merge-split phases) and the
number of threads per merge-split workgroup.  ``tune`` times candidate
(tile, threads) pairs on a real batch with a captured plan -- first the tile
size at a fixed width, then the width at the best tile size -- checks that
every candidate gives the same bits, and stores the winner in a JSON cache
keyed by device name and workload.  ``lookup`` reads that cache.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")
DEFAULT = (256, 256)
TILES = (128, 256, 512)
MERGE_THREADS = (64, 128, 256, 512, 1024)


def _device_key(device_name: str) -> str:
    return f"{device_name} gfx950"


def load_cache(path: str = CACHE) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(device_name: str, workload: str, path: str = CACHE) -> Tuple[int, int, str]:
    """(tile_keys, merge_threads, source) for this device and workload."""
    entry = load_cache(path).get(_device_key(device_name), {}).get(workload)
    if entry:
        return int(entry["tile_keys"]), int(entry["merge_threads"]), "autotune cache"
    return DEFAULT[0], DEFAULT[1], "default"


def _time_plan(bs, torch, args, tile: int, mt: int, reps: int):
    bytes_t, offsets_t, req_t, h_req, max_len = args
    total = int(h_req[-1])
    cap_req = int(np.diff(h_req).max())
    plan = bs.Plan(total, len(h_req) - 1, cap_req, max_len, bs.tuning(tile, mt))
    ws = bs.Workspace(plan.workspace_bytes, offsets_t.device)
    out = torch.empty(total, dtype=torch.int32, device=offsets_t.device)
    plan.execute(bytes_t, offsets_t, req_t, h_req, ws, out=out)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        plan.execute(bytes_t, offsets_t, req_t, h_req, ws, out=out)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    bs.check_device_status(ws)
    plan.close()
    return best * 1e3, out


def tune(bytes_t, offsets_t, req_t, h_req: np.ndarray, max_len: int, workload: str,
         tiles: Sequence[int] = TILES, merge_threads: Sequence[int] = MERGE_THREADS,
         reps: int = 3, save: bool = True, path: str = CACHE, log=print) -> Dict:
    import torch
    import paper_1407_6603_amd as bs

    args = (bytes_t, offsets_t, req_t, np.ascontiguousarray(h_req, np.int64), max_len)
    sweep = []
    ref: Optional[np.ndarray] = None

    def run(tile, mt):
        nonlocal ref
        ms, out = _time_plan(bs, torch, args, tile, mt, reps)
        got = out.cpu().numpy()
        if ref is None:
            ref = got
        elif not np.array_equal(ref, got):
            raise AssertionError(f"tile={tile} threads={mt} changed the result")
        sweep.append({"tile_keys": tile, "merge_threads": mt, "ms": ms})
        log(f"autotune {workload}: tile={tile:5d} threads={mt:5d} {ms:9.3f} ms")
        return ms

    mt0 = DEFAULT[1]
    best_tile = min(tiles, key=lambda t: run(t, mt0))
    best_mt = min(merge_threads, key=lambda m: run(best_tile, m) if m != mt0 else
                  next(s["ms"] for s in sweep if s["tile_keys"] == best_tile and
                       s["merge_threads"] == mt0))
    best = min((s for s in sweep if s["tile_keys"] == best_tile and s["merge_threads"] == best_mt),
               key=lambda s: s["ms"])
    entry = {"tile_keys": best_tile, "merge_threads": best_mt, "ms": best["ms"],
             "words": int(h_req[-1]), "sweep": sweep}
    if save:
        cache = load_cache(path)
        cache.setdefault(_device_key(torch.cuda.get_device_name(0)), {})[workload] = entry
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


if __name__ == "__main__":
    import argparse
    import sys

    sys.path.insert(0, os.path.dirname(HERE))
    import torch
    import wordgen
    import paper_1407_6603_amd as bs

    ap = argparse.ArgumentParser(description="tune the batched sort on this GPU")
    ap.add_argument("--workload", default="batch4096")
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args()
    batch = wordgen.batch(workers=8)       # before the GPU is opened
    b_t, o_t = bs.to_device(batch.bytes, batch.offsets)
    r_t = torch.from_numpy(batch.req_start).cuda()
    e = tune(b_t, o_t, r_t, batch.req_start, 12, a.workload, path=a.out)
    print(json.dumps({k: v for k, v in e.items() if k != "sweep"}))
