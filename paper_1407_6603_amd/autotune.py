"""Launch-shape autotuner for the batched sort.

Two knobs decide speed, never the result:

* the odd-even transposition tile size (``tile_keys``): sorting a tile costs
  about T/2 compare-exchanges per word, while a sub-array of n words sorted
  in LDS needs about n/T merge-split phases;
* the merge-split block width of sub-arrays merged through HBM
  (``hbm_tile_keys``): wider blocks mean fewer phases over the whole
  sub-array but bigger chunks to sort first.

``tune`` times candidates on a real workload with eager batch sorts: first
the tile size at the default block width, then the block width at the best
tile size.  It checks that every candidate gives the same bits, and stores
the winner in a JSON cache keyed by device name and workload.  ``lookup``
reads that cache.  Two workloads are tuned: the 4,096-list batch (no
sub-array reaches the HBM path there) and four 1,000,000-word requests of
the serving workload (their largest sub-arrays merge through HBM).
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")
DEFAULT = (256, 0)                       # (tile_keys, hbm_tile_keys); 0 = library default
TILES = (128, 256, 512)
HBM_TILES = (1024, 2048, 4096, 8192)


def _device_key(device_name: str) -> str:
    return f"{device_name} gfx950"


def load_cache(path: str = CACHE) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(device_name: str, workload: str, path: str = CACHE) -> Tuple[int, int, str]:
    """(tile_keys, hbm_tile_keys, source) for this device and workload."""
    entry = load_cache(path).get(_device_key(device_name), {}).get(workload)
    if entry and "hbm_tile_keys" in entry:
        return int(entry["tile_keys"]), int(entry["hbm_tile_keys"]), "autotune cache"
    return DEFAULT[0], DEFAULT[1], "default"


def _time(bs, torch, args, tile: int, hbm: int, reps: int):
    bytes_t, offsets_t, req_t, h_req, max_len = args
    total = int(h_req[-1])
    ws = bs.Workspace(bs.workspace_bytes(total, max_len, len(h_req) - 1), offsets_t.device)
    out = torch.empty(total, dtype=torch.int32, device=offsets_t.device)
    tune = bs.tuning(tile, 0, 0, hbm)
    bs.sort_batch(bytes_t, offsets_t, req_t, h_req, max_len, tune, ws, out=out)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        bs.sort_batch(bytes_t, offsets_t, req_t, h_req, max_len, tune, ws, out=out)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    bs.check_device_status(ws)
    return best * 1e3, out


def tune(bytes_t, offsets_t, req_t, h_req: np.ndarray, max_len: int, workload: str,
         tiles: Sequence[int] = TILES, hbm_tiles: Sequence[int] = HBM_TILES,
         reps: int = 3, save: bool = True, path: str = CACHE, log=print) -> Dict:
    import torch
    import paper_1407_6603_amd as bs

    args = (bytes_t, offsets_t, req_t, np.ascontiguousarray(h_req, np.int64), max_len)
    sweep = []
    ref: Optional[np.ndarray] = None

    def run(tile, hbm):
        nonlocal ref
        for s in sweep:
            if s["tile_keys"] == tile and s["hbm_tile_keys"] == hbm:
                return s["ms"]
        ms, out = _time(bs, torch, args, tile, hbm, reps)
        got = out.cpu().numpy()
        if ref is None:
            ref = got
        elif not np.array_equal(ref, got):
            raise AssertionError(f"tile={tile} hbm_tile={hbm} changed the result")
        sweep.append({"tile_keys": tile, "hbm_tile_keys": hbm, "ms": ms})
        log(f"autotune {workload}: tile={tile:5d} hbm_tile={hbm:5d} {ms:9.3f} ms")
        return ms

    best_tile = min(tiles, key=lambda t: run(t, DEFAULT[1]))
    best_hbm = min(list(hbm_tiles) + [DEFAULT[1]], key=lambda h: run(best_tile, h))
    entry = {"tile_keys": best_tile, "hbm_tile_keys": best_hbm,
             "ms": run(best_tile, best_hbm), "words": int(h_req[-1]), "sweep": sweep}
    if save:
        cache = load_cache(path)
        cache.setdefault(_device_key(torch.cuda.get_device_name(0)), {})[workload] = entry
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def workload_inputs(name: str, workers: int = 8):
    """Host arrays (Batch, max_len) of a tuning workload; call before the GPU
    is opened when workers > 1."""
    import wordgen
    if name == "batch4096":
        return wordgen.batch(workers=workers), 12
    if name == "large4x1M":
        lists = [wordgen.serve_request(10_000 + i, 1_000_000) for i in range(4)]
        return wordgen.Batch.concat(lists), 32
    raise ValueError(f"unknown tuning workload {name}")


if __name__ == "__main__":
    import argparse
    import sys

    sys.path.insert(0, os.path.dirname(HERE))
    ap = argparse.ArgumentParser(description="tune the batched sort on this GPU")
    ap.add_argument("--workload", action="append", default=None,
                    help="batch4096 and/or large4x1M (default: both)")
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args()
    names = a.workload or ["batch4096", "large4x1M"]
    inputs = {n: workload_inputs(n) for n in names}     # before the GPU is opened
    import torch
    import paper_1407_6603_amd as bs
    for n in names:
        batch, ml = inputs[n]
        b_t, o_t = bs.to_device(batch.bytes, batch.offsets)
        r_t = torch.from_numpy(batch.req_start).cuda()
        e = tune(b_t, o_t, r_t, batch.req_start, ml, n, path=a.out)
        print(json.dumps({k: v for k, v in e.items() if k != "sweep"}), flush=True)
        del b_t, o_t, r_t
