"""Launch-shape autotuner for the batched sort.

The knobs decide speed, never the result:

* the odd-even transposition tile size (``tile_keys``): sorting a tile costs
  about T/2 compare-exchanges per word, while a sub-array of n words sorted
  in LDS needs about n/T merge-split phases;
* where that tile applies (``BSORT_FLAG_LDS_TILE``): by default sub-arrays
  sorted in LDS use 512-word tiles for keys of up to 4 bytes (their tile
  sort is two fp64 instructions per compare-exchange) and, for longer keys,
  the tuned tile doubled until at most 16 phases remain; with the flag they
  use the tuned tile itself, so the dominant in-LDS classes are tuned too;
* the merge-split block width of sub-arrays merged through HBM
  (``hbm_tile_keys``): wider blocks mean fewer phases over the whole
  sub-array but bigger chunks to sort first.

``tune`` times every (tile, LDS-tile mode) pair at the default block width,
then the block width at the best pair, with eager batch sorts timed by HIP
events; it also times the longest in-LDS stage alone (every stage in order)
for each pair, so the record says how much each knob moved the dominant
kernel.  Every candidate must give the same bits.  The winner is stored in
a JSON cache keyed by GPU architecture and compute-unit count, per
workload.  Two workloads are tuned: the 4,096-list batch (no sub-array
reaches the HBM path there) and four 1,000,000-word requests of the serving
workload (their largest sub-arrays merge through HBM).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")
FLAG_LDS_TILE = 16                        # BSORT_FLAG_LDS_TILE
DEFAULT = (256, 0, 0)                     # (tile_keys, hbm_tile_keys, flags); 0 = library default
TILES = (128, 256, 512)
LDS_MODES = (0, FLAG_LDS_TILE)
HBM_TILES = (1024, 2048, 4096, 8192)


def device_key(arch: str, cus: int) -> str:
    return f"{arch}:{int(cus)}cu"


def current_device_key() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    arch = getattr(p, "gcnArchName", "gfx950").split(":")[0]
    return device_key(arch, p.multi_processor_count)


def load_cache(path: str = CACHE) -> Dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(workload: str, key: Optional[str] = None,
           path: str = CACHE) -> Tuple[int, int, int, str]:
    """(tile_keys, hbm_tile_keys, flags, source) for this device and workload."""
    key = key or current_device_key()
    entry = load_cache(path).get(key, {}).get(workload)
    if entry and "hbm_tile_keys" in entry:
        return (int(entry["tile_keys"]), int(entry["hbm_tile_keys"]), int(entry.get("flags", 0)),
                f"autotune cache ({key})")
    return DEFAULT[0], DEFAULT[1], DEFAULT[2], "default"


def _time(bs, torch, args, tile: int, hbm: int, flags: int, reps: int, dominant: str):
    bytes_t, offsets_t, req_t, h_req, max_len = args
    total = int(h_req[-1])
    ws = bs.Workspace(bs.workspace_bytes(total, max_len, len(h_req) - 1), offsets_t.device)
    out = torch.empty(total, dtype=torch.int32, device=offsets_t.device)
    tune = bs.tuning(tile, 0, flags, hbm)
    bs.sort_batch(bytes_t, offsets_t, req_t, h_req, max_len, tune, ws, out=out)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(reps):
        ev[0].record()
        bs.sort_batch(bytes_t, offsets_t, req_t, h_req, max_len, tune, ws, out=out)
        ev[1].record()
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    bs.check_device_status(ws)
    dom_ms = None
    if dominant:
        # the dominant stage alone: every stage in order on one stream
        timer = bs.StageTimer(max_len, only=[dominant])
        st = bs.tuning(tile, 0, flags | bs.FLAG_SERIAL_STAGES, hbm)
        d = []
        for _ in range(reps):
            bs.sort_batch_staged(bytes_t, offsets_t, req_t, h_req, max_len, timer, st, ws,
                                 out=out)
            d.append(timer.ms()[dominant])
        dom_ms = float(np.median(d))
    return float(np.median(ms)), dom_ms, out


def tune(bytes_t, offsets_t, req_t, h_req: np.ndarray, max_len: int, workload: str,
         tiles: Sequence[int] = TILES, modes: Sequence[int] = LDS_MODES,
         hbm_tiles: Sequence[int] = HBM_TILES, reps: int = 5, dominant: str = "",
         save: bool = True, path: str = CACHE, log=print) -> Dict:
    import torch
    import paper_1407_6603_amd as bs

    args = (bytes_t, offsets_t, req_t, np.ascontiguousarray(h_req, np.int64), max_len)
    sweep = []
    ref: Optional[np.ndarray] = None

    def run(tile, hbm, flags):
        nonlocal ref
        for s in sweep:
            if (s["tile_keys"], s["hbm_tile_keys"], s["flags"]) == (tile, hbm, flags):
                return s["ms"]
        ms, dom_ms, out = _time(bs, torch, args, tile, hbm, flags, reps, dominant)
        got = out.cpu().numpy()
        if ref is None:
            ref = got
        elif not np.array_equal(ref, got):
            raise AssertionError(f"tile={tile} hbm_tile={hbm} flags={flags} changed the result")
        sweep.append({"tile_keys": tile, "hbm_tile_keys": hbm, "flags": flags, "ms": ms,
                      "dominant_stage_ms": dom_ms})
        log(f"autotune {workload}: tile={tile:5d} lds_tile={'tuned' if flags else 'library'} "
            f"hbm_tile={hbm:5d} {ms:9.3f} ms"
            + (f"  {dominant} alone {dom_ms:.3f} ms" if dom_ms is not None else ""))
        return ms

    pairs = [(t, f) for f in modes for t in tiles]
    best_tile, best_flags = min(pairs, key=lambda p: run(p[0], DEFAULT[1], p[1]))
    best_hbm = min(list(hbm_tiles) + [DEFAULT[1]], key=lambda h: run(best_tile, h, best_flags))
    base = run(DEFAULT[0], DEFAULT[1], DEFAULT[2])
    entry = {"tile_keys": best_tile, "hbm_tile_keys": best_hbm, "flags": best_flags,
             "ms": run(best_tile, best_hbm, best_flags), "default_ms": base,
             "words": int(h_req[-1]), "dominant_stage": dominant, "sweep": sweep}
    if save:
        cache = load_cache(path)
        cache.setdefault(current_device_key(), {})[workload] = entry
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def workload_inputs(name: str, workers: int = 8):
    """Host arrays (Batch, max_len, dominant stage) of a tuning workload; call
    before the GPU is opened when workers > 1."""
    import wordgen
    if name == "batch4096":
        return wordgen.batch(workers=workers), 12, "lds_d2_16320"
    if name == "large4x1M":
        lists = [wordgen.serve_request(10_000 + i, 1_000_000) for i in range(4)]
        return wordgen.Batch.concat(lists), 32, "merge_split"
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
        batch, ml, dom = inputs[n]
        b_t, o_t = bs.to_device(batch.bytes, batch.offsets)
        r_t = torch.from_numpy(batch.req_start).cuda()
        e = tune(b_t, o_t, r_t, batch.req_start, ml, n, path=a.out, dominant=dom)
        print(json.dumps({k: v for k, v in e.items() if k != "sweep"}), flush=True)
        del b_t, o_t, r_t
