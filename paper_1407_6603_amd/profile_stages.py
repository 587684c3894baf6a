"""Stage times of the batch workload for profiling: every stage alone, in
order on one stream (``BSORT_FLAG_SERIAL_STAGES``), timed with HIP events,
either in full or with the merge-split phases skipped
(``BSORT_FLAG_TILES_ONLY``, every tile of the given size).  Run it under
``rocprofv3`` to read counters per kernel of one mode:

    python -m paper_1407_6603_amd.profile_stages --mode full --reps 2
    python -m paper_1407_6603_amd.profile_stages --mode tiles_only --tile 512

Prints one JSON line per mode: the median milliseconds of every tile and
in-LDS stage over ``--reps`` sorts (after one untimed sort).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--mode", choices=("full", "tiles_only", "both"), default="both")
    ap.add_argument("--tile", type=int, default=512,
                    help="tile size of tiles_only (the in-LDS classes of two-dword "
                         "records sort 512-word tiles in full mode)")
    ap.add_argument("--full-tile", type=int, default=128, help="tuned tile of full mode")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--gen-workers", type=int, default=8,
                    help="generator processes (1 under a profiler)")
    a = ap.parse_args()

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import wordgen
    batch = wordgen.batch(workers=a.gen_workers)      # before the GPU is opened
    import torch
    import paper_1407_6603_amd as bs

    b_t, o_t = bs.to_device(batch.bytes, batch.offsets)
    rs = torch.from_numpy(batch.req_start).cuda()
    ml = 12
    ws = bs.Workspace(bs.workspace_bytes(batch.total, ml, batch.R))
    out = torch.empty(batch.total, dtype=torch.int32, device="cuda")
    names = [n for n in bs.stage_names(ml) if n.startswith(("lds_", "tiles"))]
    modes = ("full", "tiles_only") if a.mode == "both" else (a.mode,)
    for mode in modes:
        flags = bs.FLAG_SERIAL_STAGES | (bs.FLAG_TILES_ONLY if mode == "tiles_only" else 0)
        tune = bs.tuning(a.tile if mode == "tiles_only" else a.full_tile, 0, flags, 0)
        timers = [bs.StageTimer(ml, only=names) for _ in range(a.reps + 1)]
        for t in timers:
            bs.sort_batch_staged(b_t, o_t, rs, batch.req_start, ml, t, tune, ws, out=out)
        bs.check_device_status(ws)
        ms = {n: float(np.median([t.ms()[n] for t in timers[1:]])) for n in names}
        print(json.dumps({"mode": mode, "tile": a.tile if mode == "tiles_only" else a.full_tile,
                          "stage_ms": {k: round(v, 4) for k, v in ms.items()}}), flush=True)


if __name__ == "__main__":
    main()
