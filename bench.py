#!/usr/bin/env python3
"""Benchmark: words sorted per second (bit-exact), batched vs per-bucket launch.

Default workload: the batching workload -- 4,096 independent word lists with
sizes log-uniform in [16, 65,536] (~31.8 M words), each drawn like the small
single-list workload (800-word seeded vocabulary, lengths 1-12, Zipf 1.1,
5% capitalised).  A step sorts the whole batch: bucketize, key pack, tile
odd-even transposition sort and block merge-split for all lists, as one
batched call (a few launches per stage, not one per list); the same batch
through one captured graph launch is timed beside it.  Inputs are
device-resident before timing starts.

Prints one JSON line.  The roofline object prices the longest kernel of the
step: its algorithmic compare-exchange lane operations per launch (3 per
record dword per compare-exchange) over its measured launch time, against
the 32-bit vector ALU peak (256 CUs x 128 lanes/clock x 2.4 GHz).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import wordgen  # noqa: E402

# Peaks derived from the chip's unit counts and clock (256 CUs, 4 SIMDs of 16
# lanes each, 2.4 GHz).  A VALU instruction (32-bit, or a 64-bit min/max)
# issues one wave of 64 lanes per SIMD every 4 clocks: 64 lanes/clk/CU, 39.3 T
# lane-instructions/s (the fp64 vector FMA figure, 78.6 TFLOP/s, is that rate
# at 2 flops per FMA).  LDS: 128 B/clk/CU written and 256 B/clk/CU read
# (CDNA4 doubled the read path).  The probes in libbsort_probe measure each.
CLK_HZ = 2.4e9
VALU_TIPS = 256 * 64 * CLK_HZ / 1e12                # 39.3 T lane-instructions/s
PEAK_HBM_GBS = 8000.0
PEAK_LDS_READ_TBS = 256 * 256 * CLK_HZ / 1e12       # 157.3 TB/s
PEAK_LDS_WRITE_TBS = 256 * 128 * CLK_HZ / 1e12      # 78.6 TB/s


def ce_cost(D, L, in_lds):
    """VALU instructions per lane for one compare-exchange of records of D
    dwords (words of L bytes) in the form the library uses: a min and a max
    (v_min_u32/v_max_u32 on one-dword records of 1- and 2-byte words and
    3-byte words in LDS, v_min_f64/v_max_f64 on two-dword records and the
    two-dword form of 5- and 6-byte words in LDS): 2; otherwise a compare per
    key dword and two selects per dword: 3D - 1 (an estimate of the
    compiler's form)."""
    if D == 2 or (in_lds and D == 3 and L <= 6):
        return 2.0
    return 3.0 * D - 1.0


# HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE counter runs in
# profiles/batch4096_hbm_traffic.md (scaled by the plain-copy calibration
# there), with a digest of the kernel sources they were taken on: a kernel
# changed since then reports no traffic.
SORT_SOURCES = ("paper_1407_6603_amd/csrc/k_oets.hip", "paper_1407_6603_amd/csrc/bsort_internal.h")
TOK_SOURCES = ("paper_1407_6603_amd/csrc/k_tokenize.hip", "paper_1407_6603_amd/csrc/bsort_internal.h")
TRAFFIC = {
    "k_bucket_lds<2, 1024, 16320>": {"read": 66795065, "write": 22089840,
                                     "files": SORT_SOURCES, "sources": "803a2ebbb5cc19a2"},
    "k_bucket_lds<3, 1024, 8192>": {"read": 38552314, "write": 12720619,
                                    "files": SORT_SOURCES, "sources": "803a2ebbb5cc19a2"},
    "k_tok_count": {"read": 189711877, "write": 738000,
                    "files": TOK_SOURCES, "sources": "eb8edcd7ea267f4b"},
    "k_tok_scan": {"read": 109053, "write": 183712,
                   "files": TOK_SOURCES, "sources": "eb8edcd7ea267f4b"},
    "k_tok_write": {"read": 191245979, "write": 404112288,
                    "files": TOK_SOURCES, "sources": "eb8edcd7ea267f4b"},
}


def sources_digest(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    t = TRAFFIC.get(kernel)
    if t is None or t["sources"] != sources_digest(t["files"]):
        return None
    return t["read"] + t["write"]


def lds_threads(cap_index, D):
    if cap_index <= 1:
        return 256
    return 512 if (cap_index <= 3 and D <= 2) or cap_index == 2 or D >= 4 else 1024


def kernel_name(stage):
    """The kernel behind a tile or in-LDS stage name."""
    if stage.startswith("tiles_d"):
        return f"k_oets_tiles<{int(stage[7:])}>"
    D, cap = (int(x) for x in stage[5:].split("_"))
    c = lds_caps_for(D).index(cap)
    return f"k_bucket_lds<{D}, {lds_threads(c, D)}, {cap}>"


def kmax_for(D):
    return 64 if D <= 2 else 32 if D <= 4 else 16 if D <= 8 else 8 if D <= 16 else 4


LDS_BYTES = 144 * 1024
LDS_MAX_D = 9                     # widest record with in-LDS classes


def lds_caps_for(D):
    """Capacities of the in-LDS size classes for record width D (empty: none)."""
    if not 2 <= D <= LDS_MAX_D:
        return []
    top = 16320 if D <= 2 else 12288 if D == 3 else 9216 if D == 4 else 7168
    caps = [1024 << c for c in range(4)] + [top]
    return [c for c in caps if D * 4 * c <= LDS_BYTES]


def lds_tile(tuned, cap, D, fixed=False):
    """Tile size inside an in-LDS sub-array of class capacity cap (fixed:
    the tuned tile itself, BSORT_FLAG_LDS_TILE)."""
    if fixed:
        return min(tuned, 512)
    target = 512 if D <= 2 else cap // 16
    t = tuned
    while t < target and t < 512:
        t <<= 1
    return t


def hbm_chunk(D):
    """Tile of sub-arrays merged through HBM for record widths with in-LDS
    classes: the largest power of two whose pair of tiles fits 144 KiB."""
    c = 8192
    while c > 128 and 2 * c * 4 * D > LDS_BYTES - 2048:   # room for the window table
        c >>= 1
    return c


def tile_ce(n, T):
    """Compare-exchanges of odd-even transposition sorts of n words cut into
    tiles of T: n_t(n_t-1)/2 per tile."""
    full = n // T
    rest = n - full * T
    return full * (T * (T - 1) // 2) + rest * (rest - 1) // 2


def workload_structure(offsets, req_start, max_len, tile_keys, hbm_tile_keys, lds_fixed=False):
    """Host-side census of the work the method does on this input, routed as
    the library routes it: per record width D, the compare-exchanges of
    single-tile sub-arrays ('tiles_dD'), of tiles inside in-LDS sub-arrays
    and the LDS bytes their merge-split phases move (per size class of
    capacity C: 'lds_dD_C'), and the
    phases and bytes of the merge-split through HBM ('merge_split').
    Computed from word lengths only."""
    lens = np.diff(offsets)
    R = len(req_start) - 1
    rid = np.repeat(np.arange(R), np.diff(req_start))
    ml1 = max_len + 1
    counts = np.bincount(rid * ml1 + lens, minlength=R * ml1).reshape(R, ml1)
    out = {}
    merge_bytes = 0
    phases_max = 0
    for L in range(1, ml1):
        D = (L + 3) // 4 + 1
        W = (L + 7) // 8
        T = min(tile_keys, 64 * kmax_for(D), 512)
        Th = hbm_chunk(D) if D <= LDS_MAX_D else min(hbm_tile_keys, 64 * kmax_for(D))
        caps = lds_caps_for(D)
        cap = max(caps) if caps else 0
        n = counts[:, L].astype(np.int64)
        n = n[n >= 2]
        single = n[n <= T]
        hbm = n[(n > max(T, cap))]
        t = out.setdefault(f"tiles_d{D}", {"ce": 0, "words": 0, "D": D, "slots": 0.0})
        tce = int(tile_ce(single, T).sum()) + int(tile_ce(hbm, Th).sum())
        t["ce"] += tce
        t["slots"] += tce * ce_cost(D, L, False)
        t["words"] += int(single.sum()) + int(hbm.sum())
        lo = T
        for c in caps:
            lds = n[(n > lo) & (n <= c)]
            lo = max(lo, c)
            if not len(lds):
                continue
            Tc = lds_tile(T, c, D, lds_fixed)
            l = out.setdefault(f"lds_d{D}_{c}", {"ce": 0, "words": 0, "D": D, "lds_bytes": 0,
                                                 "buckets": 0, "tile": Tc, "slots": 0.0})
            l["buckets"] += int(len(lds))
            lce = int(tile_ce(lds, Tc).sum())
            l["ce"] += lce
            l["slots"] += lce * ce_cost(D, L, True)
            l["words"] += int(lds.sum())
            p = (lds + Tc - 1) // Tc
            # each phase reads and writes the paired part of the sub-array in LDS
            l["lds_bytes"] += int((2 * 4 * D * lds * p).sum())
        for nb in hbm:
            p = (int(nb) + Th - 1) // Th
            phases_max = max(phases_max, p)
            for s_ in range(p):
                for a in range(s_ & 1, p - 1, 2):
                    tot = Th + min(Th, int(nb) - (a + 1) * Th)
                    merge_bytes += 2 * tot * (8 * W + 4)
    return out, merge_bytes, phases_max


def cpu_info():
    n = len(os.sched_getaffinity(0))
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, model


METRIC = "words sorted/sec (bit-exact) batched vs per-bucket launch; p50/p99 request latency"
SERVE_DESC = ("serve: 2,000 Poisson arrivals at 2,000/s, sizes log-uniform in [1e3, 1e6] words, "
              "plus one 4,000,000-word request at arrival 1,000; lengths 1-32, Zipf 1.0 over one "
              "200,000-word vocabulary; 16 GB admission pool")


def check_sorted_on_device(bytes_h, offsets_h, req_start, perm_h, max_len):
    """Full-size validity check of a batch result with plain torch ops (no
    library kernel): every list's perm is a permutation of its indices and
    (length, bytes, index) strictly increases along it.  The result is
    unique, so this is its exact definition.  Returns the number of lists
    that fail."""
    import torch
    dev = torch.device("cuda")
    rs = torch.from_numpy(np.ascontiguousarray(req_start, np.int64)).to(dev)
    n = int(req_start[-1])
    if n == 0:
        return 0
    sizes = rs[1:] - rs[:-1]
    first = torch.repeat_interleave(rs[:-1], sizes)           # first word of each word's list
    local = torch.from_numpy(np.ascontiguousarray(perm_h)).to(dev).to(torch.int64)
    R = len(req_start) - 1
    bad = torch.zeros(R, dtype=torch.int64, device=dev)
    lid = torch.repeat_interleave(torch.arange(R, device=dev), sizes)
    inside = (local >= 0) & (local < sizes[lid])
    bad.index_add_(0, lid, (~inside).to(torch.int64))
    g = torch.where(inside, first + local, torch.zeros_like(local))
    count = torch.bincount(g, minlength=n)
    bad.index_add_(0, lid, (count != 1).to(torch.int64))
    offs = torch.from_numpy(np.ascontiguousarray(offsets_h, np.int64)).to(dev)
    buf = torch.from_numpy(np.ascontiguousarray(bytes_h)).to(dev)
    lo = offs[g]
    ln = offs[g + 1] - lo
    # keys: length, then 4-byte big-endian lanes (non-negative int64), then index
    lanes = []
    for w in range((max_len + 3) // 4):
        v = torch.zeros(n, dtype=torch.int64, device=dev)
        for j in range(4):
            k = 4 * w + j
            m = ln > k
            byte = buf[torch.where(m, lo + k, torch.zeros_like(lo))].to(torch.int64)
            v |= torch.where(m, byte, torch.zeros_like(byte)) << (24 - 8 * j)
        lanes.append(v)
    keys = [ln] + lanes + [local]
    lt = torch.zeros(n - 1, dtype=torch.bool, device=dev)
    eq = torch.ones(n - 1, dtype=torch.bool, device=dev)
    for k in keys:
        lt |= eq & (k[:-1] < k[1:])
        eq &= k[:-1] == k[1:]
    bad.index_add_(0, lid[:-1], ((lid[:-1] == lid[1:]) & ~lt).to(torch.int64))
    return int((bad > 0).sum())


SERVE_RATES = (1.0, 4.0, float("inf"))


def serve_run(sw, args):
    """The serving loop on the serve workload at wall-clock arrival times:
    admission by a 16 GB device arena (the pool), every admitted run of
    requests launched as one batch when one of 3 streams is free,
    host-to-device copies and result reads included.  Then the same requests
    offered faster (arrival times divided by 4, then all at once: the
    server's capacity).  Returns latency percentiles, words/s and parity (a
    full-size validity check of every request, and the definition oracle on
    sampled requests)."""
    import torch
    from paper_1407_6603_amd import serve
    b = sw.batch
    staging = serve.Staging(b.bytes, b.offsets, 32)
    from paper_1407_6603_amd import autotune
    tile, hbm, tflags, src = autotune.lookup("large4x1M", path=args.tune_cache or autotune.CACHE)
    ex = serve.GpuExecutor(staging, arena_bytes=16 << 30, streams=3,
                           tune=bs_tuning(tile, hbm, tflags))

    def requests(rate):
        return [serve.Request(i, float(sw.arrivals[i]) / rate if rate != float("inf") else 0.0,
                              int(b.req_start[i]), int(b.req_start[i + 1]),
                              int(b.offsets[b.req_start[i + 1]] - b.offsets[b.req_start[i]]))
                for i in range(b.R)]

    # warm-up: first launches on each stream (library load)
    serve.Server(ex).run(requests(1.0)[:20], keep_perms=False)
    torch.cuda.synchronize()
    legs = []
    st = None
    for rate in SERVE_RATES:
        srv = serve.Server(ex)
        res = srv.run(requests(rate), keep_perms=True)
        lst = serve.latency_stats(res)
        lst.update({"rate_multiplier": rate if rate != float("inf") else "all at once",
                    "batches": srv.batches, "pool_high_bytes": srv.pool_high})
        perm_all = np.concatenate([r.perm for r in res]) if res else np.zeros(0, np.int32)
        lst["lists_failing_check"] = check_sorted_on_device(b.bytes, b.offsets, b.req_start,
                                                            perm_all, 32)
        legs.append(lst)
        if st is None:
            st = dict(lst)
            sample_res = res
    st.update({"tile_keys": tile, "hbm_tile_keys": hbm or "default",
               "lds_tile": "tuned" if tflags & autotune.FLAG_LDS_TILE else "library",
               "tuning_source": src,
               "offered_words_per_s": float(b.total / max(sw.arrivals[-1], 1e-9)),
               "arena_bytes": ex.arena_bytes,
               "saturation": legs,
               "max_sustained_words_per_s": max(x["words_per_s"] for x in legs),
               "workload": SERVE_DESC + (f" (first {b.R} arrivals)" if args.serve_arrivals else "")})
    st["validity_check"] = {"requests_checked": b.R, "words_checked": int(b.total),
                            "what": "every request: perm is a permutation and (length, bytes, "
                                    "index) strictly increases along it (torch ops)",
                            "all_pass": all(x["lists_failing_check"] == 0 for x in legs)}
    if not args.no_cpu_baseline:
        import oracle
        pick = sorted(set(list(range(0, b.R, max(b.R // 64, 1))) + [min(1000, b.R - 1)]))
        ok = True
        for r in pick:
            w = b.request(r)
            ok &= bool(np.array_equal(sample_res[r].perm,
                                      oracle.definition_sort(w.bytes, w.offsets)))
        st["parity"] = {"requests_checked": len(pick),
                        "words_checked": int(sum(sample_res[r].n for r in pick)),
                        "bit_exact": ok,
                        "oracle": "definition (stable sort by length, bytes, index)"}
    return st


def bs_tuning(tile, hbm, flags=0):
    import paper_1407_6603_amd as bs
    return bs.tuning(tile, 0, flags, hbm)


def serve_line(sw, args, gen_s):
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    st = serve_run(sw, args)
    return {"metric": METRIC, "value": st["words_per_s"], "unit": "words/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": st["span_s"] * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
            "data": "synthetic", "config": {"workload": st.pop("workload")},
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "serving": st, "gen_seconds": gen_s}


def copy_calibration(mib):
    """A plain copy of mib MiB, three times: each launch reads and writes
    exactly mib MiB, so the HBM byte counters read for it give the scale
    between counter units and bytes."""
    import torch
    n = mib << 20
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)


CU_COUNTS = (8, 16, 32, 64, 128, 256)


def cu_child(args):
    """Child of the compute-unit scaling leg.  HSA_CU_MASK, set by the parent,
    limits this process's kernels to part of the GPU; time the serial-stage
    sort of the saved batch and print one JSON line."""
    import hashlib
    d = args.cu_data
    bytes_ = np.load(os.path.join(d, "bytes.npy"))
    offsets = np.load(os.path.join(d, "offsets.npy"))
    req = np.load(os.path.join(d, "req_start.npy"))
    import torch
    import paper_1407_6603_amd as bs
    from paper_1407_6603_amd import autotune
    tile, hbm, tflags = args.tile, args.hbm_tile, args.tune_flags
    if tile == 0 and hbm == 0:
        tile, hbm, tflags, _ = autotune.lookup("batch4096", path=args.tune_cache or autotune.CACHE)
    dev = torch.device("cuda:0")
    total, R, max_len = int(req[-1]), len(req) - 1, 12
    b_t, o_t = bs.to_device(bytes_, offsets, dev)
    rs_t = torch.from_numpy(req).to(dev)
    ws = bs.Workspace(bs.workspace_bytes(total, max_len, R), dev)
    perm = torch.empty(total, dtype=torch.int32, device=dev)
    tune = bs.tuning(tile, 0, bs.FLAG_SERIAL_STAGES | tflags, hbm)
    timer = bs.StageTimer(max_len)
    bs.sort_batch_staged(b_t, o_t, rs_t, req, max_len, timer, tune, ws, out=perm)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        bs.sort_batch_staged(b_t, o_t, rs_t, req, max_len, timer, tune, ws, out=perm)
    e1.record()
    torch.cuda.synchronize()
    bs.check_device_status(ws)
    print(json.dumps({"ms": e0.elapsed_time(e1) / reps, "stage_ms": timer.ms(),
                      "perm_sha": hashlib.sha256(perm.cpu().numpy().tobytes()).hexdigest()[:16]}),
          flush=True)


def cu_scaling_run(batch, args):
    """The sort with every stage in order on 8, 16, ... 256 compute units:
    one child process per count, its kernels limited by HSA_CU_MASK (CU ids
    0..n-1), the GPU counterpart of the paper's runs with 1, 2, 4, ...
    threads.  Runs before this process opens the GPU."""
    import shutil
    import subprocess
    import tempfile
    base = "/dev/shm" if os.path.isdir("/dev/shm") else None
    d = tempfile.mkdtemp(prefix="bsort_cu_", dir=base)
    try:
        np.save(os.path.join(d, "bytes.npy"), batch.bytes)
        np.save(os.path.join(d, "offsets.npy"), batch.offsets)
        np.save(os.path.join(d, "req_start.npy"), batch.req_start)
        rows = []
        for n in CU_COUNTS:
            env = dict(os.environ)
            env["HSA_CU_MASK"] = f"0:0-{n - 1}"
            cmd = [sys.executable, os.path.abspath(__file__), "--cu-child", "--cu-data", d,
                   "--tile", str(args.tile), "--hbm-tile", str(args.hbm_tile),
                   "--tune-flags", str(args.tune_flags)]
            if args.tune_cache:
                cmd += ["--tune-cache", args.tune_cache]
            res = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=300)
            print(f"cu scaling: {n} CUs, exit {res.returncode}", file=sys.stderr, flush=True)
            if res.returncode != 0:
                return {"error": f"{n} CUs: exit {res.returncode}: {res.stderr[-600:]}"}
            row = json.loads(res.stdout.strip().splitlines()[-1])
            st = row["stage_ms"]
            big = max((k for k in st if k.startswith(("lds_", "tiles_"))), key=st.get)
            row.update({"cus": n, "hsa_cu_mask": env["HSA_CU_MASK"],
                        "words_per_s": batch.total / (row["ms"] / 1e3),
                        "longest_stage": big, "longest_stage_ms": st[big]})
            rows.append(row)
        for r in rows:
            r["speedup"] = rows[0]["ms"] / r["ms"]
            r["efficiency"] = r["speedup"] * rows[0]["cus"] / r["cus"]
        return {"stages": "all in order on one stream (FLAG_SERIAL_STAGES)",
                "limit": "HSA_CU_MASK per child process", "rows": rows}
    finally:
        shutil.rmtree(d, ignore_errors=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tile", type=int, default=0, help="tile_keys (0: autotune cache or default)")
    ap.add_argument("--tune-flags", type=int, default=0,
                    help="tuning flags with --tile/--hbm-tile (16: BSORT_FLAG_LDS_TILE)")
    ap.add_argument("--hbm-tile", type=int, default=0,
                    help="hbm_tile_keys, the merge-split block width through HBM "
                         "(0: autotune cache or library default)")
    ap.add_argument("--no-plain", action="store_true", help="skip the per-bucket launch form")
    ap.add_argument("--no-probes", action="store_true", help="skip the roofline probes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the captured-graph timing")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving run")
    ap.add_argument("--no-cu-scaling", action="store_true",
                    help="skip the sort on 8, 16, ... 256 compute units (child processes)")
    ap.add_argument("--cu-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cu-data", default="", help=argparse.SUPPRESS)
    ap.add_argument("--no-layout", action="store_true",
                    help="skip the data-structure (packed keys vs text) comparison")
    ap.add_argument("--no-unbucketed", action="store_true",
                    help="skip the whole-list (unbucketed) sorts")
    ap.add_argument("--no-tokenize", action="store_true",
                    help="skip the raw-text pre-processing leg")
    ap.add_argument("--no-serial", action="store_true",
                    help="skip the per-stage timing with every stage on one stream")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the serving run (its own JSON line)")
    ap.add_argument("--serve-arrivals", type=int, default=0,
                    help="serve only the first N arrivals (0: all)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times "
                         "(reference reading for the HBM byte counters) and exit")
    ap.add_argument("--cpu-stride", type=int, default=1,
                    help="CPU baseline samples every k-th list of the batch (1: all of it, "
                         "about 10 s on 16 host threads)")
    ap.add_argument("--json-out", default="")
    ap.add_argument("--tune-cache", default="", help="autotune cache file (default: package cache)")
    ap.add_argument("--gen-workers", type=int, default=8,
                    help="input generator processes; use 1 under a profiler that opens the "
                         "GPU before main")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(lists are independent: several GPUs would shard whole lists by size)",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.cu_child:
        cu_child(args)
        return

    # inputs first (spawned worker processes, before the GPU is opened)
    t0 = time.time()
    sw = None
    if not args.no_serve or args.serve_only:
        sw = wordgen.serve(workers=args.gen_workers, count=args.serve_arrivals or None)
    if args.serve_only:
        print(json.dumps(serve_line(sw, args, time.time() - t0)), flush=True)
        return
    batch = wordgen.batch(workers=args.gen_workers)
    text = None
    if not args.no_tokenize:
        text = wordgen.raw_text(wordgen.Words(batch.bytes, batch.offsets), seed=4)
    gen_s = time.time() - t0
    # child processes first: this process must not have opened the GPU yet
    cu_scaling = None if args.no_cu_scaling else cu_scaling_run(batch, args)
    max_len = 12
    total = batch.total

    import torch
    import paper_1407_6603_amd as bs
    from paper_1407_6603_amd import autotune

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # measured ceilings (libbsort_probe.so) beside the derived ones
    peaks = None
    if not args.no_probes:
        from paper_1407_6603_amd import probe
        peaks = probe.peaks(reps=2)

    tile, hbm_tile, tflags, tuned_from = args.tile, args.hbm_tile, args.tune_flags, "flags"
    if tile == 0 and hbm_tile == 0:
        tile, hbm_tile, tflags, tuned_from = autotune.lookup(
            "batch4096", path=args.tune_cache or autotune.CACHE)

    b_t, o_t = bs.to_device(batch.bytes, batch.offsets, dev)
    rs_t = torch.from_numpy(batch.req_start).to(dev)
    perm = torch.empty(total, dtype=torch.int32, device=dev)
    tune = bs.tuning(tile, 0, tflags, hbm_tile)
    stream = torch.cuda.current_stream()
    ws = bs.Workspace(bs.workspace_bytes(total, max_len, batch.R), dev)
    struct, merge_bytes, phases_max = workload_structure(
        batch.offsets, batch.req_start, max_len, tile or 256, 2048,
        lds_fixed=bool(tflags & autotune.FLAG_LDS_TILE))

    def step(timer):
        bs.sort_batch_staged(b_t, o_t, rs_t, batch.req_start, max_len, timer, tune, ws, out=perm)

    untimed = bs.StageTimer(max_len, stream, only=())
    for _ in range(args.warmup):
        step(untimed)
    torch.cuda.synchronize()
    bs.check_device_status(ws)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    # ---- per-stage times with each stage alone on the GPU (every stage in
    # order on one stream); the timed region below runs them side by side
    serial = None
    sperm = None
    if not args.no_serial:
        stune = bs.tuning(tile, 0, bs.FLAG_SERIAL_STAGES | tflags, hbm_tile)
        sperm = torch.empty(total, dtype=torch.int32, device=dev)
        reps = min(max(args.steps, 1), 5)
        stimers = [bs.StageTimer(max_len, stream) for _ in range(reps)]
        bs.sort_batch_staged(b_t, o_t, rs_t, batch.req_start, max_len, stimers[0], stune, ws,
                             out=sperm)
        torch.cuda.synchronize()
        ev0.record(stream)
        for k in range(reps):
            bs.sort_batch_staged(b_t, o_t, rs_t, batch.req_start, max_len, stimers[k], stune, ws,
                                 out=sperm)
        ev1.record(stream)
        torch.cuda.synchronize()
        bs.check_device_status(ws)
        ssum = {}
        for t in stimers:
            for name, v in t.ms().items():
                ssum[name] = ssum.get(name, 0.0) + v
        serial = {"ms_per_step": ev0.elapsed_time(ev1) / reps, "steps": reps,
                  "stage_ms": {k: v / reps for k, v in ssum.items()}}

    # ---- per-stage times side by side: every stage's events recorded (each
    # event is a marker in its stream, so these steps run a little slower
    # than the timed region's)
    timers = [bs.StageTimer(max_len, stream) for _ in range(max(args.steps, 1))]
    torch.cuda.synchronize()
    ev0.record(stream)
    for k in range(args.steps):
        step(timers[k])
    ev1.record(stream)
    torch.cuda.synchronize()
    all_events_ms = ev0.elapsed_time(ev1) / args.steps
    stage_sum = {}
    lds_span = 0.0
    for k in range(args.steps):
        for name, v in timers[k].ms().items():
            stage_sum[name] = stage_sum.get(name, 0.0) + v
        lds_span += timers[k].span_ms(lambda n: n.startswith("lds_"))
    stage_ms = {k: v / args.steps for k, v in stage_sum.items()}
    lds_span /= args.steps
    bs.check_device_status(ws)

    # the dominant kernel is the one with the most work: the longest launch
    # with the GPU to itself (the serial leg), among stages that have work on
    # this input.  Side by side a launch's duration includes waiting for CUs
    # that other stages hold (the short tile sorts queue behind the in-LDS
    # classes), so that time alone would pick the wrong kernel.
    worked = [k for k in stage_ms if k in struct or (k == "merge_split" and merge_bytes)]
    alone = serial["stage_ms"] if serial else stage_ms
    dom = max(worked, key=lambda k: alone.get(k, 0.0))

    # ---- the dominant in-LDS stage with its merge phases skipped (tiles
    # only, every stage alone in order; its tile size as in the full sort)
    tiles_only_ms = None
    if not args.no_serial and dom in struct and dom.startswith("lds_"):
        ttune = bs.tuning(struct[dom]["tile"], 0,
                          bs.FLAG_SERIAL_STAGES | bs.FLAG_TILES_ONLY | tflags, hbm_tile)
        tperm = torch.empty(total, dtype=torch.int32, device=dev)
        reps = min(max(args.steps, 1), 5)
        ttimers = [bs.StageTimer(max_len, stream, only={dom}) for _ in range(reps + 1)]
        for t in ttimers:
            bs.sort_batch_staged(b_t, o_t, rs_t, batch.req_start, max_len, t, ttune, ws,
                                 out=tperm)
        torch.cuda.synchronize()
        bs.check_device_status(ws)
        tiles_only_ms = sum(t.ms()[dom] for t in ttimers[1:]) / reps
        del tperm

    # ---- timed region: K steps back to back on one stream, HIP events
    # around the dominant stage's launch only (read after the region)
    dtimers = [bs.StageTimer(max_len, stream, only={dom}) for _ in range(max(args.steps, 1))]
    torch.cuda.synchronize()
    ev0.record(stream)
    for k in range(args.steps):
        step(dtimers[k])
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    dom_ms = sum(t.ms()[dom] for t in dtimers[:args.steps]) / args.steps
    value = total / (ms_per_step / 1e3)
    bs.check_device_status(ws)
    got = perm.cpu().numpy()
    if serial is not None:
        serial["identical"] = bool(np.array_equal(sperm.cpu().numpy(), got))
    del sperm
    if cu_scaling is not None and "rows" in cu_scaling:
        import hashlib
        sha = hashlib.sha256(got.tobytes()).hexdigest()[:16]
        cu_scaling["identical"] = all(r["perm_sha"] == sha for r in cu_scaling["rows"])

    # ---- the same batch through a captured graph plan (one graph launch per step)
    graph = None
    if not args.no_graph:
        cap_req = int(np.diff(batch.req_start).max())
        plan = bs.Plan(total, batch.R, cap_req, max_len, tune)
        gws = bs.Workspace(plan.workspace_bytes, dev)
        gperm = torch.empty(total, dtype=torch.int32, device=dev)
        for _ in range(args.warmup):
            plan.execute(b_t, o_t, rs_t, batch.req_start, gws, out=gperm)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            plan.execute(b_t, o_t, rs_t, batch.req_start, gws, out=gperm)
        ev1.record(stream)
        torch.cuda.synchronize()
        bs.check_device_status(gws)
        g_ms = ev0.elapsed_time(ev1) / args.steps
        graph = {"value": total / (g_ms / 1e3), "unit": "words/s", "ms_per_step": g_ms,
                 "identical": bool(np.array_equal(gperm.cpu().numpy(), got))}
        plan.close()
        del gws, gperm

    # ---- the plain form: the same kernels, one launch per (list, length)
    # sub-array and per merge-split phase (plus per-list bucketize launches
    # and one host read of the sub-array sizes); 3 timed steps with events
    plain = None
    if not args.no_plain:
        ptune = bs.tuning(tile, 0, bs.FLAG_PER_BUCKET_LAUNCH | tflags, hbm_tile)
        pws = bs.Workspace(bs.workspace_bytes(total, max_len, batch.R), dev)
        pperm = torch.empty(total, dtype=torch.int32, device=dev)
        bs.sort_batch(b_t, o_t, rs_t, batch.req_start, max_len, ptune, pws, out=pperm)
        torch.cuda.synchronize()
        preps = 3
        pev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        pms = []
        for _ in range(preps):
            pev[0].record()
            bs.sort_batch(b_t, o_t, rs_t, batch.req_start, max_len, ptune, pws, out=pperm)
            pev[1].record()
            torch.cuda.synchronize()
            pms.append(pev[0].elapsed_time(pev[1]))
        bs.check_device_status(pws)
        same = bool(np.array_equal(pperm.cpu().numpy(), got))
        plain_ms = float(np.median(pms))
        plain = {"value": total / (plain_ms / 1e3), "unit": "words/s", "ms_per_step": plain_ms,
                 "steps": preps, "ms_each": pms, "identical_to_batched": same,
                 "kernels": "the batched form's: per-list bucketize with the fused pack; per "
                            "sub-array k_oets_bucket (one register tile), k_bucket_lds_one (in "
                            "LDS, or the chunks of a sub-array merged through HBM) and one "
                            "k_merge_phase_one per merge-split phase"}
        del pws, pperm

    # ---- pre-processing leg: the batch's words as one raw text (separators
    # of TEXT_SEPARATORS), tokenized back into words
    tok = None
    if text is not None:
        text_t = torch.from_numpy(text).to(dev)
        tws = bs.Workspace(device=dev)
        words_t, offsets_t, res_t = bs.tokenize(text_t, ws=tws, sync=False)
        torch.cuda.synchronize()
        reps = max(args.steps, 1)
        ev0.record(stream)
        for _ in range(reps):
            bs.tokenize(text_t, ws=tws, sync=False)
        ev1.record(stream)
        torch.cuda.synchronize()
        t_ms = ev0.elapsed_time(ev1) / reps
        nw, nl, ml, st = (int(x) for x in res_t.cpu())
        same = (st == 0 and nw == total
                and bool(np.array_equal(offsets_t[:nw + 1].cpu().numpy(), batch.offsets))
                and bool(np.array_equal(words_t[:nl].cpu().numpy(), batch.bytes)))
        # algorithmic HBM bytes: the text read once, the letters and the
        # int64 offsets written once
        tb = len(text) + nl + 8 * (nw + 1)
        parts = [measured_traffic(k) for k in ("k_tok_count", "k_tok_scan", "k_tok_write")]
        tok_traffic = None if None in parts else sum(parts)
        gbs = tb / (t_ms / 1e3) / 1e9
        tok = {"text_bytes": len(text), "words": nw, "letters": nl, "max_len": ml,
               "ms": t_ms, "words_per_s": nw / (t_ms / 1e3), "text_gb_per_s": len(text) / t_ms / 1e6,
               "identical_to_batch_words": same,
               "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                            "frac": gbs / PEAK_HBM_GBS, "bytes_algorithmic": tb,
                            "traffic": tok_traffic,
                            "kernels": "k_tok_count, k_tok_scan, k_tok_write"}}
        del text_t, tws, words_t, offsets_t, res_t

    # ---- data-structure ablation (Section III, Tables 2 and 3): the medium
    # list, each sub-array sorted whole by one workgroup, with the words as
    # packed keys or read from the text through the offsets; the library's
    # tiled path on the same list beside them
    layout = None
    if not args.no_layout:
        w2 = wordgen.single(2)
        ml2 = wordgen.SINGLE[2].lmax
        lb_t, lo_t = bs.to_device(w2.bytes, w2.offsets, dev)
        lws = bs.Workspace(device=dev)
        counts_t, starts_t, order_t = bs.bucketize(lb_t, lo_t, ml2, ws=lws)
        lperm = torch.empty(w2.n, dtype=torch.int32, device=dev)
        res = {}
        ref = None
        for name, fn in (("packed", lambda: bs.oets_buckets(lb_t, lo_t, counts_t, starts_t,
                                                             order_t, ml2, bs.LAYOUT_PACKED,
                                                             out=lperm, check=False)),
                         ("text", lambda: bs.oets_buckets(lb_t, lo_t, counts_t, starts_t,
                                                           order_t, ml2, bs.LAYOUT_TEXT,
                                                           out=lperm, check=False)),
                         ("library_path", lambda: bs.sort_buckets(lb_t, lo_t, counts_t,
                                                                   starts_t, order_t, ml2,
                                                                   tune, lws, out=lperm))):
            fn()
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(3):
                fn()
            ev1.record(stream)
            torch.cuda.synchronize()
            l_ms = ev0.elapsed_time(ev1) / 3
            got2 = lperm.cpu().numpy()
            ref = got2 if ref is None else ref
            res[name] = {"ms": l_ms, "words_per_s": w2.n / (l_ms / 1e3),
                         "identical": bool(np.array_equal(got2, ref))}
        bs.check_device_status(lws)
        layout = {"workload": f"medium list: {w2.n} words, lengths 1-{ml2}", "sorts": res,
                  "text_over_packed": res["text"]["ms"] / res["packed"]["ms"],
                  "packed_over_library_path": res["packed"]["ms"] / res["library_path"]["ms"]}
        del lb_t, lo_t, lws, counts_t, starts_t, order_t, lperm

    # ---- unbucketed ablation (Table 1 rows 2-3): every list sorted whole by
    # fixed-width keys (alphabetic; length only; length then bytes), the same
    # OETS and merge-split, no sub-arrays
    unb = None
    if not args.no_unbucketed:
        lens = np.diff(batch.offsets)
        lid = np.repeat(np.arange(batch.R), np.diff(batch.req_start))
        n_r = np.diff(batch.req_start).astype(np.float64)
        cnt = np.bincount(lid * (max_len + 1) + lens, minlength=batch.R * (max_len + 1))
        cmp_bucketed = float((cnt * (cnt - 1) / 2).sum())
        cmp_whole = float((n_r * (n_r - 1) / 2).sum())
        uws = bs.Workspace(device=dev)
        legs = {}
        for name, mode, width in (("alphabetic", bs.KEY_BYTES, max_len),
                                  ("length", bs.KEY_LENGTH, 1),
                                  ("length_then_bytes", bs.KEY_LENGTH_BYTES, max_len + 1)):
            kb, ko = bs.fixed_width(b_t, o_t, width, mode)
            uperm = torch.empty(total, dtype=torch.int32, device=dev)
            bs.sort_batch(kb, ko, rs_t, batch.req_start, width, tune, uws, out=uperm)
            torch.cuda.synchronize()
            reps = 3
            ev0.record(stream)
            for _ in range(reps):
                bs.sort_batch(kb, ko, rs_t, batch.req_start, width, tune, uws, out=uperm)
            ev1.record(stream)
            torch.cuda.synchronize()
            bs.check_device_status(uws)
            u_ms = ev0.elapsed_time(ev1) / reps
            up = uperm.cpu().numpy()
            if mode == bs.KEY_LENGTH_BYTES:
                ok = bool(np.array_equal(up, got))
            else:                                  # library routines on 16 sampled lists
                ok = True
                for r in range(0, batch.R, batch.R // 16):
                    a, e = int(batch.req_start[r]), int(batch.req_start[r + 1])
                    if mode == bs.KEY_LENGTH:
                        ex = np.argsort(lens[a:e], kind="stable")
                    else:
                        wl = [batch.bytes[batch.offsets[i]:batch.offsets[i + 1]].tobytes()
                              for i in range(a, e)]
                        ex = np.array(sorted(range(e - a), key=lambda i: wl[i]))
                    ok = ok and bool(np.array_equal(up[a:e], ex))
            legs[name] = {"ms": u_ms, "words_per_s": total / (u_ms / 1e3), "key_bytes": width,
                          "vs_bucketed": u_ms / ms_per_step, "checked": ok}
            del kb, ko, uperm
        unb = {"bucketed_ms": ms_per_step, "sorts": legs,
               "bubble_comparisons": {"bucketed": cmp_bucketed, "whole_list": cmp_whole,
                                      "ratio": cmp_whole / cmp_bucketed},
               "check": "length_then_bytes against the bucketed result (all lists); the "
                        "others against a stable library sort on 16 sampled lists"}
        del uws

    # ---- roofline of the dominant kernel (chosen above; every tile and in-LDS
    # stage is exactly one kernel launch), at its launch time in the timed region
    roof = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": None, "traffic": None}
    if dom in struct:
        w = struct[dom]
        D, ce, sec = w["D"], w["ce"], dom_ms / 1e3
        # the tile sorts' compare-exchanges at their VALU cost (ce_cost), over
        # the whole launch (tile sorts and merge phases)
        achieved = w["slots"] / sec / 1e12
        roof = {"bound": "alu", "kernel": kernel_name(dom), "achieved": achieved,
                "peak": VALU_TIPS, "unit": "T lane-instructions/s",
                "frac": achieved / VALU_TIPS,
                "work": "tile compare-exchanges x VALU instructions each (min + max: 2)",
                "traffic": measured_traffic(kernel_name(dom)),
                # key lanes (8 B each) read, perm read and written (4 + 4 B) per word
                "hbm_bytes_algorithmic": (8 * (D // 2) + 8) * w["words"],
                "launch_ms": dom_ms, "launch_ms_alone": alone.get(dom),
                "ce_per_launch": ce, "ce_per_s": ce / sec,
                "valu_lane_instructions_per_launch": w["slots"], "words_per_launch": w["words"]}
        if peaks:
            m = peaks["f64_minmax"]["rate"] / 1e12
            roof["peak_measured"] = m
            roof["peak_measured_probe"] = "f64_minmax"
            roof["frac_measured"] = achieved / m
        if tiles_only_ms:
            # the same launch with the merge phases skipped: the tile sorts'
            # own rate, and the share of the launch the merge phases take
            roof["tiles_only_ms"] = tiles_only_ms
            roof["tiles_only_frac"] = w["slots"] / (tiles_only_ms / 1e3) / 1e12 / VALU_TIPS
            if alone.get(dom):
                roof["merge_share_alone"] = 1.0 - tiles_only_ms / alone[dom]
        if "lds_bytes" in w:
            # the tile step at its issue floor plus the merge phases' LDS bytes
            # (half read, half written) at the LDS peaks
            roof["merge_lds_bytes"] = w["lds_bytes"]
            roof["floor_ms"] = (w["slots"] / (VALU_TIPS * 1e12)
                                + w["lds_bytes"] / 2 / (PEAK_LDS_READ_TBS * 1e12)
                                + w["lds_bytes"] / 2 / (PEAK_LDS_WRITE_TBS * 1e12)) * 1e3
            roof["frac_of_floor"] = roof["floor_ms"] / dom_ms
            # the roofline the paper's compare-exchange count suggests if every
            # compare-exchange read and wrote its records in LDS: 2 reads and 2
            # writes of (8W + 4) bytes (W = 1 key lane here).  The tiles keep
            # records in registers, so it does not bind: frac > 1
            ce_rd = ce * 2 * 12
            lds_ce_ms = (ce_rd / (PEAK_LDS_READ_TBS * 1e12)
                         + ce_rd / (PEAK_LDS_WRITE_TBS * 1e12)) * 1e3
            roof["lds_compare_exchange"] = {
                "bytes": 2 * ce_rd, "floor_ms": lds_ce_ms, "frac": lds_ce_ms / dom_ms,
                "peaks_tb_s": {"read": PEAK_LDS_READ_TBS, "write": PEAK_LDS_WRITE_TBS}}
        # all in-LDS classes together, over the span from the first class's
        # start to the last one's end (they run concurrently)
        lds_slots = sum(w["slots"] for k, w in struct.items() if k.startswith("lds_"))
        roof["lds_all_classes"] = {
            "span_ms": lds_span, "valu_lane_instructions": lds_slots,
            "achieved": lds_slots / (lds_span / 1e3) / 1e12, "peak": VALU_TIPS,
            "unit": "T lane-instructions/s",
            "frac": lds_slots / (lds_span / 1e3) / 1e12 / VALU_TIPS}
    elif dom == "merge_split" and merge_bytes:
        achieved = merge_bytes / (dom_ms / 1e3) / 1e9
        roof = {"bound": "hbm", "kernel": "k_merge_sched", "achieved": achieved,
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                "traffic": None, "bytes_per_step": merge_bytes}

    # ---- CPU baseline: the oracle (paper's procedure) on the batch (or every k-th list)
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        ncores, model = cpu_info()
        idx = list(range(0, batch.R, args.cpu_stride))
        sub = wordgen.Batch.concat([batch.request(r) for r in idx])
        t2 = time.perf_counter()
        operm, ncmp = oracle.bubble_sort_batch(sub.bytes, sub.offsets, sub.req_start, max_len,
                                               threads=ncores)
        cpu_s = time.perf_counter() - t2
        cpu = {"value": sub.total / cpu_s, "unit": "words/s", "cores": ncores, "kind": "oracle",
               "cpu_model": model, "seconds": cpu_s, "comparisons": ncmp,
               "sample": (f"every {args.cpu_stride}th list of the 4,096" if args.cpu_stride > 1
                          else "the whole batch") +
                         f" ({len(idx)} lists, {sub.total} words); bucket-then-bubble "
                         f"procedure, one list per thread, {ncores} threads"}
        gsub = np.concatenate([got[batch.req_start[r]:batch.req_start[r + 1]] for r in idx])
        parity = {"lists_checked": len(idx), "words_checked": sub.total,
                  "bit_exact": bool(np.array_equal(gsub, operm))}

    serving = serve_run(sw, args) if sw is not None else None

    line = {
        "metric": METRIC,
        "value": value, "unit": "words/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "batch-4096: 4,096 lists, sizes log-uniform in [16, 65536], "
                               f"{total} words, lengths 1-12, Zipf 1.1 over an 800-word "
                               "vocabulary per list, 5% capitalised",
                   "global_batch": batch.R, "words": total, "max_len": max_len,
                   "tile_keys": tile or 256, "hbm_tile_keys": hbm_tile or "default",
                   "lds_tile": "tuned" if tflags & autotune.FLAG_LDS_TILE else "library",
                   "tuning_source": tuned_from, "parallelism": "single GPU"},
        "graph_plan": graph,
        "measured_peaks": peaks,
        "derived_peaks": {"valu_t_lane_instr_per_s": VALU_TIPS,
                          "lds_read_tb_s": PEAK_LDS_READ_TBS,
                          "lds_write_tb_s": PEAK_LDS_WRITE_TBS, "hbm_gb_s": PEAK_HBM_GBS},
        "per_bucket_launch": plain,
        "batched_over_per_bucket": (value / plain["value"]) if plain else None,
        "stage_ms": stage_ms,
        "all_stage_events_ms_per_step": all_events_ms,
        "serial_stages": serial,
        "tokenize": tok,
        "unbucketed": unb,
        "data_structure": layout,
        "cu_scaling": cu_scaling,
        "merge_phases_max": phases_max,
        "work": struct,
        "roofline": roof,
        "cpu_baseline": cpu,
        "parity": parity,
        "serving": serving,
        "gpu": torch.cuda.get_device_name(0),
        "gen_seconds": gen_s,
    }
    s = json.dumps(line)
    print(s, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(s + "\n")


if __name__ == "__main__":
    main()
