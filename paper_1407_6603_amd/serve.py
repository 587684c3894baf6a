"""Continuous-batching sort service.

Requests (word lists) arrive over time.  The server admits them in arrival
order while their device footprint fits a memory pool, keeps admitted
requests resident, and as soon as a launch slot (a stream) is free sends every
admitted-but-unlaunched request to the device as one batch.  Batches on
different streams run concurrently, so a request that arrives while another
batch is sorting starts on the device without waiting for it.  Completed
requests free their pool bytes.  Latency is completion time minus arrival
time.

The scheduler is independent of the device: ``GpuExecutor`` runs batches
through libbsort on HIP streams; tests drive the same ``Server`` with a
virtual clock and a host executor.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds on the server clock
    first_word: int           # global word range [first_word, last_word) in the staging arrays
    last_word: int
    n_bytes: int

    @property
    def n(self) -> int:
        return self.last_word - self.first_word


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: Optional[float] = None
    launched: Optional[float] = None
    done: Optional[float] = None
    refused: bool = False
    batch: int = -1
    perm: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class WallClock:
    def __init__(self):
        self.t0 = time.monotonic()

    def now(self) -> float:
        return time.monotonic() - self.t0

    def wait_until(self, t: float):
        d = t - self.now()
        if d > 0:
            time.sleep(min(d, 0.0005))

    def idle(self):
        time.sleep(0.00005)


class VirtualClock:
    """Time advances only when the server has nothing to do."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def wait_until(self, t: float):
        self.t = max(self.t, t)

    def idle(self):
        pass


@dataclasses.dataclass
class Staging:
    """All request data as received, in host memory: concatenated bytes and
    int64 offsets into them (word i of the stream is
    bytes[offsets[i]:offsets[i+1]])."""
    bytes: np.ndarray
    offsets: np.ndarray
    max_len: int


class Server:
    def __init__(self, executor, pool_bytes: int = 16 << 30, max_batch_words: int = 1 << 26,
                 clock=None):
        self.ex = executor
        self.pool = int(pool_bytes)
        self.max_batch_words = int(max_batch_words)
        self.clock = clock if clock is not None else WallClock()
        self.pool_used = 0
        self.pool_high = 0
        self.batches = 0

    def run(self, requests: Sequence[Request], keep_perms: bool = True) -> List[Result]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        results: Dict[int, Result] = {r.rid: Result(r.rid, r.n, r.arrival) for r in reqs}
        fp = {r.rid: self.ex.footprint(r) for r in reqs}
        nxt = 0
        queue: List[Request] = []          # arrived, not admitted
        ready: List[Request] = []          # admitted, not launched
        inflight = []                      # (handle, [Request])
        clock = self.clock
        while nxt < len(reqs) or queue or ready or inflight:
            now = clock.now()
            progressed = False
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
                progressed = True
            # admission, in arrival order, by pool bytes
            while queue:
                r = queue[0]
                if fp[r.rid] > self.pool:
                    results[r.rid].refused = True
                    results[r.rid].done = now
                    queue.pop(0)
                    progressed = True
                    continue
                if self.pool_used + fp[r.rid] > self.pool:
                    break
                self.pool_used += fp[r.rid]
                self.pool_high = max(self.pool_high, self.pool_used)
                results[r.rid].admitted = now
                ready.append(queue.pop(0))
                progressed = True
            # completions
            still = []
            for h, members in inflight:
                if self.ex.poll(h):
                    perms = self.ex.collect(h)
                    t = clock.now()
                    for r, p in zip(members, perms):
                        res = results[r.rid]
                        res.done = t
                        if keep_perms:
                            res.perm = p
                        self.pool_used -= fp[r.rid]
                    progressed = True
                else:
                    still.append((h, members))
            inflight = still
            # launch every admitted request as one batch when a slot is free
            if ready and len(inflight) < self.ex.slots:
                batch, words = [], 0
                while ready and (not batch or words + ready[0].n <= self.max_batch_words):
                    words += ready[0].n
                    batch.append(ready.pop(0))
                h = self.ex.launch(batch)
                t = clock.now()
                for r in batch:
                    results[r.rid].launched = t
                    results[r.rid].batch = self.batches
                self.batches += 1
                inflight.append((h, batch))
                progressed = True
            if not progressed:
                wake = [reqs[nxt].arrival] if nxt < len(reqs) else []
                wake += [self.ex.finish_time(h) for h, _ in inflight
                         if self.ex.finish_time(h) is not None]
                if wake:
                    clock.wait_until(min(wake))
                else:
                    clock.idle()
        return [results[r.rid] for r in requests]


def latency_stats(results: Iterable[Result]) -> Dict[str, float]:
    done = [r for r in results if not r.refused]
    lat = np.array([r.latency for r in done], dtype=np.float64)
    words = sum(r.n for r in done)
    t0 = min(r.arrival for r in done)
    t1 = max(r.done for r in done)
    waits = np.array([r.launched - r.arrival for r in done], dtype=np.float64)
    return {
        "requests": len(done),
        "refused": sum(1 for r in results if r.refused),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "mean_queue_ms": float(waits.mean() * 1e3),
        "words": int(words),
        "span_s": float(t1 - t0),
        "words_per_s": float(words / (t1 - t0)) if t1 > t0 else float("nan"),
    }


class GpuExecutor:
    """Runs batches through libbsort.  Each batch: host-to-device copies of its
    byte and offset ranges, bsort_sort_batch, device-to-host copy of perm, all
    on one of ``streams`` HIP streams (default priority), ordered by an event.
    Host staging arrays are pinned once up front."""

    def __init__(self, staging: Staging, streams: int = 3, tune=None, device="cuda"):
        import torch
        from . import api
        self.torch, self.api = torch, api
        self.dev = torch.device(device)
        self.st = staging
        self.tune = tune
        self.bytes_h = torch.from_numpy(staging.bytes).pin_memory()
        self.offs_h = torch.from_numpy(staging.offsets).pin_memory()
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        self.ws = [api.Workspace(device=self.dev) for _ in range(streams)]
        self.busy = [False] * streams
        self.slots = streams
        self.max_len = staging.max_len
        self._ws_fixed = api.workspace_bytes(0, self.max_len, 1)

    def footprint(self, r: Request) -> int:
        ws = self.api.workspace_bytes(r.n, self.max_len, 1) - self._ws_fixed
        return int(r.n_bytes + 8 * (r.n + 1) + 4 * r.n + ws)

    def launch(self, batch: List[Request]):
        torch, api = self.torch, self.api
        k = self.busy.index(False)
        self.busy[k] = True
        s = self.streams[k]
        w0, w1 = batch[0].first_word, batch[-1].last_word
        b0, b1 = int(self.st.offsets[w0]), int(self.st.offsets[w1])
        rs = np.zeros(len(batch) + 1, dtype=np.int64)
        np.cumsum([r.n for r in batch], out=rs[1:])
        with torch.cuda.stream(s):
            nb = max(b1 - b0, 1)
            bytes_d = torch.empty(nb, dtype=torch.uint8, device=self.dev)
            bytes_d[:b1 - b0].copy_(self.bytes_h[b0:b1], non_blocking=True)
            offs_d = torch.empty(w1 - w0 + 1, dtype=torch.int64, device=self.dev)
            offs_d.copy_(self.offs_h[w0:w1 + 1], non_blocking=True)
            rs_d = torch.from_numpy(rs).to(self.dev, non_blocking=False)
            perm_d = torch.empty(w1 - w0, dtype=torch.int32, device=self.dev)
            # offsets index the staging byte stream; the device copy holds its
            # bytes [b0, b1), so it is passed with origin b0
            api.sort_batch(bytes_d, offs_d, rs_d, rs, self.max_len, self.tune, self.ws[k], s,
                           perm_d, byte_origin=b0)
            perm_h = torch.empty(w1 - w0, dtype=torch.int32, pin_memory=True)
            perm_h.copy_(perm_d, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"k": k, "ev": ev, "perm_h": perm_h, "rs": rs,
                "keep": (bytes_d, offs_d, rs_d, perm_d)}

    def poll(self, h) -> bool:
        return h["ev"].query()

    def finish_time(self, h):
        return None

    def collect(self, h):
        api = self.api
        api.check_device_status(self.ws[h["k"]], self.streams[h["k"]])
        self.busy[h["k"]] = False
        p = h["perm_h"].numpy()
        rs = h["rs"]
        return [p[rs[i]:rs[i + 1]].copy() for i in range(len(rs) - 1)]


class HostExecutor:
    """Executes batches with a host sort function on a virtual timeline:
    a batch occupies one of ``slots`` lanes for ``cost(words)`` seconds.  For
    testing the scheduler without a device."""

    def __init__(self, staging: Staging, sort_fn: Callable, clock: VirtualClock,
                 slots: int = 2, cost=lambda words: 1e-3 + 1e-8 * words,
                 footprint=lambda r: 64 * r.n + r.n_bytes):
        self.st = staging
        self.sort_fn = sort_fn
        self.clock = clock
        self.slots = slots
        self.cost = cost
        self._fp = footprint
        self.lane_free = [0.0] * slots
        self.busy = [False] * slots
        self.log = []

    def footprint(self, r: Request) -> int:
        return int(self._fp(r))

    def launch(self, batch: List[Request]):
        k = self.busy.index(False)
        self.busy[k] = True
        start = max(self.clock.now(), self.lane_free[k])
        words = sum(r.n for r in batch)
        end = start + self.cost(words)
        self.lane_free[k] = end
        perms = []
        for r in batch:
            o = self.st.offsets[r.first_word:r.last_word + 1]
            perms.append(self.sort_fn(self.st.bytes, o))
        h = {"k": k, "start": start, "end": end, "perms": perms, "rids": [r.rid for r in batch]}
        self.log.append(h)
        return h

    def poll(self, h) -> bool:
        return self.clock.now() >= h["end"]

    def finish_time(self, h):
        return h["end"]

    def collect(self, h):
        self.busy[h["k"]] = False
        return h["perms"]


def build_staging(word_lists, max_len: int):
    """Concatenate word lists (objects with .bytes and request-local .offsets)
    into one staging stream; returns (staging, [(first_word, last_word,
    n_bytes)])."""
    total_words = sum(w.n for w in word_lists)
    total_bytes = sum(int(w.offsets[-1]) for w in word_lists)
    b = np.empty(max(total_bytes, 1), dtype=np.uint8)
    o = np.zeros(total_words + 1, dtype=np.int64)
    spans = []
    wpos = bpos = 0
    for w in word_lists:
        nbw = int(w.offsets[-1])
        b[bpos:bpos + nbw] = w.bytes[:nbw]
        o[wpos:wpos + w.n + 1] = w.offsets + bpos
        spans.append((wpos, wpos + w.n, nbw))
        wpos += w.n
        bpos += nbw
    return Staging(b, o, max_len), spans
