"""Continuous-batching sort service.

Requests (word lists) arrive over time.  The server admits them in arrival
order while their device footprint fits a memory pool, keeps admitted
requests resident, and as soon as a launch slot (a stream) is free sends the
admitted-but-unlaunched requests to the device as one batch.  Batches on
different streams run concurrently, so a request that arrives while another
batch is sorting starts on the device without waiting for it.  Completed
requests free their pool bytes.  Latency is completion time minus arrival
time.  Queued requests (arrived, or admitted but not yet launched) can be
cancelled.

The pool is a ring over one device arena (``RingArena``): admission carves a
request's footprint from it, in admission order, and a batch's buffers
(bytes, offsets, perm, request bounds, workspace) are laid out inside the
span its members hold.  A batch is therefore a run of requests that are
consecutive in the arena and in the staging arrays (a refusal, a
cancellation or out-of-order arrival ends a batch there).

The scheduler is independent of the device: ``GpuExecutor`` runs batches
through libbsort on HIP streams; tests drive the same ``Server`` with a
virtual clock and a host executor.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

ALIGN = 256


def _up(x: int, a: int = ALIGN) -> int:
    return (int(x) + a - 1) // a * a


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
    cancelled: bool = False
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


class RingArena:
    """First-in-first-out allocator over [0, capacity) bytes.

    Blocks are carved at the head in allocation order and may be freed in
    any order; the tail advances over freed blocks at the front.  A block
    that does not fit before the end of the arena starts at 0 (the skipped
    end is held by a padding block freed with it).  With every block freed
    the ring starts over at 0, so a block of at most ``capacity`` bytes
    always fits eventually."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity) // ALIGN * ALIGN
        self.blocks = collections.deque()     # [offset, size, freed] in allocation order
        self.head = 0
        self.live = {}                        # offset -> block
        self.used = 0

    def _tail(self) -> int:
        return self.blocks[0][0] if self.blocks else self.head

    def alloc(self, size: int) -> Optional[int]:
        size = _up(max(size, 1))
        if size > self.capacity:
            return None
        if not self.blocks:
            self.head = 0
        tail = self._tail()
        if self.blocks and self.head <= tail:           # free space is [head, tail)
            if self.head + size > tail:
                return None
            off = self.head
        elif self.head + size <= self.capacity:          # free space is [head, cap) + [0, tail)
            off = self.head
        elif size <= tail:                               # wrap: pad out the end
            pad = [self.head, self.capacity - self.head, True]
            if pad[1] > 0:
                self.blocks.append(pad)
            off = 0
        else:
            return None
        blk = [off, size, False]
        self.blocks.append(blk)
        self.live[off] = blk
        self.head = off + size
        self.used += size
        return off

    def free(self, off: int):
        blk = self.live.pop(off)
        blk[2] = True
        self.used -= blk[1]
        while self.blocks and self.blocks[0][2]:
            self.blocks.popleft()
        if not self.blocks:
            self.head = 0


@dataclasses.dataclass
class Staging:
    """All request data as received, in host memory: concatenated bytes and
    int64 offsets into them (word i of the stream is
    bytes[offsets[i]:offsets[i+1]])."""
    bytes: np.ndarray
    offsets: np.ndarray
    max_len: int


def batch_layout(n_bytes: int, n_words: int, n_requests: int, ws_bytes: int) -> Dict[str, int]:
    """Byte offsets of a batch's buffers inside its arena span (256-aligned
    sections: bytes, offsets, perm, request bounds, workspace) and the span
    size they need."""
    lay = {"bytes": 0}
    lay["offsets"] = _up(n_bytes)
    lay["perm"] = lay["offsets"] + _up(8 * (n_words + 1))
    lay["req_start"] = lay["perm"] + _up(4 * n_words)
    lay["ws"] = lay["req_start"] + _up(8 * (n_requests + 1))
    lay["size"] = lay["ws"] + _up(ws_bytes)
    return lay


def request_footprint(n_words: int, n_bytes: int, max_len: int, workspace_bytes) -> int:
    """Arena bytes a request holds: its share of every batch section.  A
    batch's workspace never exceeds the sum of its members' one-list
    workspaces, so the members' footprints cover the batch layout."""
    return batch_layout(n_bytes, n_words, 1, workspace_bytes(n_words, max_len, 1))["size"]


class Server:
    def __init__(self, executor, pool_bytes: Optional[int] = None, max_batch_words: int = 1 << 26,
                 clock=None):
        self.ex = executor
        if pool_bytes is None:
            pool_bytes = getattr(executor, "arena_bytes")
        self.pool = int(pool_bytes)
        arena = getattr(executor, "arena_bytes", None)
        if arena is not None and self.pool > arena:
            raise ValueError(f"pool of {self.pool} bytes exceeds the executor's arena ({arena})")
        self.max_batch_words = int(max_batch_words)
        self.clock = clock if clock is not None else WallClock()
        self.pool_used = 0
        self.pool_high = 0
        self.batches = 0

    def _take_batch(self, ready: List[Request], where: Dict[int, Tuple[int, int]]):
        """The longest prefix of ready that is one run in the arena and in
        the staging arrays, within max_batch_words."""
        batch = [ready[0]]
        words = ready[0].n
        for r in ready[1:]:
            prev = batch[-1]
            po, ps = where[prev.rid]
            if (r.first_word != prev.last_word or where[r.rid][0] != po + ps
                    or words + r.n > self.max_batch_words):
                break
            batch.append(r)
            words += r.n
        del ready[:len(batch)]
        return batch

    def run(self, requests: Sequence[Request], keep_perms: bool = True,
            cancels: Sequence[Tuple[float, int]] = ()) -> List[Result]:
        """Serve requests; cancels: (time, rid) pairs.  A cancel takes effect
        if the request has not been launched by then (it is dropped, and its
        pool bytes freed); later it does nothing."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        results: Dict[int, Result] = {r.rid: Result(r.rid, r.n, r.arrival) for r in reqs}
        fp = {r.rid: self.ex.footprint(r) for r in reqs}
        arena = RingArena(self.pool)
        where: Dict[int, Tuple[int, int]] = {}         # rid -> (arena offset, size)
        cq = sorted(cancels)
        ci = 0
        cancelled = set()
        nxt = 0
        queue: List[Request] = []          # arrived, not admitted
        ready: List[Request] = []          # admitted, not launched
        inflight = []                      # (handle, [Request])
        clock = self.clock
        while nxt < len(reqs) or queue or ready or inflight:
            now = clock.now()
            progressed = False
            while ci < len(cq) and cq[ci][0] <= now:
                rid = cq[ci][1]
                ci += 1
                res = results.get(rid)
                if res is None or res.launched is not None or res.refused or res.cancelled:
                    continue
                res.cancelled = True
                res.done = now
                cancelled.add(rid)
                for lst in (queue, ready):
                    for i, r in enumerate(lst):
                        if r.rid == rid:
                            del lst[i]
                            break
                if rid in where:
                    off, size = where.pop(rid)
                    arena.free(off)
                    self.pool_used -= size
                progressed = True
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                if reqs[nxt].rid not in cancelled:
                    queue.append(reqs[nxt])
                nxt += 1
                progressed = True
            # admission, in arrival order, by pool bytes
            while queue:
                r = queue[0]
                if _up(fp[r.rid]) > arena.capacity:
                    results[r.rid].refused = True
                    results[r.rid].done = now
                    queue.pop(0)
                    progressed = True
                    continue
                off = arena.alloc(fp[r.rid])
                if off is None:
                    break
                where[r.rid] = (off, _up(fp[r.rid]))
                self.pool_used += _up(fp[r.rid])
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
                        off, size = where.pop(r.rid)
                        arena.free(off)
                        self.pool_used -= size
                    progressed = True
                else:
                    still.append((h, members))
            inflight = still
            # launch the admitted requests that form one run as a batch when a slot is free
            if ready and len(inflight) < self.ex.slots:
                batch = self._take_batch(ready, where)
                span = (where[batch[0].rid][0],
                        sum(where[r.rid][1] for r in batch))
                h = self.ex.launch(batch, span)
                t = clock.now()
                for r in batch:
                    results[r.rid].launched = t
                    results[r.rid].batch = self.batches
                self.batches += 1
                inflight.append((h, batch))
                progressed = True
            if not progressed:
                wake = [reqs[nxt].arrival] if nxt < len(reqs) else []
                if ci < len(cq):
                    wake.append(cq[ci][0])
                wake += [self.ex.finish_time(h) for h, _ in inflight
                         if self.ex.finish_time(h) is not None]
                if wake:
                    clock.wait_until(min(wake))
                else:
                    clock.idle()
        return [results[r.rid] for r in requests]


def latency_stats(results: Iterable[Result]) -> Dict[str, float]:
    results = list(results)
    done = [r for r in results if not r.refused and not r.cancelled]
    lat = np.array([r.latency for r in done], dtype=np.float64)
    words = sum(r.n for r in done)
    t0 = min(r.arrival for r in done)
    t1 = max(r.done for r in done)
    waits = np.array([r.launched - r.arrival for r in done], dtype=np.float64)
    return {
        "requests": len(done),
        "refused": sum(1 for r in results if r.refused),
        "cancelled": sum(1 for r in results if r.cancelled),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "mean_queue_ms": float(waits.mean() * 1e3),
        "words": int(words),
        "span_s": float(t1 - t0),
        "words_per_s": float(words / (t1 - t0)) if t1 > t0 else float("nan"),
    }


class GpuExecutor:
    """Runs batches through libbsort inside one device arena.

    The arena (``arena_bytes``, allocated once) is the server's admission
    pool: a batch's bytes, offsets, perm, request bounds and workspace are
    views into the span its members hold, so no device memory is allocated
    per batch.  Each batch: host-to-device copies of its byte and offset
    ranges and its request bounds (from pinned memory), bsort_sort_batch, and
    a device-to-host copy of perm into one pinned result array, all on one of
    ``streams`` HIP streams (default priority), ordered by an event."""

    def __init__(self, staging: Staging, arena_bytes: int = 16 << 30, streams: int = 3,
                 tune=None, device="cuda"):
        import torch
        from . import api
        self.torch, self.api = torch, api
        self.dev = torch.device(device)
        self.st = staging
        self.tune = tune
        self.bytes_h = torch.from_numpy(staging.bytes).pin_memory()
        self.offs_h = torch.from_numpy(staging.offsets).pin_memory()
        n_all = len(staging.offsets) - 1
        self.perm_h = torch.empty(max(n_all, 1), dtype=torch.int32, pin_memory=True)
        self.arena_bytes = int(arena_bytes) // ALIGN * ALIGN
        self.arena = torch.empty(self.arena_bytes + ALIGN, dtype=torch.uint8, device=self.dev)
        self.base = (self.arena.data_ptr() + ALIGN - 1) // ALIGN * ALIGN - self.arena.data_ptr()
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(streams)]
        # request bounds per stream, pinned; reused once the stream's batch is collected
        self.rs_cap = 1 << 12
        self.rs_h = [torch.empty(self.rs_cap + 1, dtype=torch.int64, pin_memory=True)
                     for _ in range(streams)]
        self.busy = [False] * streams
        self.slots = streams
        self.max_len = staging.max_len
        self._ws_fixed = api.workspace_bytes(0, self.max_len, 1)

    def footprint(self, r: Request) -> int:
        return request_footprint(r.n, r.n_bytes, self.max_len, self.api.workspace_bytes)

    def _view(self, off: int, nbytes: int, dtype):
        torch = self.torch
        a = self.base + off
        t = self.arena[a:a + nbytes]
        return t.view(dtype) if dtype is not torch.uint8 else t

    def launch(self, batch: List[Request], span: Tuple[int, int]):
        torch, api = self.torch, self.api
        k = self.busy.index(False)
        self.busy[k] = True
        s = self.streams[k]
        R = len(batch)
        if R > self.rs_cap:
            raise ValueError(f"batch of {R} requests exceeds {self.rs_cap}")
        w0, w1 = batch[0].first_word, batch[-1].last_word
        b0, b1 = int(self.st.offsets[w0]), int(self.st.offsets[w1])
        n = w1 - w0
        rs = self.rs_h[k][:R + 1]
        rs[0] = 0
        rs[1:] = torch.from_numpy(np.cumsum([r.n for r in batch], dtype=np.int64))
        ws_bytes = api.workspace_bytes(n, self.max_len, R)
        lay = batch_layout(b1 - b0, n, R, ws_bytes)
        off, size = span
        if lay["size"] > size:
            raise RuntimeError(f"batch needs {lay['size']} arena bytes, its span holds {size}")
        bytes_d = self._view(off + lay["bytes"], max(b1 - b0, 1), torch.uint8)
        offs_d = self._view(off + lay["offsets"], 8 * (n + 1), torch.int64)
        perm_d = self._view(off + lay["perm"], 4 * n, torch.int32)
        rs_d = self._view(off + lay["req_start"], 8 * (R + 1), torch.int64)
        ws = api.Workspace.wrap(self._view(off + lay["ws"], ws_bytes, torch.uint8))
        with torch.cuda.stream(s):
            if b1 > b0:
                bytes_d[:b1 - b0].copy_(self.bytes_h[b0:b1], non_blocking=True)
            offs_d.copy_(self.offs_h[w0:w1 + 1], non_blocking=True)
            rs_d.copy_(rs, non_blocking=True)
            # offsets index the staging byte stream; the device copy holds its
            # bytes [b0, b1), so it is passed with origin b0
            api.sort_batch(bytes_d, offs_d, rs_d, rs.numpy(), self.max_len, self.tune, ws, s,
                           perm_d, byte_origin=b0)
            self.perm_h[w0:w1].copy_(perm_d, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"k": k, "ev": ev, "w0": w0, "w1": w1, "rs": rs.numpy().copy(), "ws": ws}

    def poll(self, h) -> bool:
        return h["ev"].query()

    def finish_time(self, h):
        return None

    def collect(self, h):
        api = self.api
        api.check_device_status(h["ws"], self.streams[h["k"]])
        self.busy[h["k"]] = False
        p = self.perm_h[h["w0"]:h["w1"]].numpy()
        rs = h["rs"]
        return [p[rs[i]:rs[i + 1]] for i in range(len(rs) - 1)]


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

    def launch(self, batch: List[Request], span: Tuple[int, int] = (0, 0)):
        k = self.busy.index(False)
        self.busy[k] = True
        start = max(self.clock.now(), self.lane_free[k])
        words = sum(r.n for r in batch)
        end = start + self.cost(words)
        self.lane_free[k] = end
        # the batch as one run of the staging arrays, split by request
        w0, w1 = batch[0].first_word, batch[-1].last_word
        assert all(a.last_word == b.first_word for a, b in zip(batch, batch[1:]))
        perms = []
        for r in batch:
            o = self.st.offsets[r.first_word:r.last_word + 1]
            perms.append(self.sort_fn(self.st.bytes, o))
        h = {"k": k, "start": start, "end": end, "perms": perms, "rids": [r.rid for r in batch],
             "span": span, "words": (w0, w1)}
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
