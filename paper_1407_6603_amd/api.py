"""Python entry points over the libbsort C ABI.

Argument marshalling only: torch provides device memory and the current HIP
stream; every step of the sort runs in libbsort's kernels.  All functions
raise if the HIP library is missing or no GPU is visible.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib

Tuning = _lib.Tuning
BsortError = _lib.BsortError
FLAG_PER_BUCKET_LAUNCH = _lib.FLAG_PER_BUCKET_LAUNCH
FLAG_TILES_ONLY = _lib.FLAG_TILES_ONLY
FLAG_SERIAL_STAGES = _lib.FLAG_SERIAL_STAGES
FLAG_STALL_TEST = _lib.FLAG_STALL_TEST
FLAG_LDS_TILE = _lib.FLAG_LDS_TILE
MAX_LEN = _lib.BSORT_MAX_LEN


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("libbsort runs on a ROCm GPU (gfx950); none is visible")
    _lib.load()


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None or t.numel() == 0:
        return None
    return t.data_ptr()


def _stream(stream: Optional[torch.cuda.Stream]) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_words(bytes_t: torch.Tensor, offsets_t: torch.Tensor):
    if bytes_t.dtype != torch.uint8 or offsets_t.dtype != torch.int64:
        raise TypeError("bytes must be uint8 and offsets int64")
    if not (bytes_t.is_cuda and offsets_t.is_cuda):
        raise ValueError("bytes and offsets must be device tensors")
    if not (bytes_t.is_contiguous() and offsets_t.is_contiguous()):
        raise ValueError("bytes and offsets must be contiguous")
    if offsets_t.dim() != 1 or offsets_t.numel() < 1:
        raise ValueError("offsets must be 1-D with n_words+1 entries")


def tuning(tile_keys: int = 0, merge_threads: int = 0, flags: int = 0,
           hbm_tile_keys: int = 0) -> Tuning:
    return Tuning(tile_keys, merge_threads, flags, hbm_tile_keys)


def workspace_bytes(total_words: int, max_len: int, n_requests: int = 1) -> int:
    n = _lib.load().bsort_workspace_bytes(int(total_words), int(max_len), int(n_requests))
    if n == 0:
        raise ValueError("invalid workspace size arguments")
    return int(n)


class Workspace:
    """Caller-owned device scratch (a uint8 tensor viewed at a 256-byte
    aligned offset).  Reuse one per stream; it grows on demand."""

    def __init__(self, nbytes: int = 0, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.tensor = None
        self.nbytes = 0
        if nbytes:
            self.ensure(nbytes)

    @classmethod
    def wrap(cls, region: "torch.Tensor") -> "Workspace":
        """A workspace over an existing 256-byte aligned uint8 device region
        (no allocation; ensure() raises if a call needs more)."""
        if region.dtype != torch.uint8 or not region.is_cuda or not region.is_contiguous():
            raise ValueError("a workspace region is a contiguous uint8 device tensor")
        if region.data_ptr() % 256:
            raise ValueError("a workspace region must be 256-byte aligned")
        ws = cls(device=region.device)
        ws.tensor = region
        ws.nbytes = region.numel()
        ws.fixed = True
        return ws

    fixed = False

    def ensure(self, nbytes: int):
        if nbytes > self.nbytes and self.fixed:
            raise ValueError(f"workspace region of {self.nbytes} bytes, {nbytes} needed")
        if nbytes > self.nbytes:
            self.tensor = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.nbytes = nbytes
        return self

    @property
    def ptr(self) -> int:
        p = self.tensor.data_ptr()
        return p if self.fixed else (p + 255) & ~255


def _ws_for(ws: Optional[Workspace], nbytes: int, device) -> Workspace:
    if ws is None:
        ws = Workspace(device=device)
    return ws.ensure(nbytes)


def bucketize(bytes_t: torch.Tensor, offsets_t: torch.Tensor, max_len: int,
              ws: Optional[Workspace] = None, stream=None
              ) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    """Sub-arrays by length: (counts[max_len+1], starts[max_len+2], order[n])."""
    _require_gpu()
    _check_words(bytes_t, offsets_t)
    n = offsets_t.numel() - 1
    dev = offsets_t.device
    counts = torch.empty(max_len + 1, dtype=torch.int32, device=dev)
    starts = torch.empty(max_len + 2, dtype=torch.int32, device=dev)
    order = torch.empty(n, dtype=torch.int32, device=dev)
    ws = _ws_for(ws, workspace_bytes(n, max_len, 1), dev)
    w = _lib.Words(_ptr(bytes_t), bytes_t.numel(), _ptr(offsets_t), n, max_len)
    b = _lib.Buckets(_ptr(counts), _ptr(starts), _ptr(order))
    _lib.check(_lib.load().bsort_bucketize(ctypes.byref(w), ctypes.byref(b), ws.ptr,
                                           ws.nbytes, _stream(stream)))
    return counts, starts, order


def sort_buckets(bytes_t: torch.Tensor, offsets_t: torch.Tensor, counts: torch.Tensor,
                 starts: torch.Tensor, order: torch.Tensor, max_len: int,
                 tune: Optional[Tuning] = None, ws: Optional[Workspace] = None,
                 stream=None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Sort the sub-arrays made by bucketize; returns perm[n] (int32)."""
    _require_gpu()
    _check_words(bytes_t, offsets_t)
    n = offsets_t.numel() - 1
    dev = offsets_t.device
    perm = out if out is not None else torch.empty(n, dtype=torch.int32, device=dev)
    ws = _ws_for(ws, workspace_bytes(n, max_len, 1), dev)
    w = _lib.Words(_ptr(bytes_t), bytes_t.numel(), _ptr(offsets_t), n, max_len)
    b = _lib.Buckets(_ptr(counts), _ptr(starts), _ptr(order))
    _lib.check(_lib.load().bsort_sort_buckets(
        ctypes.byref(w), ctypes.byref(b), _ptr(perm),
        ctypes.byref(tune) if tune is not None else None, ws.ptr, ws.nbytes, _stream(stream)))
    return perm


def sort(bytes_t: torch.Tensor, offsets_t: torch.Tensor, max_len: int,
         tune: Optional[Tuning] = None, ws: Optional[Workspace] = None,
         stream=None) -> torch.Tensor:
    """bucketize then sort_buckets: the final order of one word list."""
    counts, starts, order = bucketize(bytes_t, offsets_t, max_len, ws, stream)
    return sort_buckets(bytes_t, offsets_t, counts, starts, order, max_len, tune, ws, stream)


def tokenize(text_t: torch.Tensor, ws: Optional[Workspace] = None, cap_words: Optional[int] = None,
             stream=None, sync: bool = True):
    """Raw text (uint8 device tensor) -> words: maximal runs of ASCII letters,
    every other byte dropped (Section II pre-processing phase 1).

    Returns (bytes_t, offsets_t, max_len).  With sync (the default) the
    call waits for the stream, reads the word count back and returns views
    of exactly the words; with sync=False it returns the full-capacity
    buffers and the device int64[4] result (words, letters, longest word,
    status) instead of max_len."""
    _require_gpu()
    if text_t.dtype != torch.uint8 or text_t.dim() != 1 or not text_t.is_cuda:
        raise ValueError("text must be a 1-D uint8 CUDA tensor")
    if not text_t.is_contiguous():
        raise ValueError("text must be contiguous")
    n = text_t.numel()
    dev = text_t.device
    cap = (n + 1) // 2 if cap_words is None else int(cap_words)
    words = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    offsets = torch.empty(cap + 1, dtype=torch.int64, device=dev)
    result = torch.empty(4, dtype=torch.int64, device=dev)
    L = _lib.load()
    ws = _ws_for(ws, L.bsort_tokenize_workspace_bytes(n), dev)
    _lib.check(L.bsort_tokenize(_ptr(text_t) if n else None, n, _ptr(words), _ptr(offsets), cap,
                                _ptr(result), ws.ptr, ws.nbytes, _stream(stream)))
    if not sync:
        return words, offsets, result
    nw, nl, ml, st = (int(x) for x in result.cpu())
    if st != 0:
        raise _lib.BsortError(st, f"{nw} words exceed cap_words={cap}")
    return words[:nl], offsets[:nw + 1], ml


KEY_BYTES, KEY_LENGTH, KEY_LENGTH_BYTES = _lib.KEY_BYTES, _lib.KEY_LENGTH, _lib.KEY_LENGTH_BYTES


def fixed_width(bytes_t: torch.Tensor, offsets_t: torch.Tensor, width: int, mode: int,
                stream=None, check: bool = True):
    """Every word as a key of one width (the unbucketed ablation): returns
    (bytes_t, offsets_t) of n words of `width` bytes each.  mode: KEY_BYTES,
    KEY_LENGTH or KEY_LENGTH_BYTES.  With check, waits and raises if a word
    did not fit."""
    _require_gpu()
    _check_words(bytes_t, offsets_t)
    n = offsets_t.numel() - 1
    dev = offsets_t.device
    out = torch.empty(max(n * width, 1), dtype=torch.uint8, device=dev)
    offs = torch.empty(n + 1, dtype=torch.int64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    _lib.check(_lib.load().bsort_fixed_width(_ptr(bytes_t), bytes_t.numel(), _ptr(offsets_t), n,
                                             width, mode,
                                             _ptr(out), _ptr(offs), _ptr(status),
                                             _stream(stream)))
    if check and int(status.cpu()) != 0:
        raise _lib.BsortError(2, f"a word does not fit a {width}-byte key")
    return out[:n * width], offs


LAYOUT_PACKED, LAYOUT_TEXT = _lib.LAYOUT_PACKED, _lib.LAYOUT_TEXT


def oets_buckets(bytes_t: torch.Tensor, offsets_t: torch.Tensor, counts: torch.Tensor,
                 starts: torch.Tensor, order: torch.Tensor, max_len: int, layout: int,
                 stream=None, out: Optional[torch.Tensor] = None, check: bool = True):
    """Data-structure ablation: each sub-array (from bucketize) sorted whole by
    one workgroup, the words held as packed keys (LAYOUT_PACKED) or read from
    the text through the offsets (LAYOUT_TEXT).  Returns perm."""
    _require_gpu()
    _check_words(bytes_t, offsets_t)
    n = offsets_t.numel() - 1
    dev = offsets_t.device
    perm = out if out is not None else torch.empty(n, dtype=torch.int32, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    w = _lib.Words(_ptr(bytes_t), bytes_t.numel(), _ptr(offsets_t), n, max_len)
    b = _lib.Buckets(_ptr(counts), _ptr(starts), _ptr(order))
    _lib.check(_lib.load().bsort_oets_buckets(ctypes.byref(w), ctypes.byref(b), _ptr(perm),
                                              layout, _ptr(status), _stream(stream)))
    if check:
        st = int(status.cpu())
        if st:
            raise _lib.BsortError(1, f"layout sort status {st} (1: a sub-array did not fit "
                                     "LDS, 2: order or offsets out of range)")
    return perm


def sort_text(text_t: torch.Tensor, tune: Optional[Tuning] = None,
              ws: Optional[Workspace] = None, stream=None):
    """The paper's three phases on raw text: tokenize, then sort the words
    by (length, bytes).  Returns (bytes_t, offsets_t, perm_t)."""
    words, offsets, ml = tokenize(text_t, ws=ws, stream=stream)
    if offsets.numel() == 1:
        return words, offsets, torch.empty(0, dtype=torch.int32, device=text_t.device)
    if ml > MAX_LEN:
        raise _lib.BsortError(2, f"a word of {ml} bytes exceeds the {MAX_LEN}-byte limit")
    perm = sort(words, offsets, max(ml, 1), tune=tune, ws=ws, stream=stream)
    return words, offsets, perm


def sort_batch(bytes_t: torch.Tensor, offsets_t: torch.Tensor, req_start_t: torch.Tensor,
               h_req_start: np.ndarray, max_len: int, tune: Optional[Tuning] = None,
               ws: Optional[Workspace] = None, stream=None,
               out: Optional[torch.Tensor] = None, byte_origin: int = 0) -> torch.Tensor:
    """Sort R lists stored back to back; perm holds list-local indices.

    ``byte_origin``: bytes_t holds bytes [byte_origin, byte_origin +
    numel) of the byte stream the offsets index (offsets[0] >= byte_origin)."""
    _require_gpu()
    _check_words(bytes_t, offsets_t)
    h = np.ascontiguousarray(h_req_start, dtype=np.int64)
    R = len(h) - 1
    total = int(h[-1]) if R > 0 else 0
    dev = offsets_t.device
    perm = out if out is not None else torch.empty(total, dtype=torch.int32, device=dev)
    ws = _ws_for(ws, workspace_bytes(total, max_len, max(R, 0)), dev)
    bptr = (bytes_t.data_ptr() - int(byte_origin)) if bytes_t.numel() else None
    b = _lib.Batch(bptr, int(byte_origin) + bytes_t.numel(), _ptr(offsets_t), _ptr(req_start_t),
                   h.ctypes.data, R, max_len)
    _lib.check(_lib.load().bsort_sort_batch(
        ctypes.byref(b), _ptr(perm), ctypes.byref(tune) if tune is not None else None,
        ws.ptr, ws.nbytes, _stream(stream)))
    return perm


STATIC_SCRATCH_BYTES = _lib.STATIC_SCRATCH_BYTES


def sort_batch_static(bytes_t: torch.Tensor, offsets_t: torch.Tensor, req_start_t: torch.Tensor,
                      h_req_start: np.ndarray, max_len: int, out: torch.Tensor,
                      status: Optional[torch.Tensor] = None, tune: Optional[Tuning] = None,
                      stream=None) -> torch.Tensor:
    """sort_batch without a workspace or any allocation: the library's static
    per-GPU scratch (STATIC_SCRATCH_BYTES) holds the work.  The caller gives
    perm (``out``) and optionally a device uint32 ``status`` (the call's
    device status word, 0 when clean)."""
    _require_gpu()
    _check_words(bytes_t, offsets_t)
    h = np.ascontiguousarray(h_req_start, dtype=np.int64)
    R = len(h) - 1
    b = _lib.Batch(_ptr(bytes_t), bytes_t.numel(), _ptr(offsets_t), _ptr(req_start_t),
                   h.ctypes.data, R, max_len)
    st = status.data_ptr() if status is not None else None
    _lib.check(_lib.load().bsort_sort_batch_static(
        ctypes.byref(b), _ptr(out), ctypes.byref(tune) if tune is not None else None, st,
        _stream(stream)))
    return out


def stage_names(max_len: int):
    """Names of the stages of a batch sort, in launch order."""
    L = _lib.load()
    return [L.bsort_stage_name(max_len, i).decode() for i in range(L.bsort_stage_count(max_len))]


class StageTimer:
    """HIP events for bsort_sort_batch_staged: a begin and an end event per
    stage, recorded on the stream that runs the stage.  ``only``: the names of
    the stages to time (default all); the others record nothing."""

    def __init__(self, max_len: int, stream=None, only=None):
        self.names = stage_names(max_len)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.timed = [i for i, n in enumerate(self.names) if only is None or n in only]
        self.events = [None] * (2 * len(self.names))
        for i in self.timed:
            for k in (2 * i, 2 * i + 1):
                e = torch.cuda.Event(enable_timing=True)
                e.record(self.stream)          # torch creates the HIP event on first record
                self.events[k] = e
        self.handles = (ctypes.c_void_p * len(self.events))(
            *[e.cuda_event if e is not None else None for e in self.events])

    def _sync(self):
        for e in self.events:
            if e is not None:
                e.synchronize()

    def ms(self):
        """Per-stage device milliseconds of the last staged sort (waits for
        it), for the timed stages."""
        self._sync()
        return {self.names[i]: self.events[2 * i].elapsed_time(self.events[2 * i + 1])
                for i in self.timed}

    def span_ms(self, pick):
        """Milliseconds from the earliest start to the latest end of the
        timed stages whose names satisfy pick (stages may overlap)."""
        idx = [i for i in self.timed if pick(self.names[i])]
        if not idx:
            return 0.0
        self._sync()
        ref = self.events[2 * self.timed[0]]
        t0 = min(ref.elapsed_time(self.events[2 * i]) for i in idx)
        t1 = max(ref.elapsed_time(self.events[2 * i + 1]) for i in idx)
        return t1 - t0


def sort_batch_staged(bytes_t, offsets_t, req_start_t, h_req_start, max_len: int,
                      timer: StageTimer, tune: Optional[Tuning] = None,
                      ws: Optional[Workspace] = None, out: Optional[torch.Tensor] = None):
    """sort_batch that records timer's events between stages on timer.stream."""
    _require_gpu()
    _check_words(bytes_t, offsets_t)
    h = np.ascontiguousarray(h_req_start, dtype=np.int64)
    R = len(h) - 1
    total = int(h[-1]) if R > 0 else 0
    dev = offsets_t.device
    perm = out if out is not None else torch.empty(total, dtype=torch.int32, device=dev)
    ws = _ws_for(ws, workspace_bytes(total, max_len, max(R, 0)), dev)
    b = _lib.Batch(_ptr(bytes_t), bytes_t.numel(), _ptr(offsets_t), _ptr(req_start_t),
                   h.ctypes.data, R, max_len)
    _lib.check(_lib.load().bsort_sort_batch_staged(
        ctypes.byref(b), _ptr(perm), ctypes.byref(tune) if tune is not None else None,
        ws.ptr, ws.nbytes, ctypes.c_void_p(timer.stream.cuda_stream), timer.handles,
        len(timer.events)))
    return perm


def device_status(ws: Workspace, stream=None) -> int:
    """Synchronise and return (then clear) the workspace status word."""
    return int(_lib.load().bsort_get_device_status(ws.ptr, _stream(stream)))


def check_device_status(ws: Workspace, stream=None):
    _lib.check(device_status(ws, stream))


class Plan:
    """A batch sort captured into a HIP graph for batches up to a capacity."""

    def __init__(self, cap_words: int, cap_requests: int, cap_request_words: int, max_len: int,
                 tune: Optional[Tuning] = None, stream=None):
        _require_gpu()
        self._lib = _lib.load()
        self._p = ctypes.c_void_p()
        _lib.check(self._lib.bsort_plan_create(
            ctypes.byref(self._p), int(cap_words), int(cap_requests), int(cap_request_words),
            int(max_len), ctypes.byref(tune) if tune is not None else None, _stream(stream)))
        self.max_len = max_len
        self.workspace_bytes = int(self._lib.bsort_plan_workspace_bytes(self._p))

    def execute(self, bytes_t, offsets_t, req_start_t, h_req_start, ws: Workspace,
                stream=None, out: Optional[torch.Tensor] = None, max_len: Optional[int] = None):
        _check_words(bytes_t, offsets_t)
        h = np.ascontiguousarray(h_req_start, dtype=np.int64)
        R = len(h) - 1
        total = int(h[-1]) if R > 0 else 0
        perm = out if out is not None else torch.empty(total, dtype=torch.int32,
                                                       device=offsets_t.device)
        ws.ensure(self.workspace_bytes)
        ml = self.max_len if max_len is None else max_len
        b = _lib.Batch(_ptr(bytes_t), bytes_t.numel(), _ptr(offsets_t), _ptr(req_start_t),
                       h.ctypes.data, R, ml)
        _lib.check(self._lib.bsort_plan_execute(self._p, ctypes.byref(b), _ptr(perm), ws.ptr,
                                                ws.nbytes, _stream(stream)))
        return perm

    def close(self):
        if self._p:
            self._lib.bsort_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_device(bytes_np: np.ndarray, offsets_np: np.ndarray, device="cuda"):
    """Host word arrays -> device tensors (uint8 bytes, int64 offsets)."""
    b = torch.from_numpy(np.ascontiguousarray(bytes_np, dtype=np.uint8))
    if b.numel() == 0:
        b = torch.zeros(1, dtype=torch.uint8)
    o = torch.from_numpy(np.ascontiguousarray(offsets_np, dtype=np.int64))
    return b.to(device), o.to(device)
