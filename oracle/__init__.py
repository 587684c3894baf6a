"""CPU oracle for length-bucketed bubble sort of words.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The GPU library neither imports nor
links anything here, and nothing here uses the GPU library.

Contents
--------
* ``bubble_sort`` -- the paper's procedure (Section II pre-processing phases
  2-3; Section III approach one step 4): sub-arrays by word length, filled in
  input order, each bubble-sorted in ASCII byte order, concatenated shortest
  first.  Plain C (``bsort_oracle.c``), optionally one sub-array per OpenMP
  thread ("Bubble sort in OpenMP").
* ``bubble_sort_batch`` -- the same over many independent word lists.
* ``definition_sort`` / ``definition_sort_batch`` -- the result's definition
  written out: the permutation ordering words by (length, unsigned bytes,
  original index), via qsort_r.
* ``bucketize`` -- sub-array sizes, their exclusive scan, and the unsorted
  sub-array contents (the paper's count array and sub-array fill).
* ``pack_keys`` -- fixed-width big-endian uint64 key lanes of equal-length
  words (Section III approach two: one fixed width per sub-array).
* ``bubble_sort_whole`` -- Section II, Table 1 rows 2-3: the whole list
  bubble-sorted without sub-arrays, by alphabetic order, by length, or by
  length then bytes.
* ``tokenize`` -- Section II pre-processing phase 1: raw text to words,
  a word being a maximal run of ASCII letters (every other byte, the paper's
  "special characters" among them, separates words and is dropped).
* ``brute_force`` -- pure Python, tiny inputs only: tries every permutation
  and returns the unique one along which (length, bytes, index) strictly
  increases.

Readings where the paper is silent: bytes compare unsigned; ties keep input
order; length = byte count; length-0 words form sub-array 0.
"""
from __future__ import annotations

import contextlib
import ctypes
import itertools
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bsort_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, E_INVALID, E_TOO_LONG, E_NO_MEMORY = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP on)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        _lib = _load(LIB)
    return _lib


@contextlib.contextmanager
def using_library(path: str):
    """Run the Python wrappers against another build of the C oracle (used
    by the tests that plant a mistake in a copy of the oracle)."""
    global _lib
    saved = _lib
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def _load(path: str):
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    L.oracle_bucketize.argtypes = [P, i64, P, i32, i32, P, P, P]
    L.oracle_bubble_sort.argtypes = [P, i64, P, i32, i32, ctypes.c_int, ctypes.c_int,
                                     P, P, P, P, P]
    L.oracle_bubble_sort_batch.argtypes = [P, i64, P, P, i32, i32, ctypes.c_int,
                                           ctypes.c_int, P, P]
    L.oracle_definition_sort.argtypes = [P, i64, P, i32, P]
    L.oracle_definition_sort_batch.argtypes = [P, i64, P, P, i32, ctypes.c_int, P]
    L.oracle_pack_keys.argtypes = [P, P, P, i32, i32, P]
    L.oracle_max_threads.argtypes = []
    L.oracle_tokenize.argtypes = [P, i64, P, P, i64, P, P]
    L.oracle_bubble_sort_whole.argtypes = [P, i64, P, i32, ctypes.c_int, P, P]
    for f in (L.oracle_bucketize, L.oracle_bubble_sort, L.oracle_bubble_sort_batch,
              L.oracle_definition_sort, L.oracle_definition_sort_batch, L.oracle_pack_keys,
              L.oracle_max_threads, L.oracle_tokenize, L.oracle_bubble_sort_whole):
        f.restype = ctypes.c_int
    return L


class OracleError(RuntimeError):
    pass


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def _prep(bytes_: np.ndarray, offsets: np.ndarray):
    b = np.ascontiguousarray(bytes_, dtype=np.uint8)
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    if b.size == 0:
        b = np.zeros(1, dtype=np.uint8)   # a valid pointer for empty text
        nb = 0
    else:
        nb = b.size
    return b, o, nb


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(f"{what}: oracle status {rc}")


def default_max_len(offsets: np.ndarray) -> int:
    return int(np.diff(offsets).max()) if len(offsets) > 1 else 0


WHOLE_ALPHABETIC, WHOLE_LENGTH, WHOLE_LENGTH_BYTES = 0, 1, 2


def bubble_sort_whole(bytes_, offsets, key: int) -> Tuple[np.ndarray, int]:
    """Section II, Table 1 rows 2-3: one bubble sort over the whole list, no
    sub-arrays, by alphabetic order (WHOLE_ALPHABETIC), by length
    (WHOLE_LENGTH) or by length then bytes (WHOLE_LENGTH_BYTES).  Returns
    (perm, comparisons).  O(n^2): small lists only."""
    b, o, nb = _prep(bytes_, offsets)
    n = len(o) - 1
    perm = np.zeros(max(n, 1), dtype=np.int32)
    cmp = ctypes.c_int64(0)
    _check(lib().oracle_bubble_sort_whole(_ptr(b), nb, _ptr(o), n, key, _ptr(perm),
                                          ctypes.byref(cmp)), "bubble_sort_whole")
    return perm[:n], cmp.value


def tokenize(text) -> Tuple[np.ndarray, np.ndarray]:
    """Section II pre-processing phase 1: raw text (bytes or uint8 array) ->
    (letters of the words back to back, int64 offsets[n_words + 1]).  A word
    is a maximal run of ASCII letters; every other byte is dropped."""
    t = np.frombuffer(text, dtype=np.uint8) if isinstance(text, (bytes, bytearray)) \
        else np.ascontiguousarray(text, dtype=np.uint8)
    n = t.size
    src = t if n else np.zeros(1, dtype=np.uint8)
    out = np.zeros(max(n, 1), dtype=np.uint8)
    cap = (n + 1) // 2
    offsets = np.zeros(cap + 1, dtype=np.int64)
    nw, nl = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().oracle_tokenize(_ptr(src), n, _ptr(out), _ptr(offsets), cap,
                                 ctypes.byref(nw), ctypes.byref(nl)), "tokenize")
    return out[:nl.value].copy(), offsets[:nw.value + 1].copy()


def bucketize(bytes_, offsets, max_len: Optional[int] = None):
    """(counts[max_len+1], starts[max_len+2], order[n])."""
    b, o, nb = _prep(bytes_, offsets)
    n = len(o) - 1
    ml = default_max_len(o) if max_len is None else max_len
    counts = np.zeros(ml + 1, np.int32)
    starts = np.zeros(ml + 2, np.int32)
    order = np.zeros(max(n, 1), np.int32)
    _check(lib().oracle_bucketize(_ptr(b), nb, _ptr(o), n, ml, _ptr(counts), _ptr(starts),
                                  _ptr(order)), "bucketize")
    return counts, starts, order[:n]


def bubble_sort(bytes_, offsets, max_len: Optional[int] = None, early_exit: bool = False,
                threads: int = 1, with_buckets: bool = False):
    """The paper's bucket-then-bubble procedure.

    Returns perm (int32[n]); with ``with_buckets`` also counts, starts, order
    and the number of comparisons made."""
    b, o, nb = _prep(bytes_, offsets)
    n = len(o) - 1
    ml = default_max_len(o) if max_len is None else max_len
    perm = np.zeros(max(n, 1), np.int32)
    counts = np.zeros(ml + 1, np.int32)
    starts = np.zeros(ml + 2, np.int32)
    order = np.zeros(max(n, 1), np.int32)
    cmp = ctypes.c_int64(0)
    _check(lib().oracle_bubble_sort(_ptr(b), nb, _ptr(o), n, ml, int(early_exit), threads,
                                    _ptr(perm), _ptr(counts), _ptr(starts), _ptr(order),
                                    ctypes.byref(cmp)), "bubble_sort")
    if with_buckets:
        return perm[:n], counts, starts, order[:n], int(cmp.value)
    return perm[:n]


def bubble_sort_batch(bytes_, offsets, req_start, max_len: int, early_exit: bool = False,
                      threads: int = 1):
    """Per-list bubble procedure over back-to-back lists; list-local perm."""
    b, o, nb = _prep(bytes_, offsets)
    rs = np.ascontiguousarray(req_start, dtype=np.int64)
    R = len(rs) - 1
    total = int(rs[-1]) if R >= 0 else 0
    perm = np.zeros(max(total, 1), np.int32)
    cmp = ctypes.c_int64(0)
    _check(lib().oracle_bubble_sort_batch(_ptr(b), nb, _ptr(o), _ptr(rs), R, max_len,
                                          int(early_exit), threads, _ptr(perm),
                                          ctypes.byref(cmp)), "bubble_sort_batch")
    return perm[:total], int(cmp.value)


def definition_sort(bytes_, offsets):
    b, o, nb = _prep(bytes_, offsets)
    n = len(o) - 1
    perm = np.zeros(max(n, 1), np.int32)
    _check(lib().oracle_definition_sort(_ptr(b), nb, _ptr(o), n, _ptr(perm)),
           "definition_sort")
    return perm[:n]


def definition_sort_batch(bytes_, offsets, req_start, threads: int = 1):
    """The definition per list over back-to-back lists; list-local perm."""
    b, o, nb = _prep(bytes_, offsets)
    rs = np.ascontiguousarray(req_start, dtype=np.int64)
    R = len(rs) - 1
    total = int(rs[-1]) if R >= 0 else 0
    perm = np.zeros(max(total, 1), np.int32)
    _check(lib().oracle_definition_sort_batch(_ptr(b), nb, _ptr(o), _ptr(rs), R, threads,
                                              _ptr(perm)), "definition_sort_batch")
    return perm[:total]


def pack_keys(bytes_, offsets, idx, L: int) -> np.ndarray:
    """uint64 lanes [W, m] of the words idx (all of length L)."""
    b, o, _ = _prep(bytes_, offsets)
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    W = (L + 7) // 8
    m = len(ix)
    lanes = np.zeros(max(W * m, 1), np.uint64)
    _check(lib().oracle_pack_keys(_ptr(b), _ptr(o), _ptr(ix), m, L, _ptr(lanes)),
           "pack_keys")
    return lanes[:W * m].reshape(W, m)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


# ---------------------------------------------------------------------------
# Pure-Python brute force (tiny inputs)
# ---------------------------------------------------------------------------

def _less(words: Sequence[bytes], i: int, j: int) -> bool:
    """(len, bytes, index) of word i is below that of word j.  bytes values
    compare element by element as integers 0..255, i.e. unsigned."""
    a, b = words[i], words[j]
    if len(a) != len(b):
        return len(a) < len(b)
    for x, y in zip(a, b):
        if x != y:
            return x < y
    return i < j


def brute_force(words: Sequence[bytes]) -> List[int]:
    """Try every permutation; return the one along which (length, bytes,
    index) strictly increases.  Exactly one exists (the key is a total
    order).  n <= 8."""
    n = len(words)
    if n > 8:
        raise ValueError("brute force is for n <= 8")
    found = None
    for p in itertools.permutations(range(n)):
        if all(_less(words, p[k], p[k + 1]) for k in range(n - 1)):
            if found is not None:
                raise AssertionError("two orders satisfy a strict total order")
            found = list(p)
    if found is None:
        found = []
    return found
