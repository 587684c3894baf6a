"""Seeded synthetic English-like word streams.

The paper sorts words taken from two Hamlet text files (190 KB and 1.38 MB,
Section II) that are not available here.  This module makes seeded stand-ins
of the same shape: English word-length statistics (mode 3-4, geometric tail),
letters drawn by English letter frequency, a Zipf-distributed vocabulary with
heavy duplicates, and a 5% chance that a token starts with a capital letter.

It holds no part of the sorting method.  It only produces inputs, in the form
both the CPU oracle and the GPU library take: a packed byte buffer of words
with no separators plus an int64 offsets array of length n+1, so word i is
``bytes[offsets[i]:offsets[i+1]]``.

Randomness: numpy ``Generator(PCG64)`` seeded from ``SeedSequence``.  Every
workload is a pure function of its seed.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import functools
import multiprocessing
import os
from typing import List, Optional, Sequence

import numpy as np

# Relative frequencies of the letters a..z in English text (percent), as
# tabulated by R. E. Lewand, "Cryptological Mathematics", MAA, 2000.
LETTER_FREQ_PCT = np.array([
    8.167, 1.492, 2.782, 4.253, 12.702, 2.228, 2.015, 6.094, 6.966, 0.153,
    0.772, 4.025, 2.406, 6.749, 7.507, 1.929, 0.095, 5.987, 6.327, 9.056,
    2.758, 0.978, 2.360, 0.150, 1.974, 0.074])
LETTER_P = LETTER_FREQ_PCT / LETTER_FREQ_PCT.sum()

CAPITAL_P = 0.05


def length_pmf(lmax: int) -> np.ndarray:
    """English-like word-length pmf over 1..lmax (index 0 is length 1).

    Weights 0.03, 0.16, 0.21, 0.18 for lengths 1-4, then 0.18 * 0.72**(L-4)
    for L >= 5, truncated at lmax and renormalised.
    """
    if lmax < 1:
        raise ValueError("lmax must be >= 1")
    w = np.empty(lmax)
    head = [0.03, 0.16, 0.21, 0.18]
    for i in range(lmax):
        L = i + 1
        w[i] = head[i] if L <= 4 else 0.18 * 0.72 ** (L - 4)
    return w / w.sum()


def zipf_weights(V: int, s: float) -> np.ndarray:
    r = np.arange(1, V + 1, dtype=np.float64)
    z = r ** (-s)
    return z / z.sum()


@functools.lru_cache(maxsize=32)
def _length_assignment(V: int, lmax: int, s: float) -> tuple:
    """Word length of each vocabulary rank (rank 1 first).

    Ranks are visited from most to least frequent; each goes to the length
    whose remaining target token mass (pmf minus mass already assigned) is
    largest, so the token length histogram tracks the pmf despite the heavy
    Zipf head.  Short lengths have few distinct strings (26**L); a full
    length class drops out and its mass spills to the others.
    """
    pmf = length_pmf(lmax)
    z = zipf_weights(V, s)
    remaining = pmf.copy()
    cap = np.array([26 ** L if L <= 4 else np.iinfo(np.int64).max
                    for L in range(1, lmax + 1)], dtype=np.float64)
    used = np.zeros(lmax, dtype=np.int64)
    out = np.empty(V, dtype=np.int64)
    for r in range(V):
        i = int(np.argmax(remaining))
        out[r] = i + 1
        remaining[i] -= z[r]
        used[i] += 1
        if used[i] >= cap[i]:
            remaining[i] = -np.inf
    return tuple(out.tolist())


@functools.lru_cache(maxsize=4)
def _log_string_p(L: int) -> np.ndarray:
    p = LETTER_P
    for _ in range(L - 1):
        p = np.outer(p, LETTER_P).ravel()
    return np.log(p)


def _distinct_strings(rng: np.random.Generator, L: int, m: int) -> np.ndarray:
    """m distinct lowercase strings of length L as a (m, L) uint8 array."""
    if m == 0:
        return np.zeros((0, L), dtype=np.uint8)
    if L <= 3:
        # small spaces: weighted sampling without replacement over all 26**L
        # strings (weight = product of letter probabilities) by the
        # Gumbel-top-k construction
        logp = _log_string_p(L)
        keys = logp + rng.gumbel(size=logp.shape)
        if m < len(keys):
            top = np.argpartition(-keys, m - 1)[:m]
            codes = top[np.argsort(-keys[top], kind="stable")]
        else:
            codes = np.argsort(-keys, kind="stable")
        digits = np.empty((m, L), dtype=np.uint8)
        for j in range(L - 1, -1, -1):
            digits[:, j] = codes % 26
            codes = codes // 26
        return digits + ord('a')
    if L <= 13:
        # base-26 codes fit in int64: dedupe vectorised, keep first occurrences
        pool = np.zeros((0, L), dtype=np.uint8)
        while True:
            want = int(m * 1.25) + 16
            cand = rng.choice(26, size=(want, L), p=LETTER_P).astype(np.uint8)
            pool = np.concatenate([pool, cand])
            codes = np.zeros(len(pool), dtype=np.int64)
            for j in range(L):
                codes = codes * 26 + pool[:, j]
            _, first = np.unique(codes, return_index=True)
            if len(first) >= m:
                keep = np.sort(first)[:m]
                return pool[keep] + ord('a')
    rows: List[np.ndarray] = []
    have = 0
    seen = set()
    while have < m:
        want = int((m - have) * 1.2) + 16
        cand = rng.choice(26, size=(want, L), p=LETTER_P).astype(np.uint8) + ord('a')
        for row in cand:
            key = row.tobytes()
            if key in seen:
                continue
            seen.add(key)
            rows.append(row)
            have += 1
            if have == m:
                break
    return np.stack(rows)


@dataclasses.dataclass
class Vocab:
    """Vocabulary in rank order (rank 1 = index 0)."""
    bytes: np.ndarray     # uint8, concatenated
    offsets: np.ndarray   # int64 [V+1]
    zipf_s: float

    @property
    def V(self) -> int:
        return len(self.offsets) - 1

    def word(self, r: int) -> bytes:
        return self.bytes[self.offsets[r]:self.offsets[r + 1]].tobytes()


def make_vocab(rng: np.random.Generator, V: int, lmax: int, s: float) -> Vocab:
    lens = np.array(_length_assignment(V, lmax, s), dtype=np.int64)
    per_len = {}
    for L in range(1, lmax + 1):
        m = int((lens == L).sum())
        per_len[L] = _distinct_strings(rng, L, m)
    offsets = np.zeros(V + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    out = np.empty(int(offsets[-1]), dtype=np.uint8)
    # place each class's strings at its ranks, in increasing rank order
    for L, arr in per_len.items():
        ranks = np.nonzero(lens == L)[0]
        if len(ranks) == 0:
            continue
        idx = offsets[ranks][:, None] + np.arange(L)[None, :]
        out[idx.ravel()] = arr.ravel()
    return Vocab(out, offsets, s)


@dataclasses.dataclass
class Words:
    """A list of words: ``bytes[offsets[i]:offsets[i+1]]`` is word i."""
    bytes: np.ndarray     # uint8
    offsets: np.ndarray   # int64 [n+1], offsets[0] == 0

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def word(self, i: int) -> bytes:
        return self.bytes[self.offsets[i]:self.offsets[i + 1]].tobytes()

    def as_list(self) -> List[bytes]:
        b = self.bytes.tobytes()
        o = self.offsets
        return [b[o[i]:o[i + 1]] for i in range(self.n)]

    @staticmethod
    def from_list(words: Sequence[bytes]) -> "Words":
        lens = np.array([len(w) for w in words], dtype=np.int64)
        offsets = np.zeros(len(words) + 1, dtype=np.int64)
        np.cumsum(lens, out=offsets[1:])
        buf = np.frombuffer(b"".join(words), dtype=np.uint8).copy()
        return Words(buf, offsets)


def draw_tokens(rng: np.random.Generator, vocab: Vocab, n: int,
                cap_p: float = CAPITAL_P) -> Words:
    """n tokens: Zipf ranks by inverse CDF, 5% capitalised first letter."""
    z = zipf_weights(vocab.V, vocab.zipf_s)
    cdf = np.cumsum(z)
    u = rng.random(n)
    ranks = np.searchsorted(cdf, u * cdf[-1], side="right")
    np.minimum(ranks, vocab.V - 1, out=ranks)
    cap = rng.random(n) < cap_p
    vlen = np.diff(vocab.offsets)
    lens = vlen[ranks]
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    total = int(offsets[-1])
    src = np.repeat(vocab.offsets[ranks] - offsets[:-1], lens) + np.arange(total, dtype=np.int64)
    out = vocab.bytes[src]
    first = offsets[:-1][cap & (lens > 0)]
    out[first] -= 32          # 'a'..'z' -> 'A'..'Z'
    return Words(out, offsets)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class SingleSpec:
    n: int
    V: int
    lmax: int
    zipf_s: float
    seed: int


SINGLE = {
    1: SingleSpec(n=2_000, V=800, lmax=12, zipf_s=1.1, seed=1),
    2: SingleSpec(n=35_000, V=5_000, lmax=20, zipf_s=1.1, seed=2),
    3: SingleSpec(n=250_000, V=25_000, lmax=24, zipf_s=1.05, seed=3),
}


def single(k: int) -> Words:
    """Single-request workloads 1-3: a 2,000-word small case, a ~190 KB
    stand-in for the first Hamlet file and a ~1.38 MB stand-in for the
    second."""
    sp = SINGLE[k]
    return single_from_spec(sp)


def single_from_spec(sp: SingleSpec) -> Words:
    ss = np.random.SeedSequence(sp.seed)
    vs, ts = ss.spawn(2)
    vocab = make_vocab(np.random.Generator(np.random.PCG64(vs)), sp.V, sp.lmax, sp.zipf_s)
    return draw_tokens(np.random.Generator(np.random.PCG64(ts)), vocab, sp.n)


@dataclasses.dataclass
class Batch:
    """R requests back to back: request r holds global words
    req_start[r] .. req_start[r+1]-1."""
    bytes: np.ndarray
    offsets: np.ndarray      # int64 [total+1], global
    req_start: np.ndarray    # int64 [R+1]

    @property
    def R(self) -> int:
        return len(self.req_start) - 1

    @property
    def total(self) -> int:
        return int(self.req_start[-1])

    def request(self, r: int) -> Words:
        a, b = int(self.req_start[r]), int(self.req_start[r + 1])
        o = self.offsets[a:b + 1]
        return Words(self.bytes[o[0]:o[-1]].copy(), o - o[0])

    @staticmethod
    def concat(reqs: Sequence[Words]) -> "Batch":
        R = len(reqs)
        req_start = np.zeros(R + 1, dtype=np.int64)
        np.cumsum([w.n for w in reqs], out=req_start[1:])
        total = int(req_start[-1])
        offsets = np.zeros(total + 1, dtype=np.int64)
        base = 0
        for r, w in enumerate(reqs):
            a = int(req_start[r])
            offsets[a:a + w.n + 1] = w.offsets + base
            base += int(w.offsets[-1])
        buf = np.concatenate([w.bytes for w in reqs]) if R else np.zeros(0, np.uint8)
        return Batch(buf.astype(np.uint8, copy=False), offsets, req_start)


BATCH_R = 4096
BATCH_NMIN = 16
BATCH_NMAX = 65_536
BATCH_SEED = 4


def batch_sizes(R: int = BATCH_R, seed: int = BATCH_SEED,
                nmin: int = BATCH_NMIN, nmax: int = BATCH_NMAX) -> np.ndarray:
    """Request sizes, log-uniform on [nmin, nmax): floor(nmin*(nmax/nmin)**u)."""
    ss = np.random.SeedSequence(seed)
    size_ss = ss.spawn(1)[0]
    u = np.random.Generator(np.random.PCG64(size_ss)).random(R)
    return np.floor(nmin * (nmax / nmin) ** u).astype(np.int64)


def batch_request(r: int, n: int, seed: int = BATCH_SEED) -> Words:
    """Request r of the batching workload: built like workload 1 (800-word
    vocabulary, lengths 1-12, Zipf 1.1) from its own seed."""
    req_ss = np.random.SeedSequence(seed, spawn_key=(1, r))
    vs, ts = req_ss.spawn(2)
    vocab = make_vocab(np.random.Generator(np.random.PCG64(vs)), 800, 12, 1.1)
    return draw_tokens(np.random.Generator(np.random.PCG64(ts)), vocab, int(n))


def batch(R: int = BATCH_R, first: int = 0, count: Optional[int] = None,
          seed: int = BATCH_SEED, workers: Optional[int] = None) -> Batch:
    """Workload 4: R independent requests, sizes log-uniform in [16, 65,536].

    ``first``/``count`` select a contiguous sub-range of the same R requests
    (the same words as in the full workload).  ``workers`` > 1 generates in
    that many worker processes (same result)."""
    sizes = batch_sizes(R, seed)
    if count is None:
        count = R - first
    ids = list(range(first, first + count))
    if workers is None:
        workers = 1
    if workers > 1:
        # worker processes: only start them from a process that has not yet
        # opened a GPU (a profiler's preload library may open it before main)
        ctx = multiprocessing.get_context("spawn")
        with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
            reqs = list(ex.map(batch_request, ids, [int(sizes[r]) for r in ids],
                               [seed] * len(ids), chunksize=64))
    else:
        reqs = [batch_request(r, sizes[r], seed) for r in ids]
    return Batch.concat(reqs)


@dataclasses.dataclass
class ServeSpec:
    n_arrivals: int = 2_000
    rate_per_s: float = 2_000.0
    nmin: int = 1_000
    nmax: int = 1_000_000
    big_n: int = 4_000_000
    big_at: int = 1_000
    V: int = 200_000
    lmax: int = 32
    zipf_s: float = 1.0
    seed: int = 5


def serve_arrivals(spec: ServeSpec = ServeSpec()):
    """Workload 5 arrival schedule: (arrival_time_s, n_words) per request.

    Poisson arrivals (exponential inter-arrival times, mean 1/rate); sizes
    log-uniform on [nmin, nmax); one request of big_n words is inserted as
    arrival number big_at."""
    ss = np.random.SeedSequence(spec.seed)
    arr_ss, size_ss = ss.spawn(2)
    gaps = np.random.Generator(np.random.PCG64(arr_ss)).exponential(
        1.0 / spec.rate_per_s, spec.n_arrivals)
    times = np.cumsum(gaps) - gaps[0]
    u = np.random.Generator(np.random.PCG64(size_ss)).random(spec.n_arrivals)
    sizes = np.floor(spec.nmin * (spec.nmax / spec.nmin) ** u).astype(np.int64)
    times = np.insert(times, spec.big_at, times[spec.big_at - 1] if spec.big_at else 0.0)
    sizes = np.insert(sizes, spec.big_at, spec.big_n)
    return times, sizes


@functools.lru_cache(maxsize=2)
def serve_vocab(V: int, lmax: int, s: float, seed: int) -> Vocab:
    vs = np.random.SeedSequence(seed, spawn_key=(7,))
    return make_vocab(np.random.Generator(np.random.PCG64(vs)), V, lmax, s)


def serve_request(i: int, n: int, spec: ServeSpec = ServeSpec()) -> Words:
    vocab = serve_vocab(spec.V, spec.lmax, spec.zipf_s, spec.seed)
    ts = np.random.SeedSequence(spec.seed, spawn_key=(8, i))
    return draw_tokens(np.random.Generator(np.random.PCG64(ts)), vocab, int(n))


def _serve_request_packed(i: int, n: int, spec: ServeSpec):
    w = serve_request(i, n, spec)
    return w.bytes, np.diff(w.offsets).astype(np.uint8)


@dataclasses.dataclass
class ServeWorkload:
    """The serving workload: every request's words back to back (as a
    Batch, request r = arrival r) and the arrival times in seconds."""
    batch: Batch
    arrivals: np.ndarray


def serve(spec: ServeSpec = ServeSpec(), workers: Optional[int] = None,
          count: Optional[int] = None) -> ServeWorkload:
    """Workload 5: all arrivals of ``spec`` (the first ``count`` if given),
    generated in ``workers`` worker processes when > 1 (same result)."""
    times, sizes = serve_arrivals(spec)
    if count is not None:
        times, sizes = times[:count], sizes[:count]
    ids = list(range(len(sizes)))
    if workers is not None and workers > 1:
        ctx = multiprocessing.get_context("spawn")
        with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
            parts = list(ex.map(_serve_request_packed, ids, [int(n) for n in sizes],
                                [spec] * len(ids), chunksize=8))
    else:
        parts = [_serve_request_packed(i, int(n), spec) for i, n in zip(ids, sizes)]
    req_start = np.zeros(len(ids) + 1, dtype=np.int64)
    np.cumsum(sizes, out=req_start[1:])
    lens = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.uint8)
    offsets = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    buf = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.uint8)
    return ServeWorkload(Batch(buf, offsets, req_start), np.asarray(times, dtype=np.float64))


def random_words(rng: np.random.Generator, n: int, lmin: int, lmax: int,
                 alphabet: Optional[bytes] = None) -> Words:
    """Uniform random words for edge-case tests (any byte values allowed)."""
    lens = rng.integers(lmin, lmax + 1, size=n).astype(np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    total = int(offsets[-1])
    if alphabet is None:
        buf = rng.integers(0, 256, size=total).astype(np.uint8)
    else:
        al = np.frombuffer(alphabet, dtype=np.uint8)
        buf = al[rng.integers(0, len(al), size=total)]
    return Words(buf, offsets)


# Separators written after each word of a raw text, with their weights: the
# paper's examples of special characters (quote, comma, full stop, question
# and exclamation marks) and other punctuation, line breaks, a tab, a digit
# and a UTF-8 right single quote.  None holds a letter, so the words of the
# text are exactly the words it was made from.
TEXT_SEPARATORS = (
    (b" ", 0.760), (b", ", 0.070), (b". ", 0.050), (b"\n", 0.040), (b"; ", 0.012),
    (b": ", 0.008), (b"? ", 0.008), (b"! ", 0.008), (b' "', 0.008), (b'" ', 0.008),
    (b" -- ", 0.006), (b".\n\n", 0.006), (b"\t", 0.004), (b" 1 ", 0.004),
    (b"\xe2\x80\x99 ", 0.004), (b"...", 0.004),
)


def raw_text(words: Words, seed: int = 0) -> np.ndarray:
    """A raw text (uint8) holding `words` in order, each followed by a
    separator drawn from TEXT_SEPARATORS (seeded)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x7E47])))
    seps = [np.frombuffer(s, dtype=np.uint8) for s, _ in TEXT_SEPARATORS]
    w = np.array([p for _, p in TEXT_SEPARATORS], dtype=np.float64)
    n = words.n
    kind = rng.choice(len(seps), size=n, p=w / w.sum())
    sep_len = np.array([len(s) for s in seps], dtype=np.int64)[kind]
    word_len = np.diff(words.offsets)
    piece = word_len + sep_len
    start = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(piece, out=start[1:])
    out = np.empty(int(start[-1]), dtype=np.uint8)
    nl = int(words.offsets[-1] - words.offsets[0])
    if nl:
        src = words.offsets[0] + np.arange(nl, dtype=np.int64)
        dst = np.repeat(start[:-1] - words.offsets[:-1], word_len) + src
        out[dst] = words.bytes[src]
    for k, s in enumerate(seps):
        idx = np.nonzero(kind == k)[0]
        base = start[idx] + word_len[idx]
        for j in range(len(s)):
            out[base + j] = s[j]
    return out
