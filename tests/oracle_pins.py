"""Pins of the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.

Each check returns None when it holds and a short message when it fails, so
the same list can be run against the real oracle (every check must hold) and
against copies of the oracle with a planted mistake (some check must fail).
"""
import itertools

import numpy as np

import wordgen
from tests.conftest import load_golden, load_golden_text


def _words(wl):
    return wordgen.Words.from_list(wl)


def pin_golden(oracle):
    """Hand-worked fixtures (tests/golden)."""
    for name in ("hand_sentence.txt", "hand_bytes.txt"):
        wl, perm, counts = load_golden(name)
        w = _words(wl)
        got, c, s, o, _ = oracle.bubble_sort(w.bytes, w.offsets, with_buckets=True)
        if got.tolist() != perm:
            return f"{name}: bubble perm {got.tolist()} != {perm}"
        if c.tolist() != counts:
            return f"{name}: counts {c.tolist()} != {counts}"
        if oracle.definition_sort(w.bytes, w.offsets).tolist() != perm:
            return f"{name}: definition perm differs"
    return None


BRUTE_SET = [b"", b"a", b"b", b"A", b"ab", b"ba", b"Ab", b"\x80", b"\xff\x00"]


def pin_brute_force(oracle, n_max=4, random_n=(5, 6), random_cases=60):
    """Every sequence of n <= n_max words over a small word set, plus random
    sequences of 5-6 words: the oracle equals the permutation found by trying
    all n! orders."""
    cases = []
    small = BRUTE_SET[:6]
    for n in range(0, n_max + 1):
        cases.extend(itertools.product(small, repeat=n))
    rng = np.random.default_rng(123)
    for n in random_n:
        for _ in range(random_cases):
            cases.append(tuple(BRUTE_SET[i] for i in rng.integers(0, len(BRUTE_SET), n)))
    for wl in cases:
        wl = list(wl)
        w = _words(wl)
        expect = oracle.brute_force(wl)
        ml = max([len(x) for x in wl], default=0)
        got = oracle.bubble_sort(w.bytes, w.offsets, max_len=ml).tolist()
        if got != expect:
            return f"brute force {wl}: {got} != {expect}"
        if oracle.definition_sort(w.bytes, w.offsets).tolist() != expect:
            return f"brute force (definition) {wl}"
    return None


def pin_library_sort(oracle):
    """Python's sort is stable and compares bytes unsigned, so sorting indices
    by (len, bytes) is the definition; checked on random words over all 256
    byte values and on the small English-like workload."""
    rng = np.random.default_rng(7)
    for w in (wordgen.random_words(rng, 3000, 0, 11),
              wordgen.random_words(rng, 3000, 1, 4, alphabet=b"aAbB\x80\xff"),
              wordgen.single(1)):
        wl = w.as_list()
        expect = sorted(range(len(wl)), key=lambda i: (len(wl[i]), wl[i]))
        if oracle.bubble_sort(w.bytes, w.offsets).tolist() != expect:
            return "bubble differs from library sort"
        if oracle.definition_sort(w.bytes, w.offsets).tolist() != expect:
            return "definition differs from library sort"
    return None


def pin_bucketize_closed_form(oracle):
    """counts = histogram of lengths, starts = its exclusive running sum,
    order = the stable arrangement of indices by length (a stable sort keyed
    on length alone)."""
    rng = np.random.default_rng(11)
    for w in (wordgen.random_words(rng, 5000, 0, 17), wordgen.single(2)):
        L = np.diff(w.offsets)
        ml = int(L.max())
        c, s, o = oracle.bucketize(w.bytes, w.offsets, ml)
        if not np.array_equal(c, np.bincount(L, minlength=ml + 1)):
            return "counts != bincount"
        if not np.array_equal(s, np.concatenate([[0], np.cumsum(np.bincount(L, minlength=ml + 1))])):
            return "starts != cumsum"
        if not np.array_equal(o, np.argsort(L, kind="stable")):
            return "order != stable argsort of lengths"
    return None


def pin_comparison_count(oracle):
    """Without early exit, bubble sort of a sub-array of m words makes
    m(m-1)/2 comparisons (the count the paper states)."""
    rng = np.random.default_rng(5)
    for w in (wordgen.single(1), wordgen.random_words(rng, 2000, 1, 6, alphabet=b"ab")):
        _, c, _, _, cmp = oracle.bubble_sort(w.bytes, w.offsets, with_buckets=True)
        c = c.astype(np.int64)
        if cmp != int((c * (c - 1) // 2).sum()):
            return f"comparisons {cmp} != sum m(m-1)/2 = {int((c * (c - 1) // 2).sum())}"
    return None


def pin_pack_closed_form(oracle):
    """Big-endian lanes: every 1- and 2-byte word packs to b0<<56 (| b1<<48);
    random words up to 64 bytes equal int.from_bytes of the zero-padded word,
    cut into 8-byte groups."""
    allb = np.arange(256, dtype=np.uint8)
    w1 = wordgen.Words(allb.copy(), np.arange(257, dtype=np.int64))
    lanes = oracle.pack_keys(w1.bytes, w1.offsets, np.arange(256, dtype=np.int32), 1)
    if not np.array_equal(lanes[0], allb.astype(np.uint64) << np.uint64(56)):
        return "1-byte lanes"
    b0, b1 = np.meshgrid(allb, allb, indexing="ij")
    buf = np.stack([b0.ravel(), b1.ravel()], axis=1).ravel().astype(np.uint8)
    w2 = wordgen.Words(buf, np.arange(0, 2 * 65536 + 1, 2, dtype=np.int64))
    lanes = oracle.pack_keys(w2.bytes, w2.offsets, np.arange(65536, dtype=np.int32), 2)
    expect = (b0.ravel().astype(np.uint64) << np.uint64(56)) | (b1.ravel().astype(np.uint64) << np.uint64(48))
    if not np.array_equal(lanes[0], expect):
        return "2-byte lanes"
    rng = np.random.default_rng(3)
    for L in (3, 7, 8, 9, 15, 16, 17, 31, 33, 64):
        w = wordgen.random_words(rng, 50, L, L)
        lanes = oracle.pack_keys(w.bytes, w.offsets, np.arange(50, dtype=np.int32), L)
        W = (L + 7) // 8
        for j, word in enumerate(w.as_list()):
            v = int.from_bytes(word + b"\x00" * (8 * W - L), "big")
            for k in range(W):
                if int(lanes[k, j]) != (v >> (64 * (W - 1 - k))) & (2 ** 64 - 1):
                    return f"lane {k} of a {L}-byte word"
    return None


def pin_batch_matches_single(oracle):
    """Sorting lists back to back gives each list its own result."""
    b = wordgen.batch(R=64, first=0, count=24, workers=1)
    perm, cmp = oracle.bubble_sort_batch(b.bytes, b.offsets, b.req_start, 12)
    total_cmp = 0
    for r in range(b.R):
        w = b.request(r)
        p, c, _, _, cr = oracle.bubble_sort(w.bytes, w.offsets, max_len=12, with_buckets=True)
        total_cmp += cr
        if not np.array_equal(perm[b.req_start[r]:b.req_start[r + 1]], p):
            return f"batch list {r} differs"
    if cmp != total_cmp:
        return "batch comparison total"
    if not np.array_equal(oracle.definition_sort_batch(b.bytes, b.offsets, b.req_start, 4), perm):
        return "definition batch differs from bubble batch"
    return None


def pin_tokenize(oracle):
    """Pre-processing (Section II phase 1), a word being a maximal run of
    ASCII letters: the hand-worked text gives its sixteen words, and then
    phases 2-3 give its hand-worked order; random byte strings over all 256
    values split as the regular expression [A-Za-z]+ splits them (a library
    routine for the same definition); a seeded raw text made by joining
    words with separators gives back exactly those words."""
    import re
    text = load_golden_text("hand_text.txt")
    wl, perm, counts = load_golden("hand_text.txt")
    b, o = oracle.tokenize(text)
    got = [bytes(b[o[i]:o[i + 1]]) for i in range(len(o) - 1)]
    if got != wl:
        return f"hand_text.txt: words {got} != {wl}"
    if oracle.bubble_sort(b, o).tolist() != perm:
        return "hand_text.txt: phases 1-3 order differs"
    rng = np.random.default_rng(17)
    cases = [b"", b"a", b"-", b"a-", b"-a", b"ab cd", b"@[`{", b"AZaz", b"\x80A\xffz"]
    for n in (1, 2, 3, 7, 64, 300, 5000):
        for _ in range(6):
            cases.append(rng.integers(0, 256, size=n).astype(np.uint8).tobytes())
            cases.append(rng.choice(np.frombuffer(b"aZ@[`{ .,", np.uint8), size=n).tobytes())
    for t in cases:
        expect = re.findall(rb"[A-Za-z]+", t)
        b, o = oracle.tokenize(t)
        got = [bytes(b[o[i]:o[i + 1]]) for i in range(len(o) - 1)]
        if got != expect:
            return f"tokenize {t[:40]!r}: {got[:5]} != {expect[:5]}"
    w = wordgen.single(1)
    b, o = oracle.tokenize(wordgen.raw_text(w, 1))
    if not (np.array_equal(b, w.bytes) and np.array_equal(o, w.offsets)):
        return "raw text round trip differs"
    return None


def pin_whole_sorts(oracle):
    """Whole-list bubble sorts (Table 1 rows 2-3): alphabetic order equals
    Python's stable sort on the words (bytes compare unsigned, a prefix
    first); length order equals numpy's stable argsort of the lengths;
    length-then-bytes equals the definition; n(n-1)/2 comparisons."""
    rng = np.random.default_rng(29)
    cases = [wordgen.random_words(rng, n, 0, 6, alphabet=b"abAB\x00\xff") for n in (0, 1, 2, 7, 60)]
    cases += [wordgen.random_words(rng, 300, 1, 9), wordgen.single(1)]
    for w in cases:
        wl = w.as_list()
        n = len(wl)
        a, ca = oracle.bubble_sort_whole(w.bytes, w.offsets, oracle.WHOLE_ALPHABETIC)
        if a.tolist() != sorted(range(n), key=lambda i: wl[i]):
            return f"alphabetic whole sort differs (n={n})"
        l, cl = oracle.bubble_sort_whole(w.bytes, w.offsets, oracle.WHOLE_LENGTH)
        if l.tolist() != np.argsort(np.diff(w.offsets), kind="stable").tolist():
            return f"length whole sort differs (n={n})"
        lb, _ = oracle.bubble_sort_whole(w.bytes, w.offsets, oracle.WHOLE_LENGTH_BYTES)
        if lb.tolist() != oracle.definition_sort(w.bytes, w.offsets).tolist():
            return f"length-then-bytes whole sort differs (n={n})"
        if ca != n * (n - 1) // 2 or cl != ca:
            return f"comparisons {ca} != {n * (n - 1) // 2}"
    return None


ALL_PINS = [pin_golden, pin_brute_force, pin_library_sort, pin_bucketize_closed_form,
            pin_comparison_count, pin_pack_closed_form, pin_batch_matches_single, pin_tokenize,
            pin_whole_sorts]


def run_all(oracle):
    failures = {}
    for p in ALL_PINS:
        try:
            msg = p(oracle)
        except Exception as e:  # a crash in a mutant counts as a failed pin
            msg = f"raised {type(e).__name__}: {e}"
        if msg is not None:
            failures[p.__name__] = msg
    return failures
