"""The CPU oracle against its pins (no GPU)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import wordgen
from tests import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(oracle_mod, pin):
    msg = pin(oracle_mod)
    assert msg is None, msg


def test_special_cases(oracle_mod):
    o = oracle_mod
    # empty input
    w = wordgen.Words.from_list([])
    assert o.bubble_sort(w.bytes, w.offsets, max_len=0).tolist() == []
    # one word
    w = wordgen.Words.from_list([b"x"])
    assert o.bubble_sort(w.bytes, w.offsets).tolist() == [0]
    # all equal: identity (ties keep input order)
    w = wordgen.Words.from_list([b"same"] * 300)
    assert o.bubble_sort(w.bytes, w.offsets).tolist() == list(range(300))
    # one sub-array, strictly decreasing: full reversal
    wl = [bytes([65 + (i // 26) % 26, 97 + i % 26]) for i in range(400)][::-1]
    w = wordgen.Words.from_list(wl)
    assert o.bubble_sort(w.bytes, w.offsets).tolist() == list(range(399, -1, -1))
    # only empty words
    w = wordgen.Words.from_list([b""] * 5)
    assert o.bubble_sort(w.bytes, w.offsets, max_len=0).tolist() == [0, 1, 2, 3, 4]


def test_early_exit_same_result(oracle_mod):
    w = wordgen.single(2)
    a = oracle_mod.bubble_sort(w.bytes, w.offsets, early_exit=False)
    b = oracle_mod.bubble_sort(w.bytes, w.offsets, early_exit=True)
    assert np.array_equal(a, b)


def test_threads_same_result(oracle_mod):
    w = wordgen.single(2)
    a = oracle_mod.bubble_sort(w.bytes, w.offsets, threads=1)
    b = oracle_mod.bubble_sort(w.bytes, w.offsets, threads=4)
    assert np.array_equal(a, b)


def test_invariants_workload2(oracle_mod):
    """Permutation, strictly increasing (len, bytes, index) along the result,
    and multiplicity: each distinct word appears as often as in the input,
    with its indices ascending."""
    w = wordgen.single(2)
    perm = oracle_mod.bubble_sort(w.bytes, w.offsets)
    n = w.n
    assert np.array_equal(np.bincount(perm, minlength=n), np.ones(n, np.int64))
    wl = w.as_list()
    for a, b in zip(perm[:-1], perm[1:]):
        ka, kb = (len(wl[a]), wl[a], a), (len(wl[b]), wl[b], b)
        assert ka < kb
    from collections import defaultdict
    seen = defaultdict(list)
    for i in perm:
        seen[wl[i]].append(int(i))
    for word, idxs in seen.items():
        assert idxs == sorted(idxs)
    assert sum(len(v) for v in seen.values()) == n


def test_errors(oracle_mod):
    w = wordgen.Words.from_list([b"abc", b"toolongword"])
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.bubble_sort(w.bytes, w.offsets, max_len=5)
    bad = wordgen.Words(np.frombuffer(b"abcdef", np.uint8).copy(), np.array([0, 4, 2, 6], np.int64))
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.bubble_sort(bad.bytes, bad.offsets, max_len=8)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.definition_sort(bad.bytes, bad.offsets)
    past_end = wordgen.Words(np.frombuffer(b"abc", np.uint8).copy(), np.array([0, 2, 9], np.int64))
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.bubble_sort(past_end.bytes, past_end.offsets, max_len=10)


def test_bubble_equals_definition_workload3_sample(oracle_mod):
    """Workload 3's words, first 40,000 (bubble sort of all 250,000 takes
    ~30 s on one core; the full size runs in the GPU parity tests)."""
    w = wordgen.single(3)
    k = 40_000
    sub = wordgen.Words(w.bytes[:w.offsets[k]], w.offsets[:k + 1])
    a = oracle_mod.bubble_sort(sub.bytes, sub.offsets, threads=8)
    b = oracle_mod.definition_sort(sub.bytes, sub.offsets)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Planted mistakes: copies of the C oracle with one plausible bug each must
# fail at least one pin.
# ---------------------------------------------------------------------------

MUTANTS = {
    "swap_on_equal": ("memcmp(s[j].p, s[j + 1].p, (size_t)L) > 0",
                      "memcmp(s[j].p, s[j + 1].p, (size_t)L) >= 0"),
    "drop_last_byte": ("memcmp(s[j].p, s[j + 1].p, (size_t)L) > 0",
                       "memcmp(s[j].p, s[j + 1].p, (size_t)(L > 0 ? L - 1 : 0)) > 0"),
    "short_inner_loop": ("for (int32_t j = 0; j + 1 < m - pass; ++j)",
                         "for (int32_t j = 0; j + 2 < m - pass; ++j)"),
    "signed_bytes": ("memcmp(s[j].p, s[j + 1].p, (size_t)L) > 0",
                     "(int)(signed char)s[j].p[0] - (int)(signed char)s[j + 1].p[0] > 0 || "
                     "(s[j].p[0] == s[j + 1].p[0] && memcmp(s[j].p, s[j + 1].p, (size_t)L) > 0)"),
    "little_endian_pack": ("v |= byte << (56 - 8 * k);", "v |= byte << (8 * k);"),
    "sign_extend_pack": ("uint64_t byte = pos < L ? (uint64_t)p[pos] : 0u;",
                         "uint64_t byte = pos < L ? (uint64_t)(int64_t)(int8_t)p[pos] : 0u;"),
    "starts_off_by_one": ("starts[L + 1] = starts[L] + counts[L];",
                          "starts[L + 1] = starts[L] + counts[L] - (L == 3);"),
    "reverse_index_tiebreak": ("return a < b ? -1 : (a > b ? 1 : 0);",
                               "return a > b ? -1 : (a < b ? 1 : 0);"),
    "tokenize_bracket_is_letter": ("return (c >= 'A' && c <= 'Z') || (c >= 'a' && c <= 'z');",
                                   "return (c >= 'A' && c <= '[') || (c >= 'a' && c <= 'z');"),
    "tokenize_high_bytes_letters": ("return (c >= 'A' && c <= 'Z') || (c >= 'a' && c <= 'z');",
                                    "return (c >= 'A' && c <= 'Z') || (c >= 'a' && c <= 'z') "
                                    "|| c >= 0x80;"),
    "tokenize_no_split": ("            in_word = 0;\n", "            ;\n"),
    "whole_prefix_last": ("    return la < lb ? -1 : (la > lb ? 1 : 0);\n}\n\nint oracle_bubble_sort_whole",
                          "    return la < lb ? 1 : (la > lb ? -1 : 0);\n}\n\nint oracle_bubble_sort_whole"),
    "definition_ignores_length": ("if (la != lb) return la < lb ? -1 : 1;",
                                  "if (la != lb) { int q = memcmp(c->bytes + c->offsets[a], "
                                  "c->bytes + c->offsets[b], (size_t)(la < lb ? la : lb)); "
                                  "if (q) return q; return la < lb ? -1 : 1; }"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(oracle_mod, name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle_mod.SRC).read()
    assert old in src, "mutation site not found"
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new, 1))
    so = str(tmp_path / f"libmutant_{name}.so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-o", so, str(mpath)])
    # run in a child process: a mutant may also crash (a crash counts as caught)
    code = ("import json, oracle; from tests import oracle_pins; "
            f"ctx = oracle.using_library({so!r}); ctx.__enter__(); "
            "print(json.dumps(oracle_pins.run_all(oracle)))")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True,
                         text=True, timeout=300)
    if res.returncode == 0:
        failures = json.loads(res.stdout.strip().splitlines()[-1])
        assert failures, f"mutant {name} passed every pin"
