"""The seeded input generator (wordgen), pinned on the CPU.

Digests freeze its output (tests/golden/wordgen_digests.txt, written by
tests/golden/make_wordgen_digests.py): the three single-list workloads, the
first 64 batch lists, the serving arrival schedule and its first 20
requests.  Statistical checks tie the output to the shape it stands in for:
the English-like length pmf (mode at 3 letters), 5% capitalised tokens,
Zipf rank-frequency slope -s, Poisson arrivals at 2,000/s, and log-uniform
list and request sizes."""
import collections
import os

import numpy as np
import pytest

import wordgen
from tests.golden.make_wordgen_digests import digest, entries

HERE = os.path.dirname(os.path.abspath(__file__))


def frozen():
    out = {}
    with open(os.path.join(HERE, "golden", "wordgen_digests.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, d = line.split()
                out[name] = d
    return out


def test_digests_unchanged():
    want = frozen()
    got = dict(entries())
    assert set(got) == set(want)
    for name in want:
        assert got[name] == want[name], f"{name} changed"


def test_digest_sees_a_one_byte_change():
    w = wordgen.single(1)
    b = w.bytes.copy()
    b[17] ^= 1
    assert digest(b, w.offsets) != digest(w.bytes, w.offsets)


@pytest.mark.parametrize("k,tv_max", [(1, 0.06), (2, 0.04), (3, 0.04)])
def test_length_histogram_follows_pmf(k, tv_max):
    w = wordgen.single(k)
    sp = wordgen.SINGLE[k]
    L = np.diff(w.offsets)
    assert L.min() >= 1 and L.max() <= sp.lmax
    h = np.bincount(L, minlength=sp.lmax + 1)[1:] / len(L)
    pmf = wordgen.length_pmf(sp.lmax)
    assert int(np.argmax(pmf)) + 1 == 3 and int(np.argmax(h)) + 1 == 3
    assert 0.5 * np.abs(h - pmf).sum() < tv_max


def test_length_pmf_closed_form():
    p = wordgen.length_pmf(12)
    w = np.array([0.03, 0.16, 0.21, 0.18] + [0.18 * 0.72 ** (L - 4) for L in range(5, 13)])
    assert np.allclose(p, w / w.sum())
    assert abs(float((np.arange(1, 13) * p).sum()) - 4.64) < 0.01


@pytest.mark.parametrize("k", [1, 2, 3])
def test_capitalised_fraction(k):
    w = wordgen.single(k)
    first = w.bytes[w.offsets[:-1]]
    frac = float(np.mean((first >= ord("A")) & (first <= ord("Z"))))
    se = (0.05 * 0.95 / w.n) ** 0.5
    assert abs(frac - wordgen.CAPITAL_P) < 4 * se
    # letters only, and only the first letter may be a capital
    assert np.all(((w.bytes >= 65) & (w.bytes <= 90)) | ((w.bytes >= 97) & (w.bytes <= 122)))
    rest = np.ones(len(w.bytes), bool)
    rest[w.offsets[:-1]] = False
    assert not np.any((w.bytes[rest] >= 65) & (w.bytes[rest] <= 90))


@pytest.mark.parametrize("k", [2, 3])
def test_zipf_rank_frequency_slope(k):
    w = wordgen.single(k)
    counts = collections.Counter(x.lower() for x in w.as_list())
    c = np.array(sorted(counts.values(), reverse=True), dtype=np.float64)[:200]
    slope = np.polyfit(np.log(np.arange(1, len(c) + 1)), np.log(c), 1)[0]
    assert abs(slope + wordgen.SINGLE[k].zipf_s) < 0.1


def test_serve_arrivals_poisson_and_log_uniform():
    spec = wordgen.ServeSpec()
    t, s = wordgen.serve_arrivals(spec)
    assert len(t) == spec.n_arrivals + 1 and s[spec.big_at] == spec.big_n
    t0, s0 = np.delete(t, spec.big_at), np.delete(s, spec.big_at)
    gaps = np.diff(t0)
    assert np.all(gaps >= 0)
    assert abs(gaps.mean() * spec.rate_per_s - 1) < 0.05            # mean gap 0.5 ms
    assert abs(gaps.std() / gaps.mean() - 1) < 0.1                   # exponential: cv 1
    assert s0.min() >= spec.nmin and s0.max() < spec.nmax
    u = np.log(s0 / spec.nmin) / np.log(spec.nmax / spec.nmin)       # uniform on [0, 1)
    assert abs(u.mean() - 0.5) < 0.02 and abs(u.var() - 1 / 12) < 0.01


def test_batch_sizes_log_uniform():
    n = wordgen.batch_sizes()
    assert len(n) == wordgen.BATCH_R
    assert n.min() >= wordgen.BATCH_NMIN and n.max() < wordgen.BATCH_NMAX
    u = np.log2(n / wordgen.BATCH_NMIN) / np.log2(wordgen.BATCH_NMAX / wordgen.BATCH_NMIN)
    assert abs(u.mean() - 0.5) < 0.02 and abs(u.var() - 1 / 12) < 0.01
    assert int(n.sum()) == 31_795_051
