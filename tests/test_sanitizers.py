"""CPU sanitizer runs.

* The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
  runs every oracle pin (tests/oracle_pins.py) in a child process; a memory
  error or undefined behaviour aborts it.
* The C oracle built with ThreadSanitizer is called from four Python threads
  at once (ctypes releases the interpreter lock, so the calls overlap in C);
  a data race between calls aborts the child.
* Four serving loops (serve.Server with the host executor and a virtual
  clock) run in four threads at once over their own requests; every result
  equals the oracle's, so the scheduler keeps no state shared between
  servers.
A planted heap overflow and a planted race show that the sanitizer runs
catch what they are for."""
import os
import subprocess
import sys
import threading

import numpy as np
import pytest

import oracle
import wordgen
from paper_1407_6603_amd import serve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    if p.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


def _build(tmp_path, flags, src_text=None, name="liboracle_san.so"):
    src = oracle.SRC
    if src_text is not None:
        src = str(tmp_path / "oracle_src.c")
        with open(src, "w") as f:
            f.write(src_text)
    so = str(tmp_path / name)
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                           "-fno-omit-frame-pointer", *flags, "-o", so, src])
    return so


def _child(code, preload, env_extra):
    env = dict(os.environ, LD_PRELOAD=preload, PYTHONPATH=ROOT, **env_extra)
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                          text=True, timeout=600)


PINS = ("import json, oracle; from tests import oracle_pins\n"
        "with oracle.using_library({so!r}):\n"
        "    print(json.dumps(oracle_pins.run_all(oracle)))\n")


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    so = _build(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
    r = _child(PINS.format(so=so), asan, {"ASAN_OPTIONS": "detect_leaks=0"})
    assert r.returncode == 0, r.stderr[-3000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.stdout.strip().splitlines()[-1] == "{}"


def test_asan_catches_a_planted_overflow(tmp_path):
    asan = _runtime("libasan.so")
    src = open(oracle.SRC).read()
    old = "calloc((size_t)max_len + 1, sizeof(int32_t))"
    assert old in src
    so = _build(tmp_path, ["-fsanitize=address", "-fno-sanitize-recover=all"],
                src.replace(old, "calloc((size_t)max_len, sizeof(int32_t))", 1))
    r = _child(PINS.format(so=so), asan, {"ASAN_OPTIONS": "detect_leaks=0"})
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr


THREADS = """
import threading, numpy as np, oracle, wordgen
ws = [wordgen.single(1), wordgen.batch(first=5, count=3).request(0),
      wordgen.batch(first=9, count=3).request(2), wordgen.single(1)]
expect = [oracle.definition_sort(w.bytes, w.offsets) for w in ws]
ok = []
def work(i):
    w = ws[i]
    for _ in range(3):
        a = oracle.bubble_sort(w.bytes, w.offsets, threads=1)
        b = oracle.definition_sort(w.bytes, w.offsets)
        c, s, o = oracle.bucketize(w.bytes, w.offsets)
        ok.append(np.array_equal(a, expect[i]) and np.array_equal(b, expect[i]))
with oracle.using_library({so!r}):
    ts = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    [t.start() for t in ts]
    [t.join() for t in ts]
print("ok" if len(ok) == 12 and all(ok) else "bad")
"""


def test_oracle_concurrent_calls_under_tsan(tmp_path):
    tsan = _runtime("libtsan.so")
    so = _build(tmp_path, ["-fsanitize=thread"])
    r = _child(THREADS.format(so=so), tsan, {"TSAN_OPTIONS": "halt_on_error=1"})
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ThreadSanitizer" not in r.stderr
    assert r.stdout.strip().splitlines()[-1] == "ok"


def test_tsan_catches_a_planted_race(tmp_path):
    tsan = _runtime("libtsan.so")
    src = open(oracle.SRC).read()
    old = "    if (n < 0) return ORACLE_E_INVALID;\n    for (int32_t i = 0; i < n; ++i)\n"
    assert old in src
    racy = src.replace(old, "    static int32_t calls; calls += 1;\n" + old, 1)
    so = _build(tmp_path, ["-fsanitize=thread"], racy)
    r = _child(THREADS.format(so=so), tsan, {"TSAN_OPTIONS": "halt_on_error=1"})
    assert r.returncode != 0 and "data race" in r.stderr


def test_servers_in_threads():
    rng = np.random.default_rng(21)
    vocab = wordgen.make_vocab(rng, 300, 12, 1.1)
    jobs = []
    for k in range(4):
        sizes = rng.integers(5, 900, 12)
        lists = [wordgen.draw_tokens(rng, vocab, int(n)) for n in sizes]
        staging, spans = serve.build_staging(lists, 12)
        arrivals = np.cumsum(rng.exponential(0.001, len(sizes)))
        reqs = [serve.Request(i, float(t), a, b, nb)
                for i, (t, (a, b, nb)) in enumerate(zip(arrivals, spans))]
        jobs.append((staging, reqs, lists))
    out = [None] * 4

    def run(k):
        staging, reqs, _ = jobs[k]
        clock = serve.VirtualClock()
        ex = serve.HostExecutor(staging, lambda b, o: oracle.bubble_sort(b, o, max_len=12),
                                clock, slots=2)
        out[k] = serve.Server(ex, pool_bytes=200_000, clock=clock).run(
            reqs, cancels=[(float(reqs[3].arrival), 3)])

    ts = [threading.Thread(target=run, args=(k,)) for k in range(4)]
    [t.start() for t in ts]
    [t.join() for t in ts]
    for k in range(4):
        for r, w in zip(out[k], jobs[k][2]):
            if r.cancelled or r.refused:
                continue
            assert np.array_equal(r.perm, oracle.definition_sort(w.bytes, w.offsets))
