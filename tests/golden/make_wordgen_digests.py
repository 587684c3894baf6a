"""Writes tests/golden/wordgen_digests.txt: sha256 digests that freeze the
seeded input generator's output (word bytes and offsets) for the three
single-list workloads, the first 64 lists of the batch workload, and the
first 20 requests and the arrival schedule of the serving workload.  Calls
only wordgen.  Run from the repository root:
    python tests/golden/make_wordgen_digests.py
"""
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import wordgen  # noqa: E402


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def entries():
    for k in (1, 2, 3):
        w = wordgen.single(k)
        yield f"single{k}", digest(w.bytes, w.offsets)
    b = wordgen.batch(first=0, count=64)
    yield "batch_first64", digest(b.bytes, b.offsets, b.req_start)
    times, sizes = wordgen.serve_arrivals()
    yield "serve_arrivals", digest(times, sizes)
    for i in range(20):
        w = wordgen.serve_request(i, int(sizes[i]))
        yield f"serve_request{i}", digest(w.bytes, w.offsets)


if __name__ == "__main__":
    with open(os.path.join(HERE, "wordgen_digests.txt"), "w") as f:
        f.write("# name sha256 -- written by tests/golden/make_wordgen_digests.py\n")
        for name, d in entries():
            f.write(f"{name} {d}\n")
