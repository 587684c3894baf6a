"""The compute-unit scaling measurement sorts correctly: a child process of
bench.py limited to 64 CUs by HSA_CU_MASK returns the oracle's order."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle
import wordgen

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cu_limited_child_matches_oracle(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    batch = wordgen.batch(first=0, count=40, workers=1)
    np.save(tmp_path / "bytes.npy", batch.bytes)
    np.save(tmp_path / "offsets.npy", batch.offsets)
    np.save(tmp_path / "req_start.npy", batch.req_start)
    expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
    env = dict(os.environ, HSA_CU_MASK="0:0-63")
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cu-child",
                          "--cu-data", str(tmp_path)], env=env, capture_output=True, text=True,
                         timeout=240, cwd=ROOT)
    assert res.returncode == 0, res.stderr[-2000:]
    row = json.loads(res.stdout.strip().splitlines()[-1])
    assert row["perm_sha"] == hashlib.sha256(expect.astype(np.int32).tobytes()).hexdigest()[:16]
    assert row["ms"] > 0
