import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on CPU")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build(force=False)
    return oracle


def load_golden(name):
    """Parse a tests/golden/*.txt hand-worked fixture."""
    path = os.path.join(ROOT, "tests", "golden", name)
    words = {}
    perm = counts = None
    with open(path) as f:
        for line in f:
            line = line.rstrip("\n")
            if not line or line.startswith("#"):
                continue
            parts = line.split(" ")
            if parts[0] == "w":
                hexs = parts[2] if len(parts) > 2 else ""
                words[int(parts[1])] = bytes.fromhex(hexs)
            elif parts[0] == "perm":
                perm = [int(x) for x in parts[1:]]
            elif parts[0] == "counts":
                counts = [int(x) for x in parts[1:]]
    wl = [words[i] for i in range(len(words))]
    return wl, perm, counts
