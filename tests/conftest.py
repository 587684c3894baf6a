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


def load_golden_text(name):
    """The "text <hex>" line of a tests/golden/*.txt fixture (raw text)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    with open(path) as f:
        for line in f:
            if line.startswith("text "):
                return bytes.fromhex(line.split(" ", 1)[1].strip())
    raise ValueError(f"{name} has no text line")


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
