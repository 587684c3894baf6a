"""The C-ABI library without a GPU: header, exported symbols, host-side
argument checks (no compute calls)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsort.h")
LIB = os.path.join(ROOT, "paper_1407_6603_amd", "libbsort.so")


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_1407_6603_amd import build
        build.build()
    return LIB


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(bsort_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_header_is_plain_c(tmp_path):
    c = tmp_path / "t.c"
    c.write_text('#include "bsort.h"\nint main(void){ bsort_words w; (void)w; return 0; }\n')
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only",
                           f"-I{os.path.dirname(HEADER)}", str(c)])


def test_exports_every_declared_symbol(built):
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(\S+)", out))
    declared = declared_functions()
    assert len(declared) >= 12
    missing = [n for n in declared if n not in exported]
    assert not missing, f"declared but not exported: {missing}"


def test_probe_library_exports_its_header():
    hdr = os.path.join(ROOT, "include", "bsort_probe.h")
    lib = os.path.join(ROOT, "paper_1407_6603_amd", "libbsort_probe.so")
    if not os.path.exists(lib):
        from paper_1407_6603_amd import build
        build.build()
    src = re.sub(r"/\*.*?\*/", "", open(hdr).read(), flags=re.S)
    declared = sorted(set(re.findall(r"\b(bsort_[a-z_]+)\s*\(", src)))
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(\S+)", out))
    assert declared and all(n in exported for n in declared)
    from paper_1407_6603_amd import probe
    assert sorted(probe.EXPORTS) == declared
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only",
                    f"-I{os.path.dirname(hdr)}", "-x", "c", "-"], check=True,
                   input=b'#include "bsort_probe.h"\nint main(void){return 0;}\n')


def test_binding_declares_every_symbol():
    from paper_1407_6603_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_functions()


def _run_child(code):
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    return res.stdout


def test_library_loads_and_host_checks(built):
    """Load through the binding (torch first) and call only host-side paths:
    sizes, strings and argument validation that returns before any launch."""
    out = _run_child(r'''
import ctypes
from paper_1407_6603_amd import _lib
L = _lib.load()
print("version", L.bsort_version().decode())
print("ws", L.bsort_workspace_bytes(1000, 12, 1), L.bsort_workspace_bytes(0, 0, 1),
      L.bsort_workspace_bytes(-1, 12, 1), L.bsort_workspace_bytes(10, 65, 1))
for s in range(7):
    print("st", s, L.bsort_status_string(s).decode())
# invalid arguments are rejected on the host, before any device work
w = _lib.Words(None, 0, None, 5, 12)             # offsets NULL with n_words > 0
b = _lib.Buckets(None, None, None)
print("rc1", L.bsort_bucketize(ctypes.byref(w), ctypes.byref(b), None, 0, None))
w = _lib.Words(None, 0, None, 0, 99)             # max_len too long
print("rc2", L.bsort_bucketize(ctypes.byref(w), ctypes.byref(b), None, 0, None))
w = _lib.Words(None, 0, None, 0, 12)
b = _lib.Buckets(8, 8, None)                     # tiny fake pointers; ws NULL -> E_WORKSPACE
print("rc3", L.bsort_bucketize(ctypes.byref(w), ctypes.byref(b), None, 0, None))
t = _lib.Tuning(100, 0, 0)                       # tile_keys not a power of two
print("rc4", L.bsort_sort_buckets(ctypes.byref(w), ctypes.byref(b), None, ctypes.byref(t), None, 0, None))
print("err", L.bsort_last_error().decode())
''')
    lines = dict((l.split(" ", 1)[0] + (l.split(" ")[1] if l.startswith("st") else ""), l)
                 for l in out.splitlines())
    assert "bsort" in lines["version"]
    ws = [int(x) for x in lines["ws"].split()[1:]]
    assert ws[0] > 0 and ws[1] > 0 and ws[2] == 0 and ws[3] == 0
    assert lines["st0"].endswith("ok")
    assert lines["rc1"] == "rc1 1"
    assert lines["rc2"] == "rc2 2"
    assert lines["rc3"] == "rc3 4"
    assert lines["rc4"] == "rc4 1"


def test_workspace_grows_with_size(built):
    out = _run_child(r'''
from paper_1407_6603_amd import _lib
L = _lib.load()
print(L.bsort_workspace_bytes(10**6, 12, 1), L.bsort_workspace_bytes(2 * 10**6, 12, 1),
      L.bsort_workspace_bytes(10**6, 32, 1), L.bsort_workspace_bytes(10**6, 12, 4096))
''')
    a, b, c, d = [int(x) for x in out.split()]
    assert a < b and a < c and a < d
    assert a % 256 == 0


def test_python_api_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import numpy as np
    import paper_1407_6603_amd as bs
    with pytest.raises(RuntimeError):
        bs.sort(torch.zeros(4, dtype=torch.uint8), torch.zeros(2, dtype=torch.int64), 4)
    with pytest.raises(RuntimeError):
        bs.sort_batch(torch.zeros(4, dtype=torch.uint8), torch.zeros(2, dtype=torch.int64),
                      torch.zeros(2, dtype=torch.int64), np.array([0, 1]), 4)


def test_stage_names(built):
    """Stage names are host-side: one tile stage per record width, one stage
    per in-LDS size class that fits 144 KiB, in launch order."""
    out = _run_child(r'''
from paper_1407_6603_amd import api
for ml in (0, 4, 12, 20, 64, 65):
    print(ml, " ".join(api.stage_names(ml)) if ml <= 64 else "-")
''')
    got = {int(l.split()[0]): l.split()[1:] for l in out.splitlines()}
    assert got[0] == ["bucketize", "pack", "merge_split"]
    assert got[4] == ["bucketize", "pack", "tiles_d2", "lds_d2_1024", "lds_d2_2048",
                      "lds_d2_4096", "lds_d2_8192", "lds_d2_16320", "merge_split"]
    lds12 = [n for n in got[12] if n.startswith("lds_")]
    assert lds12 == ["lds_d2_1024", "lds_d2_2048", "lds_d2_4096", "lds_d2_8192", "lds_d2_16320",
                     "lds_d3_1024", "lds_d3_2048", "lds_d3_4096", "lds_d3_8192", "lds_d3_12288",
                     "lds_d4_1024", "lds_d4_2048", "lds_d4_4096", "lds_d4_8192", "lds_d4_9216"]
    assert [n for n in got[20] if n.startswith("lds_d5")] == \
        ["lds_d5_1024", "lds_d5_2048", "lds_d5_4096", "lds_d5_7168"]
    assert [n for n in got[64] if n.startswith("tiles_")] == [f"tiles_d{d}" for d in range(2, 18)]
