"""Unbucketed ablation (Table 1 rows 2-3): fixed-width keys and the whole-list
sorts they give, against the CPU oracle's whole-list bubble sorts.

Byte and index work: bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import wordgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6603_amd as m
    return m


@pytest.fixture(scope="module")
def ws(bs):
    return bs.Workspace(device="cuda")


def expected_keys(w, width, mode):
    """The fixed-width keys written out on the host (numpy)."""
    n = w.n
    out = np.zeros((n, width), dtype=np.uint8)
    lens = np.diff(w.offsets)
    lead = 0 if mode == 0 else 1
    for i in range(n):
        a = int(w.offsets[i])
        if mode == 1:
            out[i, 0] = lens[i]
            continue
        if lead:
            out[i, 0] = lens[i]
        out[i, lead:lead + lens[i]] = w.bytes[a:a + lens[i]]
    return out.reshape(-1)


@pytest.mark.parametrize("mode,extra", [(0, 0), (1, None), (2, 1)])
def test_fixed_width_bytes(bs, mode, extra):
    rng = np.random.default_rng(mode)
    w = wordgen.random_words(rng, 3001, 0, 9)             # all byte values, empty words
    width = 1 if extra is None else 9 + extra
    b, o = bs.to_device(w.bytes, w.offsets)
    kb, ko = bs.fixed_width(b, o, width, mode)
    assert np.array_equal(kb.cpu().numpy(), expected_keys(w, width, mode))
    assert np.array_equal(ko.cpu().numpy(), np.arange(w.n + 1, dtype=np.int64) * width)


def test_fixed_width_rejects_long_words(bs):
    w = wordgen.Words.from_list([b"abc", b"toolongword", b"x"])
    b, o = bs.to_device(w.bytes, w.offsets)
    with pytest.raises(bs.BsortError):
        bs.fixed_width(b, o, 5, bs.KEY_BYTES)
    with pytest.raises(bs.BsortError):
        bs.fixed_width(b, o, 11, bs.KEY_LENGTH_BYTES)       # needs 12 with the length byte
    kb, _ = bs.fixed_width(b, o, 12, bs.KEY_LENGTH_BYTES)
    assert kb.numel() == 36


def unbucketed(bs, ws, w, mode):
    width = {0: int(np.diff(w.offsets).max()), 1: 1, 2: int(np.diff(w.offsets).max()) + 1}[mode]
    b, o = bs.to_device(w.bytes, w.offsets)
    kb, ko = bs.fixed_width(b, o, width, mode)
    rs = torch.tensor([0, w.n], dtype=torch.int64, device="cuda")
    perm = bs.sort_batch(kb, ko, rs, np.array([0, w.n], np.int64), width, ws=ws)
    bs.check_device_status(ws)
    return perm.cpu().numpy()


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_unbucketed_sort_matches_whole_bubble(bs, ws, k, mode):
    """The whole list as one sub-array, sorted by OETS and merge-split,
    equals one bubble sort of the whole list by the same key (the 35,000-word
    list crosses the in-LDS limit and merges through HBM)."""
    w = wordgen.single(k)
    expect, _ = oracle.bubble_sort_whole(w.bytes, w.offsets, mode)
    assert np.array_equal(unbucketed(bs, ws, w, mode), expect)


def test_unbucketed_length_bytes_equals_bucketed(bs, ws):
    """Length then bytes as one sub-array per list reaches the bucketed
    order, on a batch of lists."""
    batch = wordgen.batch(first=0, count=64, workers=1)
    b, o = bs.to_device(batch.bytes, batch.offsets)
    rs = torch.from_numpy(batch.req_start).cuda()
    bucketed = bs.sort_batch(b, o, rs, batch.req_start, 12, ws=ws).cpu().numpy()
    kb, ko = bs.fixed_width(b, o, 13, bs.KEY_LENGTH_BYTES)
    whole = bs.sort_batch(kb, ko, rs, batch.req_start, 13, ws=ws).cpu().numpy()
    bs.check_device_status(ws)
    assert np.array_equal(whole, bucketed)
    expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
    assert np.array_equal(whole, expect)
