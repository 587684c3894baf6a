"""Data-structure ablation (Section III approaches one and two): each
sub-array sorted whole by one workgroup with its words as packed keys or
read from the text through the offsets; both against the oracle.

Index work: bit-exact.
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


def layout_sort(bs, w, max_len, layout):
    b, o = bs.to_device(w.bytes, w.offsets)
    counts, starts, order = bs.bucketize(b, o, max_len)
    perm = bs.oets_buckets(b, o, counts, starts, order, max_len, layout)
    return perm.cpu().numpy()


@pytest.mark.parametrize("layout", [0, 1])
@pytest.mark.parametrize("k", [1, 2])
def test_layouts_match_bubble_oracle(bs, k, layout):
    w = wordgen.single(k)
    ml = wordgen.SINGLE[k].lmax
    expect = oracle.bubble_sort(w.bytes, w.offsets, max_len=ml, threads=8)
    assert np.array_equal(layout_sort(bs, w, ml, layout), expect)


@pytest.mark.parametrize("layout", [0, 1])
def test_layouts_edge_words(bs, layout):
    """All byte values, empty words, ties, one-word and empty sub-arrays."""
    rng = np.random.default_rng(9)
    w = wordgen.random_words(rng, 1500, 0, 13, alphabet=b"aAz\x00\x80\xff")
    expect = oracle.definition_sort(w.bytes, w.offsets)
    assert np.array_equal(layout_sort(bs, w, 13, layout), expect)
    w1 = wordgen.Words.from_list([b"b", b"a", b"abc"])
    assert layout_sort(bs, w1, 5, layout).tolist() == [1, 0, 2]


def test_layout_too_large_reports(bs):
    """A sub-array beyond the LDS budget is reported, not sorted."""
    w = wordgen.Words.from_list([b"ab"] * 40_000)
    b, o = bs.to_device(w.bytes, w.offsets)
    counts, starts, order = bs.bucketize(b, o, 2)
    with pytest.raises(bs.BsortError):
        bs.oets_buckets(b, o, counts, starts, order, 2, bs.LAYOUT_PACKED)
