"""bsort_sort_batch_static, the entry point that allocates nothing, against
bsort_sort_batch (the workspace entry point) through the C ABI: two calls
in a row, the second on a smaller batch, each bit-exact with the workspace
call and with a clean device status; a list whose sub-arrays merge through
HBM; and a batch too large for the static scratch, refused before any
launch."""
import ctypes

import numpy as np
import pytest
import torch

import wordgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6603_amd as m
    return m


def _both(bs, batch, max_len):
    b, o = bs.to_device(batch.bytes, batch.offsets)
    rs = torch.from_numpy(batch.req_start).cuda()
    ref = bs.sort_batch(b, o, rs, batch.req_start, max_len, ws=bs.Workspace())
    out = torch.full((batch.total,), -1, dtype=torch.int32, device="cuda")
    status = torch.full((1,), 0xFFFF, dtype=torch.int32, device="cuda")
    bs.sort_batch_static(b, o, rs, batch.req_start, max_len, out, status=status)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy(), int(status.cpu()[0])


def test_static_entry_equals_workspace_entry(bs):
    big = wordgen.batch(first=0, count=160)
    small = wordgen.batch(first=3000, count=23)
    assert bs.workspace_bytes(big.total, 12, big.R) <= bs.STATIC_SCRATCH_BYTES
    assert small.total < big.total
    for batch in (big, small):
        ref, got, st = _both(bs, batch, 12)
        assert st == 0
        assert np.array_equal(got, ref)


def test_static_entry_merges_through_hbm(bs):
    w = wordgen.serve_request(3, 1_000_000)
    second = wordgen.Batch.concat([wordgen.serve_request(11, 200_000),
                                   wordgen.serve_request(12, 7_000)])
    for batch in (wordgen.Batch.concat([w]), second):
        ref, got, st = _both(bs, batch, 32)
        assert st == 0
        assert np.array_equal(got, ref)


def test_static_entry_refuses_a_batch_too_large(bs):
    batch = wordgen.batch(first=0, count=600)
    assert bs.workspace_bytes(batch.total, 12, batch.R) > bs.STATIC_SCRATCH_BYTES
    b, o = bs.to_device(batch.bytes, batch.offsets)
    rs = torch.from_numpy(batch.req_start).cuda()
    out = torch.empty(batch.total, dtype=torch.int32, device="cuda")
    with pytest.raises(bs.BsortError, match="static scratch"):
        bs.sort_batch_static(b, o, rs, batch.req_start, 12, out)
