"""The serving loop: admission by memory, continuous batching, latency
statistics.  CPU tests use a virtual clock and a host executor whose sort is
the oracle; the GPU test runs the same server over libbsort."""
import numpy as np
import pytest

import oracle
import wordgen
from paper_1407_6603_amd import serve


def make_requests(sizes, arrivals, seed=0, lmax=12):
    rng = np.random.default_rng(seed)
    vocab = wordgen.make_vocab(rng, 400, lmax, 1.1)
    lists = [wordgen.draw_tokens(rng, vocab, int(n)) for n in sizes]
    staging, spans = serve.build_staging(lists, lmax)
    reqs = [serve.Request(i, float(t), a, b, nb) for i, (t, (a, b, nb)) in
            enumerate(zip(arrivals, spans))]
    return staging, reqs, lists


def oracle_sort(bytes_, offsets):
    return oracle.bubble_sort(bytes_, offsets, max_len=12)


def run_virtual(staging, reqs, pool, slots=2, cost=None):
    clock = serve.VirtualClock()
    kw = {} if cost is None else {"cost": cost}
    ex = serve.HostExecutor(staging, oracle_sort, clock, slots=slots, **kw)
    srv = serve.Server(ex, pool_bytes=pool, clock=clock)
    return srv.run(reqs), srv, ex


def test_results_match_oracle_per_request():
    sizes = [50, 300, 7, 1200, 90, 640]
    staging, reqs, lists = make_requests(sizes, [0.0, 0.001, 0.001, 0.002, 0.01, 0.011])
    res, _, _ = run_virtual(staging, reqs, pool=1 << 30)
    for r, w in zip(res, lists):
        assert not r.refused
        assert np.array_equal(r.perm, oracle.bubble_sort(w.bytes, w.offsets, max_len=12))


def test_admission_respects_pool_and_fifo():
    sizes = [400] * 12
    staging, reqs, _ = make_requests(sizes, [0.0] * 12)
    fp = 64 * 400 + int(np.mean([r.n_bytes for r in reqs]))
    pool = int(fp * 2.5)                      # at most two requests resident
    res, srv, ex = run_virtual(staging, reqs, pool=pool)
    assert srv.pool_high <= pool
    assert all(not r.refused for r in res)
    admitted = [r.admitted for r in sorted(res, key=lambda r: r.rid)]
    assert admitted == sorted(admitted)       # arrival order
    # never more than two requests resident at once
    events = sorted([(r.admitted, 1) for r in res] + [(r.done, -1) for r in res],
                    key=lambda e: (e[0], e[1]))
    live = peak = 0
    for _, d in events:
        live += d
        peak = max(peak, live)
    assert peak <= 2


def test_oversized_request_is_refused_others_complete():
    staging, reqs, lists = make_requests([100, 5000, 100], [0.0, 0.0, 0.0])
    res, _, _ = run_virtual(staging, reqs, pool=64 * 1000)
    assert [r.refused for r in res] == [False, True, False]
    assert np.array_equal(res[2].perm, oracle_sort(lists[2].bytes, lists[2].offsets))


def test_arrivals_join_while_a_batch_runs():
    """Continuous batching: a request arriving while a long batch is on the
    device is launched on the second slot before that batch ends."""
    staging, reqs, _ = make_requests([20000, 50, 60], [0.0, 0.0001, 0.0002])
    res, _, ex = run_virtual(staging, reqs, pool=1 << 30, slots=2,
                             cost=lambda w: 1e-3 + 1e-6 * w)
    first, second = ex.log[0], ex.log[1]
    assert first["rids"] == [0]
    assert second["start"] < first["end"]               # overlapped on the device
    assert res[1].done < res[0].done


def test_latency_stats_on_a_fixed_schedule():
    staging, reqs, _ = make_requests([100] * 5, [0.0, 0.01, 0.02, 0.03, 0.04])
    res, _, _ = run_virtual(staging, reqs, pool=1 << 30, slots=1, cost=lambda w: 0.002)
    st = serve.latency_stats(res)
    assert st["requests"] == 5 and st["refused"] == 0
    assert abs(st["p50_ms"] - 2.0) < 1e-6 and abs(st["max_ms"] - 2.0) < 1e-6
    assert st["words"] == 500


def test_deterministic_replay():
    sizes = [30, 700, 12, 3000, 45, 800, 5]
    arrivals = np.cumsum(np.full(7, 0.0004))
    staging, reqs, _ = make_requests(sizes, arrivals)
    a, _, _ = run_virtual(staging, reqs, pool=300_000)
    b, _, _ = run_virtual(staging, reqs, pool=300_000)
    assert [(r.admitted, r.launched, r.done, r.batch) for r in a] == \
           [(r.admitted, r.launched, r.done, r.batch) for r in b]
    for x, y in zip(a, b):
        assert np.array_equal(x.perm, y.perm)


def test_refused_request_in_the_middle_splits_the_batch():
    """Requests 0 and 2 are admitted and 1 (between them in the staging
    arrays) is refused: a batch is one run of the staging arrays, so 0 and 2
    go in separate batches and each gets its own words."""
    staging, reqs, lists = make_requests([100, 5000, 120, 90], [0.0, 0.0, 0.0, 0.0])
    res, _, ex = run_virtual(staging, reqs, pool=64 * 1000)
    assert [r.refused for r in res] == [False, True, False, False]
    for h in ex.log:
        assert 1 not in h["rids"]
        assert not (0 in h["rids"] and 2 in h["rids"])
    for k in (0, 2, 3):
        assert np.array_equal(res[k].perm, oracle_sort(lists[k].bytes, lists[k].offsets))


def test_arrival_order_unlike_staging_order_splits_batches():
    staging, reqs, lists = make_requests([80, 90, 100, 110], [0.003, 0.001, 0.002, 0.0])
    res, _, ex = run_virtual(staging, reqs, pool=1 << 30, slots=1, cost=lambda w: 0.01)
    for h in ex.log:
        a, b = h["words"]
        assert b - a == sum(reqs[r].n for r in h["rids"])
    for r, w in zip(res, lists):
        assert np.array_equal(r.perm, oracle_sort(w.bytes, w.offsets))


def test_ring_arena_blocks_never_overlap():
    rng = np.random.default_rng(3)
    for trial in range(20):
        cap = int(rng.integers(1, 64)) * 4096
        ar = serve.RingArena(cap)
        live = {}
        for step in range(400):
            if live and (rng.random() < 0.45 or len(live) > 12):
                off = list(live)[int(rng.integers(len(live)))]
                ar.free(off)
                del live[off]
            else:
                size = int(rng.integers(1, cap // 3 + 2))
                off = ar.alloc(size)
                if off is None:
                    continue
                sz = serve._up(size)
                assert 0 <= off and off + sz <= ar.capacity and off % serve.ALIGN == 0
                for o, z in live.items():
                    assert off + sz <= o or o + z <= off, "blocks overlap"
                live[off] = sz
            assert ar.used == sum(live.values())
        for off in list(live):
            ar.free(off)
        assert ar.alloc(ar.capacity) == 0          # everything freed: the whole arena fits


def test_footprints_cover_the_batch_layout():
    """A batch's buffers fit in the span its members' footprints hold (the
    library's workspace size is sub-additive over lists)."""
    from paper_1407_6603_amd import _lib
    L = _lib.load()
    wsb = lambda n, ml, R: int(L.bsort_workspace_bytes(n, ml, R))
    rng = np.random.default_rng(9)
    for ml in (1, 12, 32, 64):
        for trial in range(60):
            R = int(rng.integers(1, 40))
            ns = np.floor(10 ** rng.uniform(0, 6.5, R)).astype(np.int64)
            ns[rng.random(R) < 0.1] = 0
            nb = [int(n * rng.uniform(1, 8)) for n in ns]
            fp = sum(serve.request_footprint(int(n), b, ml, wsb) for n, b in zip(ns, nb))
            lay = serve.batch_layout(sum(nb), int(ns.sum()), R, wsb(int(ns.sum()), ml, R))
            assert lay["size"] <= fp


def test_cancel_queued_request_frees_its_place():
    """Pool for two requests: 0 and 1 run, 2 waits for the pool and is
    cancelled; 3 then takes its place and every other result is exact."""
    sizes = [400] * 5
    staging, reqs, lists = make_requests(sizes, [0.0] * 5)
    fp = 64 * 400 + max(r.n_bytes for r in reqs)
    pool = serve._up(fp) * 2 + 512
    clock = serve.VirtualClock()
    ex = serve.HostExecutor(staging, oracle_sort, clock, slots=2, cost=lambda w: 0.01)
    srv = serve.Server(ex, pool_bytes=pool, clock=clock)
    res = srv.run(reqs, cancels=[(0.001, 2), (0.001, 0), (0.5, 4)])
    assert res[2].cancelled and res[2].launched is None and res[2].perm is None
    assert not res[0].cancelled                  # launched at 0: the cancel came too late
    assert not res[4].cancelled                  # done before its cancel
    assert all(2 not in h["rids"] for h in ex.log)
    assert res[3].launched == pytest.approx(0.01)   # admitted when 0 and 1 finished
    for k in (0, 1, 3, 4):
        assert np.array_equal(res[k].perm, oracle_sort(lists[k].bytes, lists[k].offsets))
    st = serve.latency_stats(res)
    assert st["cancelled"] == 1 and st["requests"] == 4
    assert srv.pool_used == 0


def test_cancel_before_arrival_and_of_admitted_request():
    staging, reqs, lists = make_requests([300, 300, 300, 300], [0.0, 0.0, 0.0, 0.02])
    clock = serve.VirtualClock()
    ex = serve.HostExecutor(staging, oracle_sort, clock, slots=1, cost=lambda w: 0.01)
    srv = serve.Server(ex, pool_bytes=1 << 30, clock=clock, max_batch_words=300)
    # 1 and 2 are admitted at 0 but wait for the one slot; 3 is cancelled before it arrives
    res = srv.run(reqs, cancels=[(0.005, 1), (0.01, 3)])
    assert [r.cancelled for r in res] == [False, True, False, True]
    assert res[2].launched == pytest.approx(0.01)
    for h in ex.log:
        assert 1 not in h["rids"] and 3 not in h["rids"]
    for k in (0, 2):
        assert np.array_equal(res[k].perm, oracle_sort(lists[k].bytes, lists[k].offsets))
    assert srv.pool_used == 0


@pytest.mark.gpu
def test_gpu_server_small_pool_refusal_and_cancel():
    """A pool for a few requests at a time: requests queue for memory, one
    too large for the pool is refused in the middle of the staging arrays,
    one queued request is cancelled; every other result equals the oracle's
    and the same list sorted alone."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6603_amd as bs
    rng = np.random.default_rng(77)
    n = 24
    sizes = np.floor(1000 * (30 ** rng.random(n))).astype(int)
    sizes[9] = 200_000                           # refused: larger than the pool
    arrivals = np.sort(rng.uniform(0, 0.004, n))
    staging, reqs, lists = make_requests(sizes, arrivals, seed=8, lmax=12)
    fps = [serve.request_footprint(r.n, r.n_bytes, 12, bs.workspace_bytes) for r in reqs]
    pool = serve._up(max(fp for i, fp in enumerate(fps) if i != 9)) * 3
    assert fps[9] > pool
    ex = serve.GpuExecutor(staging, arena_bytes=pool, streams=2)
    srv = serve.Server(ex, clock=serve.WallClock())
    res = srv.run(reqs, cancels=[(float(arrivals[15]), 15)])
    assert res[9].refused
    assert srv.pool_high <= pool
    ws = bs.Workspace()
    for k, (r, w) in enumerate(zip(res, lists)):
        if k == 9 or r.cancelled:
            continue
        expect = oracle.definition_sort(w.bytes, w.offsets)
        assert np.array_equal(r.perm, expect), f"request {k}"
        b, o = bs.to_device(w.bytes, w.offsets)
        assert np.array_equal(bs.sort(b, o, 12, ws=ws).cpu().numpy(), expect)


@pytest.mark.gpu
def test_gpu_server_results_same_alone_and_in_the_mix():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6603_amd as bs
    rng = np.random.default_rng(55)
    n = 60
    sizes = np.floor(1000 * (100 ** rng.random(n))).astype(int)      # 1e3 .. 1e5 words
    arrivals = np.cumsum(rng.exponential(1 / 2000.0, n))
    staging, reqs, lists = make_requests(sizes, arrivals, seed=7, lmax=12)
    ex = serve.GpuExecutor(staging, arena_bytes=1 << 30, streams=3)
    srv = serve.Server(ex)
    res = srv.run(reqs)
    ws = bs.Workspace()
    for r, w in zip(res, lists):
        assert not r.refused
        expect = oracle.definition_sort(w.bytes, w.offsets)
        assert np.array_equal(r.perm, expect)
        b, o = bs.to_device(w.bytes, w.offsets)
        alone = bs.sort(b, o, 12, ws=ws).cpu().numpy()
        assert np.array_equal(alone, r.perm)
    assert srv.batches < n                    # requests were batched together
    st = serve.latency_stats(res)
    assert st["requests"] == n
