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
    ex = serve.GpuExecutor(staging, streams=3)
    srv = serve.Server(ex, pool_bytes=1 << 30)
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
