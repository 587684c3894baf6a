"""GPU path vs the CPU oracle, element by element, through the C ABI.

Integer work: every comparison is bit-exact.
"""
import numpy as np
import pytest
import torch

import oracle
import wordgen
from tests.conftest import load_golden

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


def gpu_sort(bs, ws, w, max_len, tune=None):
    b, o = bs.to_device(w.bytes, w.offsets)
    perm = bs.sort(b, o, max_len, tune=tune, ws=ws)
    bs.check_device_status(ws)
    return perm.cpu().numpy()


def gpu_batch(bs, ws, batch, max_len, tune=None):
    b, o = bs.to_device(batch.bytes, batch.offsets)
    rs = torch.from_numpy(batch.req_start).cuda()
    perm = bs.sort_batch(b, o, rs, batch.req_start, max_len, tune=tune, ws=ws)
    bs.check_device_status(ws)
    return perm.cpu().numpy()


def maxlen(w):
    return int(np.diff(w.offsets).max()) if w.n else 0


# ------------------------------------------------------------- single lists

@pytest.mark.parametrize("k", [1, 2, 3])
def test_bucketize_matches_oracle(bs, ws, k):
    w = wordgen.single(k)
    ml = wordgen.SINGLE[k].lmax
    b, o = bs.to_device(w.bytes, w.offsets)
    counts, starts, order = bs.bucketize(b, o, ml, ws=ws)
    bs.check_device_status(ws)
    c, s, od = oracle.bucketize(w.bytes, w.offsets, ml)
    assert np.array_equal(counts.cpu().numpy(), c)
    assert np.array_equal(starts.cpu().numpy(), s)
    assert np.array_equal(order.cpu().numpy(), od)


@pytest.mark.parametrize("k", [1, 2])
def test_sort_matches_bubble_oracle(bs, ws, k):
    w = wordgen.single(k)
    ml = wordgen.SINGLE[k].lmax
    expect = oracle.bubble_sort(w.bytes, w.offsets, max_len=ml, threads=8)
    assert np.array_equal(gpu_sort(bs, ws, w, ml), expect)


def test_sort_workload3_full(bs, ws):
    """250,000 words; buckets far beyond one tile (merge-split path)."""
    w = wordgen.single(3)
    expect = oracle.bubble_sort(w.bytes, w.offsets, max_len=24, threads=16)
    assert np.array_equal(gpu_sort(bs, ws, w, 24), expect)


@pytest.mark.parametrize("tile,mt", [(128, 256), (256, 64), (512, 256), (1024, 1024),
                                     (2048, 128), (4096, 256), (0, 0)])
def test_tuning_does_not_change_bits(bs, ws, tile, mt):
    w = wordgen.single(2)
    expect = oracle.definition_sort(w.bytes, w.offsets)
    got = gpu_sort(bs, ws, w, 20, tune=bs.tuning(tile, mt))
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("tile,hbm_tile,mt", [(128, 128, 64), (256, 2048, 256), (1024, 4096, 1024),
                                              (512, 256, 512)])
def test_hbm_and_lds_paths_workload3(bs, ws, tile, hbm_tile, mt):
    """250,000 words: sub-arrays up to ~50,000 words exceed LDS and take the
    HBM merge-split path; the rest are sorted whole in LDS."""
    w = wordgen.single(3)
    expect = oracle.definition_sort(w.bytes, w.offsets)
    got = gpu_sort(bs, ws, w, 24, tune=bs.tuning(tile, mt, 0, hbm_tile))
    assert np.array_equal(got, expect)


def test_tiles_only_sorts_each_tile(bs, ws):
    """With the merge-split switched off every tile is sorted on its own:
    tile t of a sub-array is the sorted form of its slice of the stable
    sub-array order (seams between tiles are not merged)."""
    w = wordgen.single(2)
    T = 128
    got = gpu_sort(bs, ws, w, 20, tune=bs.tuning(T, 0, bs.FLAG_TILES_ONLY, hbm_tile_keys=T))
    counts, starts, order = oracle.bucketize(w.bytes, w.offsets, 20)
    wl = w.as_list()
    for L in range(1, 21):
        a, n = int(starts[L]), int(counts[L])
        if n < 2:
            continue
        for t0 in range(0, n, T):
            idx = order[a + t0:a + min(n, t0 + T)]
            exp = sorted(idx.tolist(), key=lambda i: (wl[i], i))
            assert got[a + t0:a + t0 + len(idx)].tolist() == exp


@pytest.mark.parametrize("name", ["hand_sentence.txt", "hand_bytes.txt"])
def test_golden_fixtures(bs, ws, name):
    wl, perm, counts = load_golden(name)
    w = wordgen.Words.from_list(wl)
    assert gpu_sort(bs, ws, w, maxlen(w)).tolist() == perm


def edge_cases():
    rng = np.random.default_rng(2024)
    cases = {
        "one_word": wordgen.Words.from_list([b"x"]),
        "two_equal": wordgen.Words.from_list([b"ab", b"ab"]),
        "all_equal_5000": wordgen.Words.from_list([b"same"] * 5000),
        "empty_words_only": wordgen.Words.from_list([b""] * 100),
        "empty_and_short": wordgen.Words.from_list([b"", b"b", b"", b"a", b"", b"ab", b"A"]),
        "high_bytes": wordgen.random_words(rng, 3000, 1, 3, alphabet=b"\x00\x01\x7f\x80\xfe\xff"),
        "all_byte_values": wordgen.random_words(rng, 20000, 0, 12),
        "max_len_64": wordgen.random_words(rng, 4000, 60, 64, alphabet=b"ab"),
        "reverse_sorted": wordgen.Words.from_list(
            [bytes([97 + (i // 676) % 26, 97 + (i // 26) % 26, 97 + i % 26]) for i in range(9000)][::-1]),
        "n_1_mod_64": wordgen.random_words(rng, 64 * 37 + 1, 4, 4, alphabet=b"abc"),
        "odd_n": wordgen.random_words(rng, 1023, 2, 2, alphabet=b"xyzXYZ"),
        "huge_dup_bucket": wordgen.random_words(rng, 100_000, 3, 3, alphabet=b"ab"),
        "one_bucket_big_distinct": wordgen.random_words(rng, 60_000, 8, 8),
    }
    for L in (4, 5, 7, 8, 9, 12, 13, 15, 16, 17, 24, 25, 31, 32, 33, 40, 48, 56, 63, 64):
        cases[f"len_{L}"] = wordgen.random_words(rng, 700, L, L, alphabet=b"aAb\xff")
    return cases


EDGE = edge_cases()


@pytest.mark.parametrize("name", sorted(EDGE))
def test_edge_cases(bs, ws, name):
    w = EDGE[name]
    ml = max(maxlen(w), 1)
    expect = oracle.definition_sort(w.bytes, w.offsets)
    if w.n <= 20000:
        assert np.array_equal(oracle.bubble_sort(w.bytes, w.offsets, max_len=ml, threads=8), expect)
    got = gpu_sort(bs, ws, w, ml)
    assert np.array_equal(got, expect), name
    got_small_tiles = gpu_sort(bs, ws, w, ml, tune=bs.tuning(128, 64))
    assert np.array_equal(got_small_tiles, expect), name


def test_sort_buckets_on_a_fresh_workspace(bs, ws):
    """sort_buckets must not depend on what bucketize left in its workspace:
    bucketize with one workspace, sort with another full of junk (status word
    cleared)."""
    w = wordgen.single(2)
    b, o = bs.to_device(w.bytes, w.offsets)
    counts, starts, order = bs.bucketize(b, o, 20, ws=ws)
    bs.check_device_status(ws)
    junk = bs.Workspace(bs.workspace_bytes(w.n, 20, 1))
    junk.tensor.fill_(0x5A)
    junk.tensor[:512].zero_()
    torch.cuda.synchronize()
    perm = bs.sort_buckets(b, o, counts, starts, order, 20, ws=junk)
    bs.check_device_status(junk)
    assert np.array_equal(perm.cpu().numpy(), oracle.definition_sort(w.bytes, w.offsets))


def test_empty_list(bs, ws):
    w = wordgen.Words.from_list([])
    b, o = bs.to_device(w.bytes, w.offsets)
    counts, starts, order = bs.bucketize(b, o, 8, ws=ws)
    bs.check_device_status(ws)
    assert counts.cpu().numpy().tolist() == [0] * 9
    assert starts.cpu().numpy().tolist() == [0] * 10
    perm = bs.sort_buckets(b, o, counts, starts, order, 8, ws=ws)
    assert perm.numel() == 0


def test_repeat_is_deterministic(bs, ws):
    """An LDS or cross-lane race would show as run-to-run differences."""
    w = wordgen.single(2)
    first = gpu_sort(bs, ws, w, 20, tune=bs.tuning(256, 64))
    for _ in range(10):
        assert np.array_equal(gpu_sort(bs, ws, w, 20, tune=bs.tuning(256, 64)), first)


# ------------------------------------------------------------- 0-1 principle

def zero_one_batch(seqs, width=1):
    pad = b"0" * (width - 1)
    words = []
    for s in seqs:
        words.extend(pad + (b"1" if x else b"0") for x in s)
    req = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum([len(s) for s in seqs], out=req[1:])
    w = wordgen.Words.from_list(words)
    return wordgen.Batch(w.bytes, w.offsets, req)


def zero_one_expect(seqs):
    out = []
    for s in seqs:
        s = np.asarray(s, dtype=np.int8)
        out.append(np.concatenate([np.nonzero(s == 0)[0], np.nonzero(s == 1)[0]]))
    return np.concatenate(out).astype(np.int32)


def test_zero_one_exhaustive(bs, ws):
    """Odd-even transposition sort is a comparator network, so it sorts all
    inputs if it sorts all 0/1 inputs (Knuth, TAOCP 3, 5.3.4).  Every 0/1
    sequence of length 1..14."""
    seqs = []
    for n in range(1, 15):
        v = np.arange(2 ** n, dtype=np.int64)[:, None]
        bits = (v >> np.arange(n - 1, -1, -1)) & 1
        seqs.extend(list(bits.astype(np.int8)))
    batch = zero_one_batch(seqs)
    got = gpu_batch(bs, ws, batch, 1, tune=bs.tuning(128, 64))
    assert np.array_equal(got, zero_one_expect(seqs))


def test_zero_one_exhaustive_15_to_20(bs, ws):
    """The 0/1 principle continued: every 0/1 sequence of length 15..20
    (2,064,384 sequences, 40.9 M words), sorted as lists of one-byte words,
    65,536 lists per batch.  The expected order of a 0/1 list is the stable
    partition: the zeros' indices, then the ones'."""
    chunk = 1 << 16
    for n in range(15, 21):
        shifts = np.arange(n - 1, -1, -1, dtype=np.int64)
        for v0 in range(0, 1 << n, chunk):
            v = np.arange(v0, min(v0 + chunk, 1 << n), dtype=np.int64)
            bits = ((v[:, None] >> shifts) & 1).astype(np.uint8)
            m = len(v)
            batch = wordgen.Batch((bits.ravel() + ord("0")).astype(np.uint8),
                                  np.arange(m * n + 1, dtype=np.int64),
                                  np.arange(0, m * n + 1, n, dtype=np.int64))
            got = gpu_batch(bs, ws, batch, 1, tune=bs.tuning(128, 64))
            expect = np.argsort(bits, axis=1, kind="stable").astype(np.int32).ravel()
            assert np.array_equal(got, expect), f"n={n}, sequences {v0}..{v0 + m - 1}"


@pytest.mark.parametrize("T", [128, 256])
def test_zero_one_merge_seams(bs, ws, T):
    """Random 0/1 lists whose sizes sit on tile seams: the merge-split
    network across tiles, ragged last tiles included."""
    rng = np.random.default_rng(T)
    seqs = []
    for n in (T - 1, T, T + 1, 2 * T - 1, 2 * T, 2 * T + 1, 3 * T, 3 * T + 7, 7 * T + 5, 16 * T + 3):
        for _ in range(40):
            p = rng.random()
            seqs.append((rng.random(n) < p).astype(np.int8))
    # past the largest in-LDS sub-array: tiles merged phase by phase through HBM
    for n in (16321, 16320 + 3 * T + 1, 20000):
        for _ in range(3):
            p = rng.random()
            seqs.append((rng.random(n) < p).astype(np.int8))
    batch = zero_one_batch(seqs)
    got = gpu_batch(bs, ws, batch, 1, tune=bs.tuning(T, 64, 0, T))
    assert np.array_equal(got, zero_one_expect(seqs))


def lds_caps(D):
    """In-LDS size-class capacities for record width D (largest class per
    width within 144 KiB of LDS; widths 6-9 have the classes up to 4,096)."""
    top = {2: 16320, 3: 12288, 4: 9216, 5: 7168}.get(D, 8192)
    return [c for c in (1024, 2048, 4096, 8192, top) if D * 4 * c <= 144 * 1024]


def lds_tile(tuned, cap, D):
    target = 512 if D <= 2 else cap // 16
    t = tuned
    while t < target and t < 512:
        t <<= 1
    return t


@pytest.mark.parametrize("L", [1, 5, 9, 13, 17, 21, 25, 29])
def test_zero_one_lds_classes(bs, ws, L):
    """0/1 keys of width L (record widths D = 2..9) at the bounds of every
    in-LDS size class, one class tile past each lower bound, and past the
    largest class (merge-split through HBM): the stable partition."""
    T = 128
    D = (L + 3) // 4 + 1
    rng = np.random.default_rng(1000 + L)
    sizes, prev = [], T
    for cap in lds_caps(D):
        sizes += [prev + 1, prev + lds_tile(T, cap, D) + 1, cap - 1, cap]
        prev = cap
    sizes += [prev + 1, prev + 3 * T + 1]
    seqs = []
    for n in sizes:
        p = rng.random()
        seqs.append((rng.random(n) < p).astype(np.int8))
    batch = zero_one_batch(seqs, L)
    got = gpu_batch(bs, ws, batch, L, tune=bs.tuning(T, 64, 0, T))
    assert np.array_equal(got, zero_one_expect(seqs))


@pytest.mark.parametrize("alphabet", [b"eatonsEAT", None, b"ab\x7f\x80\xff"])
def test_five_six_byte_words_in_every_class(bs, ws, alphabet):
    """5- and 6-byte words, whose in-LDS records carry the word's position in
    the key's spare low bits: letters (exact fp64 tiles), all byte values and
    bytes at and above 0x7F (the integer fallback for some or all tiles),
    heavy duplicates, sizes at every three-dword size class and past the
    largest (merged through HBM, without the spare-bit form)."""
    rng = np.random.default_rng(56)
    lists = []
    for cap in lds_caps(3) + [12288 + 129]:
        for L in (5, 6):
            for n in (cap - 1, cap // 2 + 3):
                if alphabet is None:
                    w = wordgen.random_words(rng, n, L, L)
                else:
                    # a few distinct words, so ties are everywhere
                    pool = wordgen.random_words(rng, 40, L, L, alphabet=alphabet).as_list()
                    w = wordgen.Words.from_list([pool[i] for i in rng.integers(0, 40, n)])
                lists.append(w)
    batch = wordgen.Batch.concat(lists)
    expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
    for T in (128, 512):
        got = gpu_batch(bs, ws, batch, 6, tune=bs.tuning(T, 0))
        assert np.array_equal(got, expect), T


@pytest.mark.parametrize("alphabet", [b"eatonsEAT", None, b"\x00\x01\x7f\x80\xfe\xff"])
def test_one_two_byte_words_in_every_class(bs, ws, alphabet):
    """1- and 2-byte words, whose in-LDS records are one dword (the key's
    high half, the position in the low half, compared whole): letters, all
    byte values, the extreme bytes (zero and all-ones keys), heavy duplicates,
    sizes at every two-dword size class and past the largest (merged through
    HBM, in the two-dword form)."""
    rng = np.random.default_rng(12)
    lists = []
    for cap in lds_caps(2) + [16320 + 129]:
        for L in (1, 2):
            for n in (cap - 1, cap // 2 + 3):
                if alphabet is None:
                    w = wordgen.random_words(rng, n, L, L)
                else:
                    pool = wordgen.random_words(rng, 40, L, L, alphabet=alphabet).as_list()
                    w = wordgen.Words.from_list([pool[i] for i in rng.integers(0, 40, n)])
                lists.append(w)
    batch = wordgen.Batch.concat(lists)
    expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
    for T in (128, 512):
        got = gpu_batch(bs, ws, batch, 2, tune=bs.tuning(T, 0))
        assert np.array_equal(got, expect), T


@pytest.mark.parametrize("alphabet", [b"eatonsEAT", None, b"\x00\x01\x7f\x80\xfe\xff",
                                      "sprinkle", "max_packed"])
def test_three_four_byte_words_in_every_class(bs, ws, alphabet):
    """3- and 4-byte words (two-dword records; in LDS a tile of 3-byte words
    whose first bytes are all below 0x80 sorts as one dword per record, the
    key's bits above the tile position): letters, all byte values and the
    extreme bytes (tiles with a first byte >= 0x80 take the two-dword form),
    letters with a sprinkle of high first bytes (some tiles packed, some
    not), and keys at the packed form's top (7F FF FE/FF, full tiles
    included), heavy duplicates, sizes at every two-dword size class and
    past the largest (merged through HBM)."""
    rng = np.random.default_rng(34)
    lists = []
    for cap in lds_caps(2) + [16320 + 129]:
        for L in (3, 4):
            for n in (cap - 1, cap // 2 + 3, 1024):
                if alphabet is None:
                    w = wordgen.random_words(rng, n, L, L)
                elif alphabet == "sprinkle":
                    pool = wordgen.random_words(rng, 40, L, L, alphabet=b"eatonsEAT").as_list()
                    words = [pool[i] for i in rng.integers(0, 40, n)]
                    for i in rng.integers(0, n, max(1, n // 700)):
                        words[i] = bytes([0x80 + int(rng.integers(0, 128))]) + words[i][1:]
                    w = wordgen.Words.from_list(words)
                elif alphabet == "max_packed":
                    head = b"\x7f" + b"\xff" * (L - 2)
                    w = wordgen.Words.from_list(
                        [head + bytes([int(x)]) for x in rng.choice([0xFE, 0xFF], n)])
                else:
                    pool = wordgen.random_words(rng, 40, L, L, alphabet=alphabet).as_list()
                    w = wordgen.Words.from_list([pool[i] for i in rng.integers(0, 40, n)])
                lists.append(w)
    batch = wordgen.Batch.concat(lists)
    expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
    for T in (128, 512):
        got = gpu_batch(bs, ws, batch, 4, tune=bs.tuning(T, 0))
        assert np.array_equal(got, expect), T
        got = gpu_batch(bs, ws, batch, 4, tune=bs.tuning(T, 0, bs.FLAG_LDS_TILE))
        assert np.array_equal(got, expect), (T, "tuned in-LDS tile")


@pytest.mark.parametrize("alphabet", [b"eatonsEAT", None, b"\x00\x01\x7f\x80\xfe\xff"])
def test_nine_ten_byte_words_in_every_class(bs, ws, alphabet):
    """9- and 10-byte words (four-dword records, the last key dword half
    padding): letters, all byte values, the extreme bytes, heavy duplicates,
    sizes at every four-dword size class and past the largest (merged
    through HBM)."""
    rng = np.random.default_rng(910)
    lists = []
    for cap in lds_caps(4) + [9216 + 129]:
        for L in (9, 10):
            for n in (cap - 1, cap // 2 + 3):
                if alphabet is None:
                    w = wordgen.random_words(rng, n, L, L)
                else:
                    pool = wordgen.random_words(rng, 40, L, L, alphabet=alphabet).as_list()
                    w = wordgen.Words.from_list([pool[i] for i in rng.integers(0, 40, n)])
                lists.append(w)
    batch = wordgen.Batch.concat(lists)
    expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
    for T in (128, 512):
        got = gpu_batch(bs, ws, batch, 10, tune=bs.tuning(T, 0))
        assert np.array_equal(got, expect), T


@pytest.mark.parametrize("alphabet", [b"eatonsEAT", None, b"\x00\x01\x7f\x80\xfe\xff", "prefix"])
def test_long_words_in_every_class(bs, ws, alphabet):
    """17- to 32-byte words (records of 6-9 dwords, whose in-LDS classes hold
    up to 4,096 words): letters, all byte values, the extreme bytes, and
    words that share all but their last two bytes (every key dword but the
    last ties), heavy duplicates, sizes at every class and past the largest
    (merged through HBM)."""
    rng = np.random.default_rng(1732)
    lists = []
    for cap in lds_caps(6) + [4096 + 129]:
        for L in (17, 24, 25, 32):
            for n in (cap - 1, cap // 2 + 3):
                if alphabet is None:
                    w = wordgen.random_words(rng, n, L, L)
                elif alphabet == "prefix":
                    head = bytes(rng.integers(97, 123, L - 2, dtype=np.uint8))
                    tails = rng.integers(0, 256, (n, 2), dtype=np.uint8)
                    w = wordgen.Words.from_list([head + bytes(t) for t in tails])
                else:
                    pool = wordgen.random_words(rng, 40, L, L, alphabet=alphabet).as_list()
                    w = wordgen.Words.from_list([pool[i] for i in rng.integers(0, 40, n)])
                lists.append(w)
    batch = wordgen.Batch.concat(lists)
    expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
    for T in (128, 512):
        got = gpu_batch(bs, ws, batch, 32, tune=bs.tuning(T, 0))
        assert np.array_equal(got, expect), T


def test_large_serve_request_merged_through_hbm(bs, ws):
    """A 1,000,000-word request of the serving workload (lengths to 32, one
    200,000-word vocabulary): its large sub-arrays are cut into chunks sorted
    in LDS and merged phase by phase through HBM."""
    w = wordgen.serve_request(3, 1_000_000)
    expect = oracle.definition_sort(w.bytes, w.offsets)
    assert np.array_equal(gpu_sort(bs, ws, w, 32), expect)
    # the same through a two-list batch
    batch = wordgen.Batch.concat([w, wordgen.serve_request(4, 3000)])
    got = gpu_batch(bs, ws, batch, 32)
    assert np.array_equal(got[:w.n], expect)


def _busy_stream(mib=2048, copies=6):
    """Queue several large device-to-device copies on the current stream, so
    that it stays busy for milliseconds after this returns."""
    a = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(copies):
        b.copy_(a)
    return a, b


def test_sort_calls_do_not_block_the_host(bs, ws):
    """bsort_sort_batch and bsort_sort_buckets on lists whose sub-arrays merge
    through HBM return while the stream still has the copies queued before
    them (no host synchronisation inside the calls); the results are exact."""
    w = wordgen.serve_request(3, 1_000_000)
    expect = oracle.definition_sort(w.bytes, w.offsets)
    batch = wordgen.Batch.concat([w, wordgen.serve_request(4, 3000)])
    b, o = bs.to_device(batch.bytes, batch.offsets)
    rs = torch.from_numpy(batch.req_start).cuda()
    bw, ow = bs.to_device(w.bytes, w.offsets)
    out = torch.empty(batch.total, dtype=torch.int32, device="cuda")
    ws.ensure(bs.workspace_bytes(batch.total, 32, batch.R))
    torch.cuda.synchronize()
    keep = _busy_stream()
    bs.sort_batch(b, o, rs, batch.req_start, 32, ws=ws, out=out)
    assert not torch.cuda.current_stream().query(), "sort_batch waited for the stream"
    bs.check_device_status(ws)
    assert np.array_equal(out[:w.n].cpu().numpy(), expect)
    keep = _busy_stream()
    perm = bs.sort(bw, ow, 32, ws=ws)
    assert not torch.cuda.current_stream().query(), "bucketize/sort_buckets waited"
    bs.check_device_status(ws)
    assert np.array_equal(perm.cpu().numpy(), expect)
    del keep


def test_merge_stall_is_reported(bs, ws):
    """With the stall test flag every merge-split wait gives up at once: the
    launch ends and the device status says so; the next call is exact."""
    w = wordgen.serve_request(3, 1_000_000)
    b, o = bs.to_device(w.bytes, w.offsets)
    bs.sort(b, o, 32, tune=bs.tuning(0, 0, bs.FLAG_STALL_TEST), ws=ws)
    with pytest.raises(bs.BsortError, match="gave up"):
        bs.check_device_status(ws)
    perm = bs.sort(b, o, 32, ws=ws)
    bs.check_device_status(ws)
    assert np.array_equal(perm.cpu().numpy(), oracle.definition_sort(w.bytes, w.offsets))


def test_plan_with_hbm_merges_replays(bs):
    """A captured plan over lists whose sub-arrays merge through HBM (one
    merge launch in the graph, its work found on the device), replayed on
    two batches; each result equals the oracle."""
    a = wordgen.Batch.concat([wordgen.serve_request(5, 600_000), wordgen.serve_request(6, 5_000)])
    c = wordgen.Batch.concat([wordgen.serve_request(7, 2_000), wordgen.serve_request(8, 400_000),
                              wordgen.serve_request(9, 90_000)])
    plan = bs.Plan(max(a.total, c.total), 3, 600_000, 32)
    pws = bs.Workspace(plan.workspace_bytes)
    for batch in (a, c, a):
        bt, ot = bs.to_device(batch.bytes, batch.offsets)
        rs = torch.from_numpy(batch.req_start).cuda()
        perm = plan.execute(bt, ot, rs, batch.req_start, pws)
        bs.check_device_status(pws)
        expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
        assert np.array_equal(perm.cpu().numpy(), expect)
    plan.close()


# ------------------------------------------------------------- batches

@pytest.fixture(scope="module")
def batch_small():
    return wordgen.batch(first=0, count=256)


def test_batch_matches_oracle(bs, ws, batch_small):
    expect, _ = oracle.bubble_sort_batch(batch_small.bytes, batch_small.offsets,
                                         batch_small.req_start, 12, threads=16)
    assert np.array_equal(gpu_batch(bs, ws, batch_small, 12), expect)


def test_batch_equals_each_list_alone(bs, ws, batch_small):
    got = gpu_batch(bs, ws, batch_small, 12)
    for r in range(0, batch_small.R, 17):
        w = batch_small.request(r)
        alone = gpu_sort(bs, ws, w, 12)
        a, b = batch_small.req_start[r], batch_small.req_start[r + 1]
        assert np.array_equal(got[a:b], alone)


def test_plain_per_bucket_form_equals_batched(bs, ws, batch_small):
    sub = wordgen.Batch.concat([batch_small.request(r) for r in range(64)])
    batched = gpu_batch(bs, ws, sub, 12)
    plain = gpu_batch(bs, ws, sub, 12, tune=bs.tuning(0, 0, bs.FLAG_PER_BUCKET_LAUNCH))
    assert np.array_equal(plain, batched)
    expect = oracle.definition_sort_batch(sub.bytes, sub.offsets, sub.req_start, 16)
    assert np.array_equal(batched, expect)


def test_serial_stages_equal_fanned_out(bs, ws, batch_small):
    """Every stage on the caller's stream gives the same bits as the default
    fan-out over the library's streams, on a batch and on a list whose
    largest sub-arrays merge through HBM."""
    fanned = gpu_batch(bs, ws, batch_small, 12)
    serial = gpu_batch(bs, ws, batch_small, 12, tune=bs.tuning(0, 0, bs.FLAG_SERIAL_STAGES))
    assert np.array_equal(serial, fanned)
    w = wordgen.single(3)
    got = gpu_sort(bs, ws, w, 24, tune=bs.tuning(0, 0, bs.FLAG_SERIAL_STAGES))
    assert np.array_equal(got, oracle.definition_sort(w.bytes, w.offsets))


def test_plan_replays_on_new_batches(bs, batch_small):
    """A captured plan run twice in a row, the second time on a smaller batch
    with other buffers; each result equals the oracle."""
    a = wordgen.Batch.concat([batch_small.request(r) for r in range(0, 120)])
    b = wordgen.Batch.concat([batch_small.request(r) for r in range(200, 240)])
    cap_req = int(max(np.diff(a.req_start).max(), np.diff(b.req_start).max()))
    plan = bs.Plan(a.total, a.R, cap_req, 12)
    pws = bs.Workspace(plan.workspace_bytes)
    for batch in (a, b, a):
        bt, ot = bs.to_device(batch.bytes, batch.offsets)
        rs = torch.from_numpy(batch.req_start).cuda()
        perm = plan.execute(bt, ot, rs, batch.req_start, pws)
        bs.check_device_status(pws)
        expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
        assert np.array_equal(perm.cpu().numpy(), expect)
    plan.close()


def test_full_batch_workload(bs, ws):
    """The batching workload at full size (4,096 lists, ~31.8 M words), in
    the launch configuration the benchmark times: every list against the
    oracle's definition sort."""
    batch = wordgen.batch()
    got = gpu_batch(bs, ws, batch, 12)
    expect = oracle.definition_sort_batch(batch.bytes, batch.offsets, batch.req_start, 16)
    assert np.array_equal(got, expect)


# ------------------------------------------------------------- faults

def test_device_status_too_long(bs, ws):
    w = wordgen.Words.from_list([b"ab", b"abcdefghij", b"a"])
    b, o = bs.to_device(w.bytes, w.offsets)
    bs.sort(b, o, 4, ws=ws)
    assert bs.device_status(ws) == 2
    assert bs.device_status(ws) == 0          # read clears it


def test_device_status_bad_offsets(bs, ws):
    buf = np.frombuffer(b"abcdefgh", np.uint8).copy()
    off = np.array([0, 4, 2, 8, 20], np.int64)   # decreasing, and past n_bytes
    b, o = bs.to_device(buf, off)
    bs.sort(b, o, 16, ws=ws)
    assert bs.device_status(ws) == 1


def test_workspace_too_small(bs):
    import ctypes
    from paper_1407_6603_amd import _lib
    w = wordgen.single(1)
    b, o = bs.to_device(w.bytes, w.offsets)
    tiny = bs.Workspace(256)
    wd = _lib.Words(b.data_ptr(), b.numel(), o.data_ptr(), w.n, 12)
    bk = _lib.Buckets(o.data_ptr(), o.data_ptr(), o.data_ptr())
    rc = _lib.load().bsort_bucketize(ctypes.byref(wd), ctypes.byref(bk), tiny.ptr, 256, None)
    assert rc == 4


def test_staged_batch_equals_unstaged(bs, ws, batch_small):
    """The stage-timed entry point records events between stages and gives
    the same bits."""
    sub = wordgen.Batch.concat([batch_small.request(r) for r in range(100)])
    b, o = bs.to_device(sub.bytes, sub.offsets)
    rs = torch.from_numpy(sub.req_start).cuda()
    timer = bs.StageTimer(12)
    perm = bs.sort_batch_staged(b, o, rs, sub.req_start, 12, timer, ws=ws)
    ms = timer.ms()
    bs.check_device_status(ws)
    assert list(ms) == bs.stage_names(12)
    assert all(v >= 0 for v in ms.values())
    assert np.array_equal(perm.cpu().numpy(), gpu_batch(bs, ws, sub, 12))



def test_staged_batch_times_only_chosen_stages(bs, ws, batch_small):
    """NULL entries of the event array record nothing: a timer of two stages
    reports those two, and the bits do not change."""
    sub = wordgen.Batch.concat([batch_small.request(r) for r in range(100)])
    b, o = bs.to_device(sub.bytes, sub.offsets)
    rs = torch.from_numpy(sub.req_start).cuda()
    pick = {"bucketize", "lds_d2_1024"}
    timer = bs.StageTimer(12, only=pick)
    assert sum(h is not None for h in timer.handles) == 2 * len(pick)
    perm = bs.sort_batch_staged(b, o, rs, sub.req_start, 12, timer, ws=ws)
    ms = timer.ms()
    bs.check_device_status(ws)
    assert set(ms) == pick and all(v >= 0 for v in ms.values())
    none = bs.StageTimer(12, only=())
    perm2 = bs.sort_batch_staged(b, o, rs, sub.req_start, 12, none, ws=ws)
    assert none.ms() == {}
    ref = gpu_batch(bs, ws, sub, 12)
    assert np.array_equal(perm.cpu().numpy(), ref)
    assert np.array_equal(perm2.cpu().numpy(), ref)
