"""GPU pre-processing (raw text -> words) vs the CPU oracle, through the C ABI.

Byte and index work: every comparison is bit-exact.  Sizes span one and many
16 KiB tiles, ragged tails, every alignment of the text pointer, words
spanning whole tiles, tiles that fill the write pass's staging, and texts of
32 and 96 MiB.
"""
import numpy as np
import pytest
import torch

import oracle
import wordgen
from tests.conftest import load_golden, load_golden_text

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


def gpu_tokenize(bs, ws, text: np.ndarray, shift: int = 0):
    """Tokenize `text` placed `shift` bytes into a device buffer (so the
    pointer the library sees has that alignment)."""
    buf = torch.zeros(len(text) + shift + 16, dtype=torch.uint8, device="cuda")
    buf[:shift] = ord("q")                   # letters just outside the text must not leak in
    buf[shift + len(text):] = ord("q")
    if len(text):
        buf[shift:shift + len(text)] = torch.from_numpy(np.ascontiguousarray(text))
    view = buf[shift:shift + len(text)]
    words, offsets, ml = bs.tokenize(view, ws=ws)
    return words.cpu().numpy(), offsets.cpu().numpy(), ml


def check_against_oracle(bs, ws, text, shift=0):
    b, o, ml = gpu_tokenize(bs, ws, text, shift)
    eb, eo = oracle.tokenize(text)
    assert np.array_equal(o, eo)
    assert np.array_equal(b, eb)
    assert ml == (int(np.diff(eo).max()) if len(eo) > 1 else 0)


def test_golden_text(bs, ws):
    text = np.frombuffer(load_golden_text("hand_text.txt"), dtype=np.uint8)
    wl, perm, _ = load_golden("hand_text.txt")
    b, o, ml = gpu_tokenize(bs, ws, text)
    assert [bytes(b[o[i]:o[i + 1]]) for i in range(len(o) - 1)] == wl
    assert ml == 8


@pytest.mark.parametrize("n", [0, 1, 2, 15, 16, 17, 255, 4095, 4096, 4097, 12289, 100_003])
def test_random_bytes_sizes(bs, ws, n):
    rng = np.random.default_rng(n)
    check_against_oracle(bs, ws, rng.integers(0, 256, size=n).astype(np.uint8))
    # mostly letters: long words crossing thread and tile edges
    al = np.frombuffer(b"abcdefghijXYZ .", dtype=np.uint8)
    check_against_oracle(bs, ws, al[rng.integers(0, len(al), size=n)])


@pytest.mark.parametrize("shift", list(range(16)))
def test_every_alignment(bs, ws, shift):
    rng = np.random.default_rng(100 + shift)
    al = np.frombuffer(b"ab Z,\x80", dtype=np.uint8)
    for n in (1, 5, 16, 31, 4100, 9000):
        check_against_oracle(bs, ws, al[rng.integers(0, len(al), size=n)], shift)


def test_edge_bytes(bs, ws):
    """The bytes around the letter ranges, each alone, in runs and mixed."""
    edge = np.array([0x00, 0x40, 0x41, 0x5A, 0x5B, 0x60, 0x61, 0x7A, 0x7B, 0x7F, 0x80, 0xC1,
                     0xDA, 0xE1, 0xFA, 0xFF], dtype=np.uint8)
    check_against_oracle(bs, ws, edge)
    check_against_oracle(bs, ws, np.repeat(edge, 17))
    rng = np.random.default_rng(7)
    check_against_oracle(bs, ws, edge[rng.integers(0, len(edge), size=50_000)])


def test_all_letters_one_word(bs, ws):
    """No separator at all: one word spanning every tile."""
    for reps in (5000, 20_000):
        text = np.frombuffer(b"Abc" * reps, dtype=np.uint8)
        b, o, ml = gpu_tokenize(bs, ws, text, shift=reps % 7)
        assert o.tolist() == [0, len(text)] and ml == len(text)
        assert np.array_equal(b, text)


@pytest.mark.parametrize("run", [16383, 16384, 16385, 40_000, 70_001])
def test_long_runs_across_tiles(bs, ws, run):
    """The longest word joined across tile edges: a long run between short
    words, starting at several offsets inside a tile."""
    for lead in (0, 1, 15, 4095, 16380):
        text = np.frombuffer(b"a " * (lead // 2) + b"-" * (lead % 2) + b"Q" * run + b" zz yy",
                             dtype=np.uint8)
        check_against_oracle(bs, ws, text)


def test_no_letters(bs, ws):
    text = np.frombuffer(b" ,.!?\n\t12\x80" * 1000, dtype=np.uint8)
    b, o, ml = gpu_tokenize(bs, ws, text)
    assert o.tolist() == [0] and len(b) == 0 and ml == 0


@pytest.mark.parametrize("k", [1, 2, 3])
def test_raw_text_round_trip(bs, ws, k):
    """Words joined by separators come back exactly (property at any size)
    and equal the oracle's tokens."""
    w = wordgen.single(k)
    text = wordgen.raw_text(w, k)
    b, o, ml = gpu_tokenize(bs, ws, text)
    assert np.array_equal(o, w.offsets)
    assert np.array_equal(b, w.bytes)
    assert ml == int(np.diff(w.offsets).max())


def test_large_random_text(bs, ws):
    """32 MiB (8192 tiles) of random bytes biased to letters and spaces."""
    rng = np.random.default_rng(32)
    al = np.frombuffer(b"etaoinshrdlucmfwypvbgkjqxzETAOIN     ,.\n\x80\xff", dtype=np.uint8)
    check_against_oracle(bs, ws, al[rng.integers(0, len(al), size=32 << 20)], shift=3)


def test_capacity_exceeded(bs, ws):
    """cap_words below the word count: status BSORT_E_CAPACITY and the first
    cap_words offsets still right."""
    text = np.frombuffer(b"a b c d e f g h", dtype=np.uint8)
    t = torch.from_numpy(text.copy()).cuda()
    with pytest.raises(bs.BsortError):
        bs.tokenize(t, ws=ws, cap_words=5)
    words, offsets, result = bs.tokenize(t, ws=ws, cap_words=5, sync=False)
    r = result.cpu().tolist()
    assert r[0] == 8 and r[1] == 8 and r[2] == 1 and r[3] == 6   # BSORT_E_CAPACITY
    assert offsets[:5].cpu().tolist() == [0, 1, 2, 3, 4]


def test_sort_text_phases_1_to_3(bs, ws):
    """Raw text through the whole path: the hand-worked order of the golden
    text, and the oracle's order on a raw text of the 35,000-word list."""
    text = load_golden_text("hand_text.txt")
    _, perm_expect, _ = load_golden("hand_text.txt")
    t = torch.frombuffer(bytearray(text), dtype=torch.uint8).cuda()
    _, _, perm = bs.sort_text(t, ws=ws)
    assert perm.cpu().tolist() == perm_expect
    w = wordgen.single(2)
    t = torch.from_numpy(wordgen.raw_text(w, 5)).cuda()
    words, offsets, perm = bs.sort_text(t, ws=ws)
    bs.check_device_status(ws)
    expect = oracle.bubble_sort(w.bytes, w.offsets, threads=8)
    assert np.array_equal(perm.cpu().numpy(), expect)


def test_sort_text_word_too_long(bs, ws):
    t = torch.from_numpy(np.frombuffer(b"ok " + b"x" * 70 + b" fine", np.uint8).copy()).cuda()
    words, offsets, ml = bs.tokenize(t, ws=ws)
    assert ml == 70
    with pytest.raises(bs.BsortError):
        bs.sort_text(t, ws=ws)


TILE = 16384


@pytest.mark.parametrize("tiles", [63, 64, 65, 128, 129, 200])
def test_tile_counts(bs, ws, tiles):
    """Texts of a few hundred tiles, exact multiples and ragged: every tile's
    offsets come from the scan of the tiles' counts."""
    rng = np.random.default_rng(tiles)
    al = np.frombuffer(b"abcdefgh  ,Q", dtype=np.uint8)
    for n in (tiles * TILE - 1, tiles * TILE, tiles * TILE + 7):
        check_against_oracle(bs, ws, al[rng.integers(0, len(al), size=n)], shift=n % 5)


def test_words_spanning_whole_tiles(bs, ws):
    """Letter runs that cover whole tiles (tiles with no word start): the
    scan must carry the letters after the last word start through them."""
    rng = np.random.default_rng(11)
    al = np.frombuffer(b"ab c", dtype=np.uint8)
    text = al[rng.integers(0, len(al), size=140 * TILE)].copy()
    for start, length in ((62 * TILE + 100, 3 * TILE), (127 * TILE - 5, TILE + 10),
                          (130 * TILE, 5 * TILE + 1)):
        text[start:start + length] = ord("Z")
        text[start - 1] = ord(" ")
    check_against_oracle(bs, ws, text)
    b, o, ml = gpu_tokenize(bs, ws, text)
    assert ml >= 5 * TILE + 1


def test_workspace_reused_across_sizes(bs, ws):
    """One workspace, calls of falling and rising size back to back on one
    stream: nothing a call leaves in it reaches the next."""
    rng = np.random.default_rng(5)
    al = np.frombuffer(b"xyz w", dtype=np.uint8)
    for n in (300 * TILE + 3, 2 * TILE, 17, 70 * TILE, 0, 5 * TILE + 1):
        check_against_oracle(bs, ws, al[rng.integers(0, len(al), size=n)])


def test_large_text_with_long_runs(bs, ws):
    """96 MiB (6,144 tiles, more than the device holds at once) with long
    runs across tiles placed at random."""
    rng = np.random.default_rng(96)
    al = np.frombuffer(b"etaoinshrdlu  ,.Q", dtype=np.uint8)
    text = al[rng.integers(0, len(al), size=96 << 20)]
    for start in rng.integers(0, len(text) - 3 * TILE, size=20):
        text[start:start + int(rng.integers(1, 3 * TILE))] = ord("k")
    check_against_oracle(bs, ws, text, shift=9)


def test_tile_staging_worst_case(bs, ws):
    """Tiles holding the most letters plus 16-bit word starts the staging can
    meet: 8,193 letters and 8,192 word starts in each 16 KiB ("aa" then
    " a" repeated), tile-aligned and shifted; and one-letter words
    throughout."""
    tile = b"aa" + b" a" * ((TILE - 2) // 2)
    assert len(tile) == TILE
    text = np.frombuffer(tile * 12, dtype=np.uint8)
    for shift in (0, 1, 5):
        check_against_oracle(bs, ws, text, shift=shift)
    check_against_oracle(bs, ws, np.frombuffer(b"a " * (6 * TILE) + b"z", dtype=np.uint8))
