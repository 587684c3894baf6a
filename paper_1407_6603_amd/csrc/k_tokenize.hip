// Pre-processing (Section II, phase 1; Section III, approach one step 2):
// raw text to words.  The paper drops "special characters" (its examples are
// quote, comma, full stop, question and exclamation marks) before splitting
// the text into words; here a word is a maximal run of ASCII letters
// [A-Za-z] and every other byte separates words and is dropped.  The words
// come out in the library's input format: their letters back to back and
// int64 offsets, word i = out[offsets[i] .. offsets[i+1]).
//
// A stream compaction bound by HBM bandwidth, over tiles of 16 KiB of text
// (one workgroup of 256 threads, four 16-byte loads per thread):
//   count   per tile: letters, word starts (a letter whose previous byte is
//           not one), and the letters before its first and after its last
//           word start (from the positions of its first non-letter, last
//           letter and last start, so its loads are coalesced);
//   scan    one workgroup: exclusive prefix of letters and words over the
//           tiles, the totals, the closing offset, and the longest word
//           that reaches past a tile's end (tiles joined in text order);
//   write   per tile again, 64 consecutive bytes per thread (its letters
//           form one 64-bit mask): a block scan gives each thread its letter
//           and word ranks; letters and word starts are compacted through
//           LDS and stored in order (letters as aligned dwords), and the
//           longest word inside the tile is folded into the result.
// Three passes read the text twice, but no workgroup waits on another.  A
// single pass (each tile folding the counts its predecessors publish) has
// to poll across the eight XCDs, whose L2 caches are not coherent with each
// other: every poll goes past L2 and queues behind the text stream.  On a
// 188 MB text that single pass took 0.21-0.23 ms, these three 0.18 ms.
// The text pointer may have any alignment: tiles are laid over the text
// rounded down to 16 bytes, interior 16-byte chunks are read with one load,
// and chunks at either end byte by byte inside the text only.
#include "../../include/bsort.h"
#include "bsort_internal.h"

namespace bsort {
namespace {

constexpr int kTokThreads = 256;
constexpr int kTokBytes = 16;                          // bytes per load
constexpr int kTokLoads = 4;                           // loads per thread
constexpr int kTokSpan = kTokBytes * kTokLoads;        // 64 consecutive text bytes per thread
constexpr int kTokTile = kTokThreads * kTokSpan;       // 16 KiB of text per workgroup
constexpr int kTokWaves = kTokThreads / kWave;
// LDS staging of a tile in the write pass: its L letters from byte skew
// (0..3) on, then its W 16-bit word starts from the next dword on.  A word
// has a letter (W <= L), and word starts inside a tile are separated by
// non-letters (W - 1 <= 16384 - L), so L + 2W is largest at L = 8193,
// W = 8192 (24,577 bytes) and the starts end by byte 24,584.  Sized for that
// rather than for 16 KiB of each, so that six workgroups fit in a compute
// unit's LDS, not four.
constexpr int kTokStageBytes = 24584;
constexpr int kTokScanThreads = 1024;

inline size_t tok_align(size_t x) { return (x + 255) & ~size_t(255); }

struct TokText {
    const uint8_t* base;   // text rounded down to a multiple of 16 bytes
    int64_t head;          // text - base (0..15)
    int64_t N;             // head + n_bytes; positions [head, N) are text
};

// Bit 7 of each byte of the result is set iff that byte of x is an ASCII
// letter (the other bits are left as they fall).  x | 0x20 maps A-Z onto
// a-z (and nothing else onto a-z); with the top bit cleared, adding 0x1F to
// a byte sets its bit 7 iff it is at least 0x61 ('a'), adding 0x05 iff it is
// at least 0x7B (past 'z'), neither sum carries into the next byte, and the
// second implies the first, so their XOR marks a-z.  Bytes with the top bit
// set are never letters.
__device__ __forceinline__ uint32_t letter_bits(uint32_t x) {
    const uint32_t y = x | 0x20202020u;
    const uint32_t v = y & 0x7F7F7F7Fu;
    return ((v + 0x1F1F1F1Fu) ^ (v + 0x05050505u)) & ~y;
}

// letter_bits of two dwords a, b -> 8-bit mask, bits 0-3 for a's bytes and
// 4-7 for b's: a's flags moved to bits 0, 8, 16, 24 and b's to 4, 12, 20,
// 28, then one multiply by 2^24 + 2^17 + 2^10 + 2^3 carries flag i of each
// to bit 24 + i (a) and 28 + i (b); every other product term lands, alone,
// below bit 24 or above bit 31
__device__ __forceinline__ uint32_t byte_mask(uint32_t fa, uint32_t fb) {
    const uint32_t x = ((fa >> 7) & 0x01010101u) | ((fb >> 3) & 0x10101010u);
    return (x * 0x01020408u) >> 24;
}

__device__ __forceinline__ bool is_letter(uint32_t b) { return ((b | 0x20u) - 0x61u) < 26u; }

// text bytes at logical positions [c, c+16), little-endian in d; positions
// outside the text read as 0 (not a letter)
__device__ __forceinline__ void load_chunk(const TokText& t, int64_t c, uint32_t (&d)[4]) {
    const gptr<const uint8_t> b = gp(t.base);
    if (c >= t.head && c + kTokBytes <= t.N) {
        const gptr<const uint64_t> q = (gptr<const uint64_t>)(b + c);
        const uint64_t lo = q[0], hi = q[1];
        d[0] = (uint32_t)lo;
        d[1] = (uint32_t)(lo >> 32);
        d[2] = (uint32_t)hi;
        d[3] = (uint32_t)(hi >> 32);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) d[k] = 0;
        for (int j = 0; j < kTokBytes; ++j) {
            const int64_t p = c + j;
            if (p >= t.head && p < t.N) d[j >> 2] |= (uint32_t)b[p] << (8 * (j & 3));
        }
    }
}

// 64-bit letter mask M (bit j: byte c+j is a letter) and word-start mask S
// of the 64 text bytes at c
__device__ __forceinline__ void span_masks(const TokText& t, int64_t c,
                                           const uint32_t (&d)[kTokLoads][4], uint64_t& M,
                                           uint64_t& S) {
    M = 0;
#pragma unroll
    for (int k = 0; k < kTokLoads; ++k)
#pragma unroll
        for (int q = 0; q < 4; q += 2)
            M |= (uint64_t)byte_mask(letter_bits(d[k][q]), letter_bits(d[k][q + 1]))
                 << (16 * k + 4 * q);
    const int64_t p = c - 1;
    const uint64_t prev = (p >= t.head && p < t.N && is_letter(gp(t.base)[p])) ? 1u : 0u;
    S = M & ~((M << 1) | prev);
}

__device__ __forceinline__ void load_span(const TokText& t, int64_t c,
                                          uint32_t (&d)[kTokLoads][4]) {
#pragma unroll
    for (int k = 0; k < kTokLoads; ++k) load_chunk(t, c + kTokBytes * k, d[k]);
}

// per-thread counts packed as (word starts << 16) | letters; a tile's sums
// stay below 2^15 and 2^14
__device__ __forceinline__ uint32_t packed_counts(uint64_t M, uint64_t S) {
    return ((uint32_t)__popcll(S) << 16) | (uint32_t)__popcll(M);
}

// Letter runs of a stretch of text: pre = letters at its start, suf =
// letters at its end, mx = longest run inside, full = all letters (then
// pre = suf = mx = its length).  Joining stretches in text order is
// associative, so the longest word of the text is the mx of all of them
// joined, whatever the grouping.
template <typename T>
struct Run {
    T pre, suf, mx;
    bool full;
};

template <typename T>
__device__ __forceinline__ Run<T> join(const Run<T>& a, const Run<T>& b) {
    Run<T> r;
    r.full = a.full && b.full;
    r.pre = a.full ? a.pre + b.pre : a.pre;
    r.suf = b.full ? b.suf + a.suf : b.suf;
    const T m = a.mx > b.mx ? a.mx : b.mx;
    const T c = a.suf + b.pre;
    r.mx = m > c ? m : c;
    return r;
}

// wave-wide join in lane order; lane 0 ends with the wave's runs
template <typename T>
__device__ __forceinline__ Run<T> wave_join(Run<T> r, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        Run<T> o;
        o.pre = __shfl_down(r.pre, d, kWave);
        o.suf = __shfl_down(r.suf, d, kWave);
        o.mx = __shfl_down(r.mx, d, kWave);
        o.full = __shfl_down((int)r.full, d, kWave) != 0;
        if ((lane & (2 * d - 1)) == 0) r = join(r, o);
    }
    return r;
}

// wave-wide max
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        const uint32_t o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// tile_counts[i] = packed counts of tile i; tile_ends[i] = (letters of the
// tile after its last word start << 16) | letters before its first one
// (both 0 when the tile has no word start).
//
// Counting needs no text order inside the tile, so the loads are laid out
// for coalescing: load k of thread t reads bytes k * 4096 + 16t .. +15 of
// the tile (a wave's load is 1 KiB of consecutive text).  A 16-byte chunk's
// previous byte is the last byte of the previous lane's chunk, or, for lane
// 0, read from memory.  The two run lengths come from positions:
//   letters before the first word start: if the byte before the tile is a
//     letter, the tile's leading letters continue a word and end at its
//     first non-letter, so they number that non-letter's position; else 0;
//   letters from the last word start on: the last start opens the tile's
//     last run of letters, so last letter's position + 1 - last start's.
__global__ __launch_bounds__(kTokThreads) void k_tok_count(TokText t, int64_t ntiles,
                                                           uint32_t* __restrict__ tile_counts,
                                                           uint32_t* __restrict__ tile_ends) {
    constexpr int kRow = kTokThreads * kTokBytes;      // 4 KiB of text per load round
    __shared__ uint32_t wsum[kTokWaves], wnon[kTokWaves], wlet[kTokWaves], wst[kTokWaves];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * kTokTile;
    uint32_t d[kTokLoads][4];
#pragma unroll
    for (int k = 0; k < kTokLoads; ++k) load_chunk(t, base + k * kRow + kTokBytes * tid, d[k]);
    // lane 0: the byte before each of its chunks
    uint32_t before0 = 0;
    if (lane == 0) {
        const gptr<const uint8_t> tb = gp(t.base);
#pragma unroll
        for (int k = 0; k < kTokLoads; ++k) {
            const int64_t p = base + k * kRow + kTokBytes * tid - 1;
            if (p >= t.head && p < t.N && is_letter(tb[p])) before0 |= 1u << k;
        }
    }
    uint32_t sum = 0;                                  // (word starts << 16) | letters
    uint32_t non = 0xFFFFFFFFu, let = 0, st = 0;       // first non-letter, last letter + 1, last start + 1
#pragma unroll
    for (int k = 0; k < kTokLoads; ++k) {
        const uint32_t m = byte_mask(letter_bits(d[k][0]), letter_bits(d[k][1])) |
                           byte_mask(letter_bits(d[k][2]), letter_bits(d[k][3])) << 8;
        const uint32_t up = (uint32_t)__shfl_up((int)(m >> 15), 1, kWave);
        const uint32_t prev = lane == 0 ? (before0 >> k) & 1u : up & 1u;
        const uint32_t sm = m & ~((m << 1) | prev) & 0xFFFFu;
        sum += ((uint32_t)__popc(sm) << 16) | (uint32_t)__popc(m);
        const uint32_t pos = (uint32_t)(k * kRow + kTokBytes * tid);
        const uint32_t nm = ~m & 0xFFFFu;
        if (nm) non = min(non, pos + (uint32_t)__builtin_ctz(nm));
        if (m) let = max(let, pos + 32u - (uint32_t)__builtin_clz(m));
        if (sm) st = max(st, pos + 32u - (uint32_t)__builtin_clz(sm));
    }
    // wave sums and extremes, then the tile's
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sum += (uint32_t)__shfl_xor((int)sum, o, kWave);
        non = min(non, (uint32_t)__shfl_xor((int)non, o, kWave));
        let = max(let, (uint32_t)__shfl_xor((int)let, o, kWave));
        st = max(st, (uint32_t)__shfl_xor((int)st, o, kWave));
    }
    if (lane == 0) {
        wsum[wv] = sum;
        wnon[wv] = non;
        wlet[wv] = let;
        wst[wv] = st;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t total = 0, fn = 0xFFFFFFFFu, ll = 0, ls = 0;
#pragma unroll
        for (int w = 0; w < kTokWaves; ++w) {
            total += wsum[w];
            fn = min(fn, wnon[w]);
            ll = max(ll, wlet[w]);
            ls = max(ls, wst[w]);
        }
        const int64_t p = base - 1;
        const bool cont = p >= t.head && p < t.N && is_letter(gp(t.base)[p]);
        const uint32_t pre = cont ? (fn == 0xFFFFFFFFu ? (uint32_t)kTokTile : fn) : 0u;
        const bool any = (total >> 16) != 0;
        gp(tile_counts)[tile] = total;
        gp(tile_ends)[tile] = any ? ((ll - (ls - 1)) << 16) | pre : 0u;
    }
}

// Exclusive prefix of (letters, words) over the tiles: each thread takes a
// contiguous stretch of tiles, one block scan across threads, then each
// thread writes its stretch's prefixes.  tile_base[2i] = letters before
// tile i, [2i+1] = words before it.
//
// Words that reach past a tile's end, as runs joined in text order: a tile
// with word starts is the run (letters before its first start, letters from
// its last start on), one without is all continuation (pre = suf = its
// letters, full), so the join of a tile's suf with the following pre is the
// length of the word crossing there; the text's last word is the suf of all.
__global__ __launch_bounds__(kTokScanThreads) void k_tok_scan(
    const uint32_t* __restrict__ tile_counts, const uint32_t* __restrict__ tile_ends,
    int64_t ntiles, int64_t* __restrict__ tile_base, int64_t* __restrict__ offsets,
    int64_t cap_words, int64_t* __restrict__ result) {
    constexpr int NW = kTokScanThreads / kWave;
    __shared__ int64_t wl[NW], ww[NW];
    __shared__ int64_t wr[NW][3];
    __shared__ int wf[NW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t per = (ntiles + kTokScanThreads - 1) / kTokScanThreads;
    const int64_t a = (int64_t)tid * per;
    const int64_t b = a + per < ntiles ? a + per : ntiles;
    const gptr<const uint32_t> tc = gp(tile_counts);
    const gptr<const uint32_t> te = gp(tile_ends);
    int64_t sl = 0, sw = 0;
    Run<int64_t> run{0, 0, 0, true};
#pragma unroll 8
    for (int64_t i = a; i < b; ++i) {
        const uint32_t v = tc[i], e = te[i];
        const int64_t nl = v & 0xFFFFu;
        sl += nl;
        sw += v >> 16;
        const bool any = (v >> 16) != 0;
        run = join(run, Run<int64_t>{any ? (int64_t)(e & 0xFFFFu) : nl,
                                     any ? (int64_t)(e >> 16) : nl, 0, !any});
    }
    const int64_t il = wave_incl_scan(sl, lane), iw = wave_incl_scan(sw, lane);
    run = wave_join(run, lane);
    if (lane == 63) {
        wl[wv] = il;
        ww[wv] = iw;
    }
    if (lane == 0) {
        wr[wv][0] = run.pre;
        wr[wv][1] = run.suf;
        wr[wv][2] = run.mx;
        wf[wv] = run.full ? 1 : 0;
    }
    __syncthreads();
    int64_t bl = il - sl, bw = iw - sw, tl = 0, tw = 0;
    for (int k = 0; k < NW; ++k) {
        if (k < wv) {
            bl += wl[k];
            bw += ww[k];
        }
        tl += wl[k];
        tw += ww[k];
    }
    const gptr<int64_t> tb = gp(tile_base);
#pragma unroll 8
    for (int64_t i = a; i < b; ++i) {
        const uint32_t v = tc[i];
        tb[2 * i] = bl;
        tb[2 * i + 1] = bw;
        bl += v & 0xFFFFu;
        bw += v >> 16;
    }
    if (tid == 0) {
        Run<int64_t> all{0, 0, 0, true};
        for (int k = 0; k < NW; ++k)
            all = join(all, Run<int64_t>{wr[k][0], wr[k][1], wr[k][2], wf[k] != 0});
        const gptr<int64_t> r = gp(result);
        r[0] = tw;
        r[1] = tl;
        r[2] = all.mx > all.suf ? all.mx : all.suf;
        r[3] = tw > cap_words ? BSORT_E_CAPACITY : BSORT_OK;
        if (tw <= cap_words) gp(offsets)[tw] = tl;
    }
}

__global__ __launch_bounds__(kTokThreads) void k_tok_write(TokText t,
                                                           const int64_t* __restrict__ tile_base,
                                                           uint8_t* __restrict__ out,
                                                           int64_t* __restrict__ offsets,
                                                           int64_t cap_words,
                                                           int64_t* __restrict__ result) {
    // the tile's letters, placed at (global letter address mod 4) + rank so
    // that aligned global dwords are aligned LDS dwords, then its word starts
    // as 16-bit letter ranks within the tile from the next dword on, both
    // stored out in order at the end (+ one dword per lane past the end:
    // every byte of a span is stored, non-letters to their lane's spare
    // dword, so the staging has no branch)
    __shared__ uint32_t stage32[kTokStageBytes / 4 + kWave];
    __shared__ uint32_t wmax[kTokWaves];
    __shared__ uint32_t wsum[kTokWaves];
    uint8_t* stage = (uint8_t*)stage32;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t c = tile * kTokTile + (int64_t)tid * kTokSpan;
    uint32_t d[kTokLoads][4];
    load_span(t, c, d);
    uint64_t M, S;
    span_masks(t, c, d, M, S);
    const uint32_t v = packed_counts(M, S);
    const uint32_t incl = wave_incl_scan(v, lane);
    if (lane == 63) wsum[wv] = incl;
    const gptr<const int64_t> tb = gp(tile_base);
    const int64_t lb = tb[2 * tile], wb = tb[2 * tile + 1];
    const int skew = (int)(((uintptr_t)out + (uint64_t)lb) & 3u);
    __syncthreads();
    uint32_t before = incl - v, total = 0;
#pragma unroll
    for (int w = 0; w < kTokWaves; ++w) {
        before += w < wv ? wsum[w] : 0u;
        total += wsum[w];
    }
    const int ll = (int)(before & 0xFFFFu);           // letters of the tile before this thread
    const int nl = (int)(total & 0xFFFFu);
    uint16_t* wstart = (uint16_t*)(stage + ((skew + nl + 3) & ~3));
    // letters, compacted in order into LDS
    int pos = skew + ll;
    const int spare = kTokStageBytes + 4 * lane;
#pragma unroll
    for (int k = 0; k < kTokLoads; ++k)
#pragma unroll
        for (int j = 0; j < kTokBytes; ++j) {
            const int bit = (int)((M >> (kTokBytes * k + j)) & 1u);
            stage[bit ? pos : spare] = (uint8_t)(d[k][j >> 2] >> (8 * (j & 3)));
            pos += bit;
        }
    // word starts: letter rank of each one's first letter
    uint64_t sm = S;
    int w = (int)(before >> 16);                      // word starts of the tile before it
    while (sm) {
        const int j = __builtin_ctzll(sm);
        wstart[w++] = (uint16_t)(ll + __popcll(M & ((1ull << j) - 1ull)));
        sm &= sm - 1ull;
    }
    __syncthreads();
    // word offsets, coalesced: offsets[wb + i] = lb + rank of word i's first letter
    const int nw = (int)(total >> 16);
    const gptr<int64_t> off = gp(offsets) + wb;
    const int64_t room = cap_words - wb;
    uint32_t inner = 0;                                // longest word inside the tile
    for (int i = tid; i < nw; i += kTokThreads) {
        const uint32_t a = wstart[i];
        if (i < room) off[i] = lb + (int64_t)a;
        if (i + 1 < nw) {
            const uint32_t len = (uint32_t)wstart[i + 1] - a;
            inner = len > inner ? len : inner;
        }
    }
    inner = wave_max(inner);
    if (lane == 0) wmax[wv] = inner;
    // letters [lb, lb + nl): the partial dwords at both ends byte by byte,
    // the rest as aligned dwords
    const gptr<uint8_t> o = gp(out) + lb;             // o - skew is 4-byte aligned
    const int first = skew ? 4 - skew : 0;             // bytes before the first aligned dword
    if (tid < first && tid < nl) o[tid] = stage[skew + tid];
    const int body = nl > first ? (nl - first) >> 2 : 0;
    const gptr<uint32_t> o32 = (gptr<uint32_t>)(o + first);
    const int s32 = (skew + first) >> 2;               // LDS dword of the first aligned one
    for (int i = tid; i < body; i += kTokThreads) o32[i] = stage32[s32 + i];
    const int tail0 = first + 4 * body;
    if (tid < nl - tail0 && tail0 + tid >= first) o[tail0 + tid] = stage[skew + tail0 + tid];
    __syncthreads();
    if (tid == 0) {
        uint32_t m = 0;
#pragma unroll
        for (int w = 0; w < kTokWaves; ++w) m = wmax[w] > m ? wmax[w] : m;
        // one address for every tile: look first, so that the atomic (which
        // serialises) only runs when this tile raises the maximum
        const gptr<int64_t> r2 = gp(result) + 2;
        if ((int64_t)m > __hip_atomic_load(r2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            __hip_atomic_fetch_max(r2, (int64_t)m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

int64_t tok_tiles(int64_t logical_bytes) { return (logical_bytes + kTokTile - 1) / kTokTile; }

}  // namespace

size_t tok_workspace_bytes(int64_t n_bytes) {
    const int64_t nt = tok_tiles(n_bytes + 15);
    return 2 * tok_align(sizeof(uint32_t) * (size_t)nt) +
           tok_align(2 * sizeof(int64_t) * (size_t)nt) + 256;
}

hipError_t launch_tokenize(const uint8_t* text, int64_t n_bytes, uint8_t* out, int64_t* offsets,
                           int64_t cap_words, int64_t* result, void* ws, hipStream_t s) {
    TokText t;
    const uintptr_t p = (uintptr_t)text;
    t.base = (const uint8_t*)(p & ~(uintptr_t)15);
    t.head = (int64_t)(p & 15);
    t.N = t.head + n_bytes;
    const int64_t nt = n_bytes > 0 ? tok_tiles(t.N) : 0;
    char* w = (char*)ws;
    uint32_t* tc = (uint32_t*)w;
    w += tok_align(sizeof(uint32_t) * (size_t)nt);
    uint32_t* te = (uint32_t*)w;
    w += tok_align(sizeof(uint32_t) * (size_t)nt);
    int64_t* tb = (int64_t*)w;
    if (nt > 0)
        k_tok_count<<<(unsigned)nt, kTokThreads, 0, s>>>(t, nt, tc, te);
    k_tok_scan<<<1, kTokScanThreads, 0, s>>>(tc, te, nt, tb, offsets, cap_words, result);
    if (nt > 0)
        k_tok_write<<<(unsigned)nt, kTokThreads, 0, s>>>(t, tb, out, offsets, cap_words, result);
    return hipGetLastError();
}

}  // namespace bsort
