// Pre-processing (Section II, phase 1; Section III, approach one step 2):
// raw text to words.  The paper drops "special characters" (its examples are
// quote, comma, full stop, question and exclamation marks) before splitting
// the text into words; here a word is a maximal run of ASCII letters
// [A-Za-z] and every other byte separates words and is dropped.  The words
// come out in the library's input format: their letters back to back and
// int64 offsets, word i = out[offsets[i] .. offsets[i+1]).
//
// A stream compaction bound by HBM bandwidth, over tiles of 16 KiB of text
// (one workgroup of 256 threads, 64 consecutive bytes per thread read with
// four 16-byte loads; a thread's letters form one 64-bit mask):
//   count   per tile: letters, word starts (a letter whose previous byte is
//           not one), and the letter runs at its two ends and inside it;
//   scan    one workgroup: exclusive prefix of letters and words over the
//           tiles, the totals, the closing offset, and the longest word
//           (the runs of all tiles joined in order);
//   write   per tile again: block scans give each thread its letter and
//           word ranks; letters and word starts are compacted through LDS
//           and stored in order (letters as aligned dwords).
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
constexpr int kTokScanThreads = 1024;

inline size_t tok_align(size_t x) { return (x + 255) & ~size_t(255); }

struct TokText {
    const uint8_t* base;   // text rounded down to a multiple of 16 bytes
    int64_t head;          // text - base (0..15)
    int64_t N;             // head + n_bytes; positions [head, N) are text
};

// Bit 7 of each byte of the result is set iff that byte of x is an ASCII
// letter.  x | 0x20 maps A-Z onto a-z (and nothing else onto a-z); with the
// top bit cleared, adding 0x1F to a byte sets its bit 7 iff it is at least
// 0x61 ('a'), adding 0x05 iff it is at least 0x7B (past 'z'), and neither
// sum carries into the next byte.  Bytes with the top bit set are never
// letters.
__device__ __forceinline__ uint32_t letter_bits(uint32_t x) {
    const uint32_t y = x | 0x20202020u;
    const uint32_t v = y & 0x7F7F7F7Fu;
    return (v + 0x1F1F1F1Fu) & ~(v + 0x05050505u) & ~y & 0x80808080u;
}

// letter_bits result -> 4-bit mask, bit i for byte i: the four flags moved
// to bit 0 of their bytes and multiplied so that they land, without carries,
// in bits 28..31
__device__ __forceinline__ uint32_t nibble_mask(uint32_t f) {
    return (((f >> 7) & 0x01010101u) * 0x10204080u) >> 28;
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
        for (int q = 0; q < 4; ++q)
            M |= (uint64_t)nibble_mask(letter_bits(d[k][q])) << (16 * k + 4 * q);
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

// the runs of 64 text bytes from their letter mask.  Longest run: x[k] has
// bit i set iff the 2^k bytes ending at i are letters (x[k] = x[k-1] &
// x[k-1] << 2^(k-1)); the length is then found bit by bit from the top,
// keeping the positions where a run of the length so far ends.
__device__ __forceinline__ Run<uint32_t> span_run(uint64_t M) {
    Run<uint32_t> r;
    r.full = M == ~0ull;
    r.pre = r.full ? 64u : (uint32_t)__builtin_ctzll(~M);
    r.suf = r.full ? 64u : (uint32_t)__builtin_clzll(~M);
    uint64_t x[7];
    x[0] = M;
#pragma unroll
    for (int k = 1; k < 7; ++k) x[k] = x[k - 1] & (x[k - 1] << (1 << (k - 1)));
    uint32_t L = 0;
    uint64_t cur = ~0ull;
#pragma unroll
    for (int k = 6; k >= 0; --k) {
        const uint64_t tk = cur & (L < 64 ? x[k] << L : 0ull);
        const bool hit = tk != 0;
        cur = hit ? tk : cur;
        L += hit ? (1u << k) : 0u;
    }
    r.mx = L;
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

// the same for the runs of 64-byte spans: every length within a wave is at
// most 4096, so (pre, suf) and (mx, full) travel as two 32-bit values
__device__ __forceinline__ Run<uint32_t> wave_join_spans(Run<uint32_t> r, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t ps = __shfl_down(r.pre | (r.suf << 16), d, kWave);
        const uint32_t mf = __shfl_down(r.mx | (r.full ? 0x10000u : 0u), d, kWave);
        const Run<uint32_t> o{ps & 0xFFFFu, ps >> 16, mf & 0xFFFFu, (mf >> 16) != 0};
        if ((lane & (2 * d - 1)) == 0) r = join(r, o);
    }
    return r;
}

// a tile's runs packed into 64 bits: pre, suf, mx (each <= 16384) and full
__device__ __forceinline__ uint64_t pack_run(const Run<uint32_t>& r) {
    return (uint64_t)r.pre | ((uint64_t)r.suf << 16) | ((uint64_t)r.mx << 32) |
           ((uint64_t)(r.full ? 1 : 0) << 48);
}
__device__ __forceinline__ Run<int64_t> unpack_run(uint64_t v) {
    Run<int64_t> r;
    r.pre = (int64_t)(v & 0xFFFFu);
    r.suf = (int64_t)((v >> 16) & 0xFFFFu);
    r.mx = (int64_t)((v >> 32) & 0xFFFFu);
    r.full = ((v >> 48) & 1u) != 0;
    return r;
}

// tile_counts[i] = packed counts of tile i; tile_runs[i] = its packed runs
__global__ __launch_bounds__(kTokThreads) void k_tok_count(TokText t,
                                                           uint32_t* __restrict__ tile_counts,
                                                           uint64_t* __restrict__ tile_runs) {
    __shared__ uint32_t wsum[kTokWaves];
    __shared__ uint32_t wrun[kTokWaves][4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t c = tile * kTokTile + (int64_t)tid * kTokSpan;
    uint32_t d[kTokLoads][4];
    load_span(t, c, d);
    uint64_t M, S;
    span_masks(t, c, d, M, S);
    const uint32_t incl = wave_incl_scan(packed_counts(M, S), lane);
    const Run<uint32_t> r = wave_join_spans(span_run(M), lane);
    if (lane == 63) wsum[wv] = incl;
    if (lane == 0) {
        wrun[wv][0] = r.pre;
        wrun[wv][1] = r.suf;
        wrun[wv][2] = r.mx;
        wrun[wv][3] = r.full ? 1u : 0u;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t s = 0;
        Run<uint32_t> acc{0, 0, 0, true};                      // the empty stretch
#pragma unroll
        for (int w = 0; w < kTokWaves; ++w) {
            s += wsum[w];
            acc = join(acc, Run<uint32_t>{wrun[w][0], wrun[w][1], wrun[w][2], wrun[w][3] != 0});
        }
        gp(tile_counts)[tile] = s;
        gp(tile_runs)[tile] = pack_run(acc);
    }
}

// Exclusive prefix of (letters, words) over the tiles and the runs of all
// tiles joined: each thread takes a contiguous stretch of tiles, one block
// scan (and join) across threads, then each thread writes its stretch's
// prefixes.  tile_base[2i] = letters before tile i, [2i+1] = words before it.
__global__ __launch_bounds__(kTokScanThreads) void k_tok_scan(
    const uint32_t* __restrict__ tile_counts, const uint64_t* __restrict__ tile_runs,
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
    const gptr<const uint64_t> tr = gp(tile_runs);
    int64_t sl = 0, sw = 0;
    Run<int64_t> run{0, 0, 0, true};
#pragma unroll 8
    for (int64_t i = a; i < b; ++i) {
        const uint32_t v = tc[i];
        sl += v & 0xFFFFu;
        sw += v >> 16;
        run = join(run, unpack_run(tr[i]));
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
        r[2] = all.mx;
        r[3] = tw > cap_words ? BSORT_E_CAPACITY : BSORT_OK;
        if (tw <= cap_words) gp(offsets)[tw] = tl;
    }
}

__global__ __launch_bounds__(kTokThreads) void k_tok_write(TokText t,
                                                           const int64_t* __restrict__ tile_base,
                                                           uint8_t* __restrict__ out,
                                                           int64_t* __restrict__ offsets,
                                                           int64_t cap_words) {
    // the tile's letters, placed at (global letter address mod 4) + rank so
    // that aligned global dwords are aligned LDS dwords, and its word starts
    // as letter ranks within the tile, both stored out in order at the end
    __shared__ uint32_t stage32[kTokTile / 4 + 2];
    __shared__ uint32_t wstart[kTokTile / 2];
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
    // letters, compacted in order into LDS
    int pos = skew + ll;
#pragma unroll
    for (int k = 0; k < kTokLoads; ++k)
#pragma unroll
        for (int j = 0; j < kTokBytes; ++j) {
            if ((M >> (kTokBytes * k + j)) & 1u)
                stage[pos++] = (uint8_t)(d[k][j >> 2] >> (8 * (j & 3)));
        }
    // word starts: letter rank of each one's first letter
    uint64_t sm = S;
    int w = (int)(before >> 16);                      // word starts of the tile before it
    while (sm) {
        const int j = __builtin_ctzll(sm);
        wstart[w++] = (uint32_t)(ll + __popcll(M & ((1ull << j) - 1ull)));
        sm &= sm - 1ull;
    }
    __syncthreads();
    // word offsets, coalesced: offsets[wb + i] = lb + rank of word i's first letter
    const int nw = (int)(total >> 16);
    const gptr<int64_t> off = gp(offsets) + wb;
    const int64_t room = cap_words - wb;
    for (int i = tid; i < nw; i += kTokThreads)
        if (i < room) off[i] = lb + (int64_t)wstart[i];
    // letters [lb, lb + nl): the partial dwords at both ends byte by byte,
    // the rest as aligned dwords
    const int nl = (int)(total & 0xFFFFu);
    const gptr<uint8_t> o = gp(out) + lb;             // o - skew is 4-byte aligned
    const int first = skew ? 4 - skew : 0;             // bytes before the first aligned dword
    if (tid < first && tid < nl) o[tid] = stage[skew + tid];
    const int body = nl > first ? (nl - first) >> 2 : 0;
    const gptr<uint32_t> o32 = (gptr<uint32_t>)(o + first);
    const int s32 = (skew + first) >> 2;               // LDS dword of the first aligned one
    for (int i = tid; i < body; i += kTokThreads) o32[i] = stage32[s32 + i];
    const int tail0 = first + 4 * body;
    if (tid < nl - tail0 && tail0 + tid >= first) o[tail0 + tid] = stage[skew + tail0 + tid];
}

int64_t tok_tiles(int64_t logical_bytes) { return (logical_bytes + kTokTile - 1) / kTokTile; }

}  // namespace

size_t tok_workspace_bytes(int64_t n_bytes) {
    const int64_t nt = tok_tiles(n_bytes + 15);
    return tok_align(sizeof(uint32_t) * (size_t)nt) + tok_align(sizeof(uint64_t) * (size_t)nt) +
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
    uint64_t* tr = (uint64_t*)w;
    w += tok_align(sizeof(uint64_t) * (size_t)nt);
    int64_t* tb = (int64_t*)w;
    if (nt > 0) k_tok_count<<<(unsigned)nt, kTokThreads, 0, s>>>(t, tc, tr);
    k_tok_scan<<<1, kTokScanThreads, 0, s>>>(tc, tr, nt, tb, offsets, cap_words, result);
    if (nt > 0) k_tok_write<<<(unsigned)nt, kTokThreads, 0, s>>>(t, tb, out, offsets, cap_words);
    return hipGetLastError();
}

}  // namespace bsort
