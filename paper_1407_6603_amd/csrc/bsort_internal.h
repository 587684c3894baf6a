// Internal definitions shared by the HIP translation units of libbsort.
//
// Data layout in HBM (all in the caller's workspace unless noted):
//   - A "job" descriptor holds every pointer and size a launch needs.  It is
//     written on the device by k_set_job from a by-value kernel argument, so
//     a captured graph can be replayed on new buffers by re-running only that
//     one small launch.
//   - A sub-array ("bucket") is (request r, length L).  Its words sit at
//     positions req_start[r] + starts[r][L] + j, j < counts[r][L], in order,
//     perm and the key lanes.
//   - Key lanes are SoA per bucket: lane w of bucket word j is
//     keys[key_off[r][L] + w * n_b + j], W = ceil(L/8) uint64 lanes, first
//     byte in the most significant position, zero padded.
//   - In registers a word is a "record" of D = ceil(L/4) + 1 dwords: the
//     ceil(L/4) big-endian key dwords then the list-local word index.  When
//     ceil(L/4) is odd the index takes the low dword of the last lane, which
//     is zero padding for such lengths.  Records compare lexicographically as
//     unsigned dwords, so (bytes, index) order is a total order and every
//     correct schedule gives the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "merge_sched.h"

namespace bsort {

// Views of pointers as global memory.  Pointers read from the job
// descriptor are generic to the compiler, which then emits flat loads and
// stores; flat operations also count against the LDS wait counter, so a
// kernel mixing them with LDS work waits for both at once.  Hot loops read
// and write through these views instead.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> gp(T* p) {
    return (gptr<T>)p;
}

constexpr int kMaxLen = 64;
constexpr int kMaxD = 17;                 // ceil(64/4) + 1
constexpr int kNumD = kMaxD + 1;          // arrays indexed by D directly
constexpr int kWave = 64;
constexpr int kChunkRounds = 16;
constexpr int kChunk = kWave * kChunkRounds;   // words per bucketize chunk
constexpr int kTileWavesPerBlock = 4;
constexpr int kMinTile = 128;             // 64 lanes x 2 records
constexpr int kFlagTilesOnly = 2;         // same value as BSORT_FLAG_TILES_ONLY
constexpr int kFlagLdsTile = 16;          // same value as BSORT_FLAG_LDS_TILE
// Job.flags: leave the status word as it is
constexpr int kJobKeepStatus = 1 << 8;
// Job.flags: the scatter by length also packs each word's key lanes and index
// payload at its place in the sub-array (batched form; order is not written)
constexpr int kJobFusedPack = 1 << 9;
constexpr int kMaxPhaseCap = 1 << 22;

// device status bits (workspace status word)
enum : uint32_t {
    ST_BAD_OFFSETS = 1u,
    ST_TOO_LONG = 2u,
    ST_BAD_REQ = 4u,
    ST_OVERFLOW = 8u,      // an internal list bound was exceeded (a library bug)
    ST_STALLED = 16u,      // a bounded wait of the merge-split launch gave up (a library bug)
};

// In-LDS sub-arrays: one workgroup holds a whole sub-array of up to
// lds_cap(c, D) words in LDS (D dwords per word, at most 144 KiB) and sorts
// it there.  Size classes c = 0..4; the largest class is sized per width D.
// The largest two-dword class holds 16,320 words (255 rows of 64): its two
// dword planes then lie 255 x 256 bytes apart, within reach of one
// ds_read2st64_b32 / ds_write2st64_b32, so a whole record moves in one LDS
// instruction (at 16,384 words the second plane is one step too far).
constexpr int kLdsClasses = 5;
constexpr int kLdsMaxD = 9;
constexpr int kLdsBytes = 144 * 1024;
__host__ __device__ constexpr int lds_cap(int c, int D) {
    return c < 4 ? (1024 << c) : (D <= 2 ? 16320 : D == 3 ? 12288 : D == 4 ? 9216 : 7168);
}
__host__ __device__ constexpr bool lds_fits(int D, int c) {
    return D >= 2 && D <= kLdsMaxD && D * 4 * lds_cap(c, D) <= kLdsBytes;
}
// Sub-arrays of class c hold more than this many words: the next smaller
// class's capacity, else the single-tile size.  A class's list holds its
// larger sub-arrays (above a quarter of the way from this floor to the
// capacity) first, so that workgroups taking entries in list order start
// the longest sorts early and end together.
__host__ __device__ constexpr int lds_class_floor(int c, int D, int tile) {
    return c > 0 && lds_cap(c - 1, D) > tile ? lds_cap(c - 1, D) : tile;
}
__host__ __device__ constexpr bool lds_class_large(int n, int c, int D, int tile) {
    return n > lds_class_floor(c, D, tile) + (lds_cap(c, D) - lds_class_floor(c, D, tile)) / 4;
}
// threads per workgroup: 1024 only where the staged merge outputs still fit
// the 128 VGPRs a 1024-thread workgroup leaves each lane (D <= 3) and LDS
// holds one workgroup per CU anyway; 512 for two-dword records up to 8192
// words, so two workgroups share a CU
__host__ __device__ constexpr int lds_threads(int c, int D) {
    return c <= 1 ? 256 : (c <= 3 && D <= 2) || c == 2 || D >= 4 ? 512 : 1024;
}
constexpr int kLdsMaxTile = 512;          // tiles inside an LDS sub-array: K <= 8
// tile size inside an in-LDS sub-array of class capacity cap when the tiles
// are merged.  Two-dword records sort their tiles with exact fp64 min/max
// (two instructions per compare-exchange), so they take the largest tile;
// wider records double the tuned tile until at most 16 merge-split phases
// remain.  Always a power of two, at most kLdsMaxTile.
__host__ __device__ constexpr int lds_tile(int tuned, int cap, int D) {
    const int target = D <= 2 ? kLdsMaxTile : cap / 16;
    int t = tuned;
    while (t < target && t < kLdsMaxTile) t <<= 1;
    return t;
}

// Sub-arrays merged through HBM: tiles of the largest power of two C whose
// pair (2C records of 4D bytes) fits the LDS budget, at most 8192 words;
// records wider than kLdsMaxD dwords keep register-sized tiles (set on the
// host).  hbm_pair_cap(D) = 2C is the pair merge's LDS capacity in records.
__host__ __device__ constexpr int hbm_chunk_max(int D) {
    int c = 8192;
    while (c > 128 && 2 * c * 4 * D > kLdsBytes - 2048) c >>= 1;   // (room for the window table)
    return c;
}
// in-LDS class that sorts chunks of up to C words of width D (-1: none)
__host__ __device__ constexpr int hbm_chunk_class(int D, int C) {
    for (int c = 0; c < kLdsClasses; ++c)
        if (lds_fits(D, c) && lds_cap(c, D) >= C) return c;
    return -1;
}

// records per lane limit by key width: D * K <= 128 VGPRs of record state
__host__ __device__ constexpr int kmax_for(int D) {
    return D <= 2 ? 64 : D <= 4 ? 32 : D <= 8 ? 16 : D <= 16 ? 8 : 4;
}
__host__ __device__ constexpr int dwords_for_len(int L) { return (L + 3) / 4 + 1; }
__host__ __device__ constexpr int lanes_for_len(int L) { return (L + 7) / 8; }
// merge-split work items of a sub-array of p tiles: ceil(p/2) even phases of
// floor(p/2) pairs and floor(p/2) odd phases of floor((p-1)/2) pairs
__host__ __device__ constexpr int64_t merge_items_for(int64_t p) {
    return ((p + 1) / 2) * (p / 2) + (p / 2) * ((p - 1) / 2);
}

struct TileDesc {            // one odd-even transposition tile
    int64_t pos0;            // global position of the bucket's first word
    int64_t key_off;         // uint64 index of the bucket's lane 0
    int32_t n_b;             // words in the bucket
    int32_t t0;              // first bucket word of this tile
    int32_t n;               // words in this tile
    int32_t L;               // word length
};

struct LBucket {             // a sub-array (or a chunk of one) sorted entirely in LDS
    int64_t pos0;            // global position of the first word
    int64_t key_off;         // uint64 index of the first word's lane 0
    int32_t n_b;             // words
    int32_t L;               // word length
    int32_t stride;          // lane stride of the key layout (the whole sub-array's size)
    int32_t wk;              // nonzero: write the sorted keys back (a chunk merged later)
};

struct MSub {                // a sub-array merged through HBM (batched form)
    int64_t pos0;            // global position of its first word
    int64_t key_off;         // uint64 index of its lane 0
    int64_t tile_base;       // its tiles' entries in the tile phase table
    int32_t n_b;             // words
    int32_t L;               // word length
    int32_t T;               // tile size (a power of two)
    int32_t p;               // tiles, >= 2
};

struct Job {
    // inputs
    const uint8_t* bytes;
    int64_t n_bytes;
    const int64_t* offsets;
    const int64_t* req_start;    // [R+1]
    int64_t total;
    int32_t R;
    int32_t max_len;
    int32_t ml1;                 // max_len + 1 (lengths 0..max_len)
    int32_t flags;
    // bucketize outputs (caller buffers or workspace)
    int32_t* counts;             // [R * ml1]
    int32_t* starts;             // [R * (ml1 + 1)]
    int32_t* order;              // [total]
    int32_t* perm;               // [total]
    // workspace
    uint32_t* status;            // [1]
    int64_t* chunk_begin;        // [R + 1]
    int32_t* chunk_list;         // [chunk_cap] list of each chunk (R > 1)
    int32_t* chunk_hist;         // [chunk_cap * ml1], scanned in place
    uint8_t* len8;               // [total] each word's length (0xFF: malformed or too long)
    int64_t chunk_cap;
    int64_t* key_off;            // [R * ml1]
    uint64_t* keys;              // [wmax * total]
    TileDesc* tiles[kNumD];      // per record width D
    int64_t tile_cap[kNumD];
    int32_t tile_keys[kNumD];    // tile size per D: single tiles and in-LDS sub-arrays
    int32_t hbm_tile_keys[kNumD];  // tile size of sub-arrays merged through HBM
    int32_t* tile_count;         // [kNumD]
    // per class list: the larger sub-arrays from the front (lb_count of
    // them), the smaller from the back (lb_back, in reverse); the class
    // kernel's workgroups take list entries in that order through lb_take
    LBucket* lbuckets;           // [kNumD * kLdsClasses][lb_cap]
    int32_t* lb_count;           // [kNumD * kLdsClasses]
    int32_t* lb_back;            // [kNumD * kLdsClasses]
    int32_t* lb_take;            // [kNumD * kLdsClasses]
    int64_t lb_cap;
    // chunks of sub-arrays merged through HBM, sorted in LDS first (D <= kLdsMaxD)
    LBucket* hchunks[kLdsMaxD + 1];   // [tile_cap[D]] each
    int32_t* hc_count;           // [kLdsMaxD + 1]
    int32_t* pmax;               // [1] most merge-split phases any sub-array needs
    // merge-split through HBM in one launch (the order is described in merge_sched.h)
    MSub* msub;                  // [msub_cap] as planned
    MSub* msorted;               // [msub_cap] in order of decreasing tile count
    int64_t msub_cap;
    int32_t* mcounts;            // [0] sub-arrays, [1] tiles in msub
    int32_t* tile_ph;            // [mtile_cap] phases done on each tile
    int64_t mtile_cap;
    int32_t* pcnt;               // [phase_cap + 2] sub-arrays per tile count
    int32_t* pfill;              // [phase_cap + 2] scatter cursors
    int32_t* active;             // [phase_cap + 2] sub-arrays with more than s tiles
    int64_t* pe;                 // [msub_cap + 1]
    int64_t* po;                 // [msub_cap + 1]
    int64_t* ps;                 // [phase_cap + 1]
    int64_t* mhead;              // [0] next item to take, [1] items in all, [2] items done
    int64_t stall_ticks;         // bound on one wait of the merge launch, in ticks of the
                                 // 100 MHz counter (< 0: give up at once)
    int32_t phase_cap;
    int64_t rs_inline[2];        // req_start storage for single-list calls
    int64_t cb_inline[2];        // chunk_begin storage for the plain form's per-list jobs
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void set_status(const Job* J, uint32_t bit) {
    __hip_atomic_fetch_or(gp(J->status), bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// largest r in [0, n) with a[r] <= x, for non-decreasing a[0..n] with a[0] <= x
template <class P>
__device__ __forceinline__ int upper_index(P a, int n, int64_t x) {
    int lo = 0, hi = n;        // invariant: a[lo] <= x, answer in [lo, hi)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    return v;
}

// list r's word range [a, b), clamped into [0, total]
__device__ __forceinline__ void req_bounds(const Job* J, int r, int64_t& a, int64_t& b) {
    const gptr<const int64_t> rs = gp(J->req_start);
    int64_t x = rs[r], y = rs[r + 1];
    x = x < 0 ? 0 : (x > J->total ? J->total : x);
    y = y < x ? x : (y > J->total ? J->total : y);
    a = x;
    b = y;
}

// Chunk c -> list r and its global word range [gs, ge).  Chunks never
// straddle lists; chunk_begin is the running sum of ceil(n_r / kChunk).
__device__ __forceinline__ bool chunk_range(const Job* J, int64_t c, int& r, int64_t& a,
                                            int64_t& b, int64_t& gs, int64_t& ge) {
    const int R = J->R;
    const gptr<const int64_t> cb = gp(J->chunk_begin);
    int64_t nch = cb[R];
    if (nch > J->chunk_cap) nch = J->chunk_cap;
    if (c >= nch) return false;
    if (R == 1) {
        r = 0;
    } else {
        r = gp(J->chunk_list)[c];
        if (r < 0 || r >= R) return false;             // table not filled: nothing to do
    }
    req_bounds(J, r, a, b);
    gs = a + (c - cb[r]) * kChunk;
    ge = gs + kChunk < b ? gs + kChunk : b;
    return true;
}

// W = ceil(L/8) big-endian uint64 lanes of the L bytes at p; bytes past L are
// zero.  Aligned dword loads when the covering dwords lie inside [lo, hi);
// single bytes otherwise.
template <class BP, class OP>
__device__ __forceinline__ void pack_word(BP lo, BP hi, BP p, int L, OP out, int64_t stride) {
    const int W = lanes_for_len(L);
    const uintptr_t addr = (uintptr_t)p;
    const uintptr_t a4 = addr & ~(uintptr_t)3;
    const int sh = (int)(addr & 3);
    const int nd = (sh + L + 3) >> 2;                // dwords covering the word
    if (a4 >= (uintptr_t)lo && a4 + 4 * (uintptr_t)nd <= (uintptr_t)hi) {
        const gptr<const uint32_t> q = (gptr<const uint32_t>)a4;
        uint32_t prev = q[0];
        uint64_t acc = 0;
        const int dk = (L + 3) >> 2;                 // key dwords
        for (int i = 0; i < dk; ++i) {
            const uint32_t next = i + 1 < nd ? q[i + 1] : 0u;
            const uint32_t raw = __builtin_amdgcn_alignbyte(next, prev, sh);   // bytes 4i..4i+3
            prev = next;
            uint32_t be = __builtin_bswap32(raw);
            const int valid = L - 4 * i;
            if (valid < 4) be &= 0xFFFFFFFFu << (8 * (4 - valid));
            if ((i & 1) == 0) {
                acc = (uint64_t)be << 32;
            } else {
                acc |= be;
                out[(int64_t)(i >> 1) * stride] = acc;
            }
        }
        if (dk & 1) out[(int64_t)(dk >> 1) * stride] = acc;
    } else {
        for (int w = 0; w < W; ++w) {
            uint64_t v = 0;
            const int k1 = L - 8 * w < 8 ? L - 8 * w : 8;
            for (int k = 0; k < k1; ++k) v |= (uint64_t)p[8 * w + k] << (56 - 8 * k);
            out[(int64_t)w * stride] = v;
        }
    }
}

// ---------------------------------------------------------------- launchers

struct Bounds {              // launch sizes fixed on the host (capacities)
    int64_t total;           // words (capacity)
    int32_t R;               // lists (capacity)
    int32_t ml1;
    int64_t chunk_cap;
    int64_t tile_cap;        // tile list capacity per record width
    int32_t dmax;            // widest record in use
    int32_t hbm_merge;       // some sub-array may be merged through HBM (launch the merges)
    int32_t pair_lds;        // dynamic LDS bytes of the batched pair merge
    int32_t tile_keys[kNumD];
    int32_t hbm_tile_keys[kNumD];
    int32_t hbm_class[kNumD];   // in-LDS class sorting HBM chunks of width D (-1: tiles)
    int32_t fused_pack;      // the scatter packs keys (kJobFusedPack); no k_pack launch
    int64_t lb_cap;
    int32_t flags;
};

hipError_t launch_set_job(const Job& j, Job* dst, hipStream_t s);
hipError_t launch_bucketize(const Job* J, const Bounds& b, hipStream_t s);
// the two halves of launch_bucketize: counts, starts and key offsets; then the scatter
hipError_t launch_bucket_starts(const Job* J, const Bounds& b, hipStream_t s);
hipError_t launch_scatter(const Job* J, const Bounds& b, hipStream_t s);
hipError_t launch_chunk_plan(const Job* J, const Bounds& b, bool clear_status, hipStream_t s);
// after_bucketize: launch_bucket_starts of this call wrote key_off already
hipError_t launch_sort_prep(const Job* J, const Bounds& b, bool after_bucketize, hipStream_t s);
hipError_t launch_oets_tiles_one(const Job* J, const Bounds& b, int D, hipStream_t s);
hipError_t launch_lds_buckets(const Job* J, const Bounds& b, int D, hipStream_t s);
hipError_t launch_lds_class(const Job* J, const Bounds& b, int D, int c, hipStream_t s);
// sub-arrays merged through HBM: chunk sorts in LDS, then the merge-split
// plan and one launch for every phase of every sub-array
hipError_t launch_merges(const Job* J, const Bounds& b, hipStream_t s);
hipError_t launch_hbm_chunks(const Job* J, const Bounds& b, int D, hipStream_t s);
hipError_t launch_merge_sched(const Job* J, const Bounds& b, hipStream_t s);
// dynamic LDS the batched pair merge needs for records up to dmax dwords
int pair_merge_lds(int dmax);

// fixed-width keys for the unbucketed ablation (k_fixed_width.hip)
hipError_t launch_fixed_width(const uint8_t* bytes, int64_t n_bytes, const int64_t* offsets,
                              int64_t n_words,
                              int32_t width, int32_t mode, uint8_t* out, int64_t* offsets_out,
                              int32_t* status, hipStream_t s);

// data-structure ablation: whole-sub-array OETS, packed keys or text (k_layout.hip)
hipError_t launch_layout_oets(const uint8_t* bytes, int64_t n_bytes, const int64_t* offsets,
                              int32_t n_words, int32_t max_len, const int32_t* counts,
                              const int32_t* starts, const int32_t* order, int32_t* perm,
                              int32_t layout, int32_t* status, hipStream_t s);

// pre-processing, raw text to words (k_tokenize.hip)
size_t tok_workspace_bytes(int64_t n_bytes);
hipError_t launch_tokenize(const uint8_t* text, int64_t n_bytes, uint8_t* out, int64_t* offsets,
                           int64_t cap_words, int64_t* result, void* ws, hipStream_t s);
// plain per-bucket form pieces: one in-LDS sort of one sub-array (nchunks = 1,
// chunk = 0) or of the nchunks chunks of chunk words of one sub-array merged
// through HBM; one merge-split phase of one such sub-array
hipError_t launch_lds_one(const Job* J, int D, int c, const LBucket& bk, int nchunks, int chunk,
                          hipStream_t s);
hipError_t launch_merge_phase_one(const Job* J, const MSub& m, int phase, int lds_bytes,
                                  hipStream_t s);
hipError_t launch_pack(const Job* J, const Bounds& b, hipStream_t s);
hipError_t launch_tile_one_bucket(const Job* J, int D, const TileDesc& first, int ntiles,
                                  int T, bool write_keys, hipStream_t s);

}  // namespace bsort
