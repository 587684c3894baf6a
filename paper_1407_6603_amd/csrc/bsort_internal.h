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

namespace bsort {

constexpr int kMaxLen = 64;
constexpr int kMaxD = 17;                 // ceil(64/4) + 1
constexpr int kNumD = kMaxD + 1;          // arrays indexed by D directly
constexpr int kWave = 64;
constexpr int kChunkRounds = 16;
constexpr int kChunk = kWave * kChunkRounds;   // words per bucketize chunk
constexpr int kTileWavesPerBlock = 4;
constexpr int kMinTile = 128;             // 64 lanes x 2 records
constexpr int kMaxPhaseCap = 1 << 22;
constexpr int kFlagTilesOnly = 2;         // same value as BSORT_FLAG_TILES_ONLY
constexpr int kJobKeepStatus = 1 << 8;    // Job.flags: leave the status word as it is

// device status bits (workspace status word)
enum : uint32_t {
    ST_BAD_OFFSETS = 1u,
    ST_TOO_LONG = 2u,
    ST_BAD_REQ = 4u,
    ST_OVERFLOW = 8u,      // an internal list bound was exceeded (a library bug)
};

// records per lane limit by key width: D * K <= 128 VGPRs of record state
__host__ __device__ constexpr int kmax_for(int D) {
    return D <= 2 ? 64 : D <= 4 ? 32 : D <= 8 ? 16 : D <= 16 ? 8 : 4;
}
__host__ __device__ constexpr int dwords_for_len(int L) { return (L + 3) / 4 + 1; }
__host__ __device__ constexpr int lanes_for_len(int L) { return (L + 7) / 8; }

struct TileDesc {            // one odd-even transposition tile
    int64_t pos0;            // global position of the bucket's first word
    int64_t key_off;         // uint64 index of the bucket's lane 0
    int32_t n_b;             // words in the bucket
    int32_t t0;              // first bucket word of this tile
    int32_t n;               // words in this tile
    int32_t L;               // word length
};

struct MergeItem {           // one merge-split of tiles a and a+1 of a bucket
    int64_t pos0;
    int64_t key_off;
    int32_t n_b;
    int32_t L;
    int32_t T;               // tile size of this bucket
    int32_t a;               // lower tile
    int32_t p;               // tiles in the bucket
    int32_t pad;
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
    int32_t* chunk_hist;         // [chunk_cap * ml1], scanned in place
    int64_t chunk_cap;
    int64_t* key_off;            // [R * ml1]
    uint64_t* keys;              // [wmax * total]
    TileDesc* tiles[kNumD];      // per record width D
    int64_t tile_cap[kNumD];
    int32_t tile_keys[kNumD];    // tile size per D
    int32_t* tile_count;         // [kNumD]
    MergeItem* mlist[2];         // double-buffered phase lists
    int64_t merge_cap;
    int32_t* mcount;             // [phase_cap + 1]
    int32_t phase_cap;
    int32_t pad0;
    int64_t rs_inline[2];        // req_start storage for single-list calls
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void set_status(const Job* J, uint32_t bit) {
    atomicOr(J->status, bit);
}

// largest r in [0, n) with a[r] <= x, for non-decreasing a[0..n] with a[0] <= x
__device__ __forceinline__ int upper_index(const int64_t* a, int n, int64_t x) {
    int lo = 0, hi = n;        // invariant: a[lo] <= x, answer in [lo, hi)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// Lexicographic a > b over D dwords, a[0] most significant.  Adjacent dwords
// are compared as one uint64, from the least significant end up.
template <int D>
__device__ __forceinline__ bool rec_gt(const uint32_t (&a)[D], const uint32_t (&b)[D]) {
    bool g;
    if constexpr (D & 1) {
        g = a[D - 1] > b[D - 1];
    } else {
        uint64_t pa = ((uint64_t)a[D - 2] << 32) | a[D - 1];
        uint64_t pb = ((uint64_t)b[D - 2] << 32) | b[D - 1];
        g = pa > pb;
    }
    constexpr int qtop = (D & 1) ? D / 2 - 1 : D / 2 - 2;
#pragma unroll
    for (int q = qtop; q >= 0; --q) {
        uint64_t pa = ((uint64_t)a[2 * q] << 32) | a[2 * q + 1];
        uint64_t pb = ((uint64_t)b[2 * q] << 32) | b[2 * q + 1];
        g = (pa > pb) | ((pa == pb) & g);
    }
    return g;
}

// compare-exchange: afterwards a <= b
template <int D>
__device__ __forceinline__ void cex(uint32_t (&a)[D], uint32_t (&b)[D]) {
    bool s = rec_gt<D>(a, b);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        uint32_t x = a[d], y = b[d];
        a[d] = s ? y : x;
        b[d] = s ? x : y;
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
    int32_t phase_bound;     // merge-split phases to launch
    int32_t merge_threads;
    int32_t merge_lds;       // dynamic LDS bytes per merge workgroup
    int32_t tile_keys[kNumD];
    int32_t flags;
};

hipError_t launch_set_job(const Job& j, Job* dst, hipStream_t s);
hipError_t launch_bucketize(const Job* J, const Bounds& b, hipStream_t s);
hipError_t launch_sort(const Job* J, const Bounds& b, hipStream_t s);
// plain per-bucket form pieces
hipError_t launch_pack(const Job* J, const Bounds& b, hipStream_t s);
hipError_t launch_tile_one_bucket(const Job* J, int D, const TileDesc& first, int ntiles,
                                  int T, bool write_keys, hipStream_t s);
hipError_t launch_merge_one_bucket(const Job* J, const MergeItem& item0, int npairs,
                                   int phase, int merge_threads, int lds, hipStream_t s);
hipError_t launch_sort_prep(const Job* J, const Bounds& b, hipStream_t s);
hipError_t launch_oets_tiles_one(const Job* J, const Bounds& b, int D, hipStream_t s);
hipError_t launch_merges(const Job* J, const Bounds& b, hipStream_t s);
hipError_t launch_merge_phase(const Job* J, const Bounds& b, int phase, hipStream_t s);


}  // namespace bsort
