// Odd-even transposition sort of one tile of a sub-array per wavefront.
//
// Bubble sort's passes (Section I; the paper's per-sub-array sort) become,
// on a 64-wide wavefront, odd-even transposition sort: n phases over n keys;
// even phases compare-exchange positions (2i, 2i+1), odd phases (2i+1, 2i+2);
// n(n-1)/2 compare-exchanges in all, the same count bubble sort makes.
//
// Layout: lane l holds K consecutive records of the tile (positions
// l*K .. l*K+K-1) in VGPRs, K even.  Even phases and all but one pair of an
// odd phase stay inside a lane; the odd phase's pair (lane l, record K-1) /
// (lane l+1, record 0) crosses lanes and moves through DPP (wave_shl:1 and
// wave_shr:1 row moves), no LDS traffic and no barrier.  Positions past the
// tile's words hold all-ones records, which compare above every word and
// never move; n phases (n = words in the tile) therefore suffice.
//
// K per tile is the smallest power of two >= ceil(n/64) (at least 2), up to a
// bound that keeps D*K <= 128 record VGPRs, so small sub-arrays do not pay
// for the full tile width.
#include "bsort_internal.h"

namespace bsort {

constexpr int kDppWaveShl1 = 0x130;   // lane i reads lane i+1
constexpr int kDppWaveShr1 = 0x138;   // lane i reads lane i-1

template <int D>
__device__ __forceinline__ void cross_lane_odd(uint32_t (&first)[D], uint32_t (&last)[D],
                                               int lane) {
    uint32_t rf[D], ll[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
#ifdef BSORT_XCHG_SHFL
        rf[d] = (uint32_t)__shfl_down((int)first[d], 1, kWave);
        ll[d] = (uint32_t)__shfl_up((int)last[d], 1, kWave);
#else
        rf[d] = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)first[d], kDppWaveShl1, 0xF, 0xF,
                                                      false);
        ll[d] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)last[d], kDppWaveShr1, 0xF, 0xF,
                                                      false);
#endif
    }
    // the same pair (lane l's last, lane l+1's first) is compared on both sides
    const bool take_right = rec_gt<D>(last, rf) && lane != kWave - 1;
    const bool take_left = rec_gt<D>(ll, first) && lane != 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        last[d] = take_right ? rf[d] : last[d];
        first[d] = take_left ? ll[d] : first[d];
    }
}

// ---- exact double min/max compare-exchange for records of two dwords (L <= 4)
//
// A record (key32, index) with index < 2^31 is the integer v = key32*2^31 +
// index.  With key32 < 0xFFC00000, v + 2^52 lies in [2^52, 0x7FEFFFFFFFFFFFFF],
// the bit patterns of positive normal doubles, whose order as doubles is the
// order of the patterns as unsigned integers; IEEE min and max return one of
// their operands unchanged.  So v_min_f64/v_max_f64 on these patterns are an
// exact compare-exchange of the records.  +inf pads the tile and 0.0 is below
// every record, so the cross-lane exchange needs no lane masks.
constexpr uint32_t kF64KeyLimit = 0xFFC00000u;
constexpr uint64_t kF64Bias = 1ull << 52;
constexpr uint64_t kF64Inf = 0x7FF0000000000000ull;

__device__ __forceinline__ double dmin(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double dmax(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double dpp_f64(double x, int ctrl_is_shl, uint64_t old_bits) {
    const uint64_t v = (uint64_t)__double_as_longlong(x);
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const int olo = (int)(uint32_t)old_bits, ohi = (int)(uint32_t)(old_bits >> 32);
    int rlo, rhi;
    if (ctrl_is_shl) {
        rlo = __builtin_amdgcn_update_dpp(olo, lo, 0x130, 0xF, 0xF, false);
        rhi = __builtin_amdgcn_update_dpp(ohi, hi, 0x130, 0xF, 0xF, false);
    } else {
        rlo = __builtin_amdgcn_update_dpp(olo, lo, 0x138, 0xF, 0xF, false);
        rhi = __builtin_amdgcn_update_dpp(ohi, hi, 0x138, 0xF, 0xF, false);
    }
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)rhi << 32) | (uint32_t)rlo));
}

template <int K>
__device__ __forceinline__ void phases_f64(uint32_t (&r)[K][2], int nph) {
    double x[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint64_t v = r[k][0] == 0xFFFFFFFFu && r[k][1] == 0xFFFFFFFFu
                               ? kF64Inf
                               : (((uint64_t)r[k][0] << 31) | r[k][1]) + kF64Bias;
        x[k] = __longlong_as_double((long long)v);
    }
    for (int ph = 0; ph < nph; ph += 2) {
#pragma unroll
        for (int k = 0; k + 1 < K; k += 2) {
            const double lo = dmin(x[k], x[k + 1]), hi = dmax(x[k], x[k + 1]);
            x[k] = lo;
            x[k + 1] = hi;
        }
        if (ph + 1 < nph) {
            const double rf = dpp_f64(x[0], 1, kF64Inf);    // right neighbour's first
            const double ll = dpp_f64(x[K - 1], 0, 0);      // left neighbour's last
#pragma unroll
            for (int k = 1; k + 1 <= K - 2; k += 2) {
                const double lo = dmin(x[k], x[k + 1]), hi = dmax(x[k], x[k + 1]);
                x[k] = lo;
                x[k + 1] = hi;
            }
            x[K - 1] = dmin(x[K - 1], rf);
            x[0] = dmax(ll, x[0]);
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint64_t v = (uint64_t)__double_as_longlong(x[k]);
        if (v == kF64Inf) {
            r[k][0] = 0xFFFFFFFFu;
            r[k][1] = 0xFFFFFFFFu;
        } else {
            const uint64_t u = v - kF64Bias;
            r[k][0] = (uint32_t)(u >> 31);
            r[k][1] = (uint32_t)(u & 0x7FFFFFFFu);
        }
    }
}

template <int D, int K>
__device__ __forceinline__ void phases_int(uint32_t (&r)[K][D], int nph, int lane) {
    for (int ph = 0; ph < nph; ph += 2) {
#pragma unroll
        for (int k = 0; k + 1 < K; k += 2) cex<D>(r[k], r[k + 1]);          // even phase
        if (ph + 1 < nph) {                                                  // odd phase
#pragma unroll
            for (int k = 1; k + 1 <= K - 2; k += 2) cex<D>(r[k], r[k + 1]);
            cross_lane_odd<D>(r[0], r[K - 1], lane);
        }
    }
}

template <int D, int K>
__device__ __forceinline__ void oets_tile(const Job* __restrict__ J, const TileDesc& t,
                                          bool write_keys, int lane) {
    static_assert(K >= 2 && (K & 1) == 0, "K must be even");
    constexpr int Dk = D - 1;            // key dwords
    constexpr int W = (Dk + 1) / 2;      // uint64 lanes
    uint32_t r[K][D];
    uint64_t* __restrict__ keys = J->keys + t.key_off;
    int32_t* __restrict__ perm = J->perm + t.pos0;
    const int64_t nbk = t.n_b;
    const int jbase = t.t0 + lane * K;
    const int jend = t.t0 + t.n;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int j = jbase + k;
        if (j < jend) {
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t v = keys[w * nbk + j];
                r[k][2 * w] = (uint32_t)(v >> 32);
                if (2 * w + 1 < Dk) r[k][2 * w + 1] = (uint32_t)v;
            }
            r[k][Dk] = (uint32_t)perm[j];
        } else {
#pragma unroll
            for (int d = 0; d < D; ++d) r[k][d] = 0xFFFFFFFFu;
        }
    }

    const int nph = t.n;
    if constexpr (D == 2) {
        bool ok = true;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (jbase + k < jend && r[k][0] >= kF64KeyLimit) ok = false;
        if (__all(ok)) phases_f64<K>(r, nph);
        else phases_int<D, K>(r, nph, lane);
    } else {
        phases_int<D, K>(r, nph, lane);
    }

#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int j = jbase + k;
        if (j < jend) {
            perm[j] = (int32_t)r[k][Dk];
            if (write_keys) {
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint64_t hi = r[k][2 * w];
                    const uint64_t lo = (2 * w + 1 < Dk) ? r[k][2 * w + 1] : 0u;
                    keys[w * nbk + j] = (hi << 32) | lo;
                }
            }
        }
    }
}

// smallest supported K >= kneed (kneed <= kmax_for(D) by construction)
template <int D, int K>
__device__ __forceinline__ void run_tile_k(const Job* J, const TileDesc& t, bool wk, int lane,
                                           int kneed) {
    if constexpr (K * 2 > kmax_for(D)) {
        oets_tile<D, K>(J, t, wk, lane);
    } else {
        if (kneed <= K) oets_tile<D, K>(J, t, wk, lane);
        else run_tile_k<D, K * 2>(J, t, wk, lane, kneed);
    }
}

template <int D>
__device__ __forceinline__ void run_tile(const Job* J, const TileDesc& t, bool wk, int lane) {
    const int kneed = (t.n + kWave - 1) / kWave;
    run_tile_k<D, 2>(J, t, wk, lane, kneed);
}

template <int D>
__global__ __launch_bounds__(256) void k_oets_tiles(const Job* __restrict__ J) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t cnt = J->tile_count[D];
    if (cnt > J->tile_cap[D]) cnt = J->tile_cap[D];
    const TileDesc* tl = J->tiles[D];
    const int T = J->tile_keys[D];
    const bool tiles_only = (J->flags & kFlagTilesOnly) != 0;
    for (int64_t i = (int64_t)blockIdx.x * kTileWavesPerBlock + wv; i < cnt;
         i += (int64_t)gridDim.x * kTileWavesPerBlock) {
        const TileDesc t = tl[i];
        const bool wk = t.n_b > T && !tiles_only;   // merge-split reads the keys back
        run_tile<D>(J, t, wk, lane);
    }
}

// plain form: one launch per sub-array, one 64-thread workgroup per tile
template <int D>
__global__ __launch_bounds__(64) void k_oets_bucket(const Job* __restrict__ J, TileDesc t,
                                                    int T, int wk) {
    const int lane = threadIdx.x;
    t.t0 = (int)blockIdx.x * T;
    t.n = t.n_b - t.t0 < T ? t.n_b - t.t0 : T;
    run_tile<D>(J, t, wk != 0, lane);
}

template <int D>
static void launch_tiles_d(const Job* J, int64_t tile_cap, hipStream_t s) {
    int64_t g = (tile_cap + kTileWavesPerBlock - 1) / kTileWavesPerBlock;
    if (g > 2048) g = 2048;
    if (g < 1) g = 1;
    k_oets_tiles<D><<<(unsigned)g, 256, 0, s>>>(J);
}

template <int D>
static void launch_bucket_d(const Job* J, const TileDesc& t, int ntiles, int T, bool wk,
                            hipStream_t s) {
    k_oets_bucket<D><<<ntiles, 64, 0, s>>>(J, t, T, wk ? 1 : 0);
}

using TileLauncher = void (*)(const Job*, int64_t, hipStream_t);
using BucketLauncher = void (*)(const Job*, const TileDesc&, int, int, bool, hipStream_t);

static const TileLauncher kTileLaunchers[kNumD] = {
    nullptr, nullptr, launch_tiles_d<2>, launch_tiles_d<3>, launch_tiles_d<4>,
    launch_tiles_d<5>, launch_tiles_d<6>, launch_tiles_d<7>, launch_tiles_d<8>,
    launch_tiles_d<9>, launch_tiles_d<10>, launch_tiles_d<11>, launch_tiles_d<12>,
    launch_tiles_d<13>, launch_tiles_d<14>, launch_tiles_d<15>, launch_tiles_d<16>,
    launch_tiles_d<17>};

static const BucketLauncher kBucketLaunchers[kNumD] = {
    nullptr, nullptr, launch_bucket_d<2>, launch_bucket_d<3>, launch_bucket_d<4>,
    launch_bucket_d<5>, launch_bucket_d<6>, launch_bucket_d<7>, launch_bucket_d<8>,
    launch_bucket_d<9>, launch_bucket_d<10>, launch_bucket_d<11>, launch_bucket_d<12>,
    launch_bucket_d<13>, launch_bucket_d<14>, launch_bucket_d<15>, launch_bucket_d<16>,
    launch_bucket_d<17>};

hipError_t launch_oets_tiles_one(const Job* J, const Bounds& b, int D, hipStream_t s) {
    if (D < 2 || D > kMaxD) return hipErrorInvalidValue;
    kTileLaunchers[D](J, b.tile_cap, s);
    return hipGetLastError();
}

hipError_t launch_tile_one_bucket(const Job* J, int D, const TileDesc& first, int ntiles, int T,
                                  bool write_keys, hipStream_t s) {
    if (D < 2 || D > kMaxD || ntiles <= 0) return hipErrorInvalidValue;
    kBucketLaunchers[D](J, first, ntiles, T, write_keys, s);
    return hipGetLastError();
}

}  // namespace bsort
