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
#include <algorithm>

#include "bsort_internal.h"

namespace bsort {

constexpr int kDppWaveShl1 = 0x130;   // lane i reads lane i+1
constexpr int kDppWaveShr1 = 0x138;   // lane i reads lane i-1

// Within a tile, records start in input order (the scatter by length is
// stable) and only adjacent records are ever exchanged, and only when the left
// key is strictly greater; equal keys therefore never pass each other and
// their indices stay increasing.  So the tile sort compares keys alone: the
// result is the (key, index) order without comparing indices.
template <int D>
__device__ __forceinline__ bool key_gt(const uint32_t (&a)[D], const uint32_t (&b)[D]) {
    constexpr int Dk = D - 1;                       // key dwords
    bool g;
    if constexpr (Dk & 1) {
        g = a[Dk - 1] > b[Dk - 1];
    } else {
        const uint64_t pa = ((uint64_t)a[Dk - 2] << 32) | a[Dk - 1];
        const uint64_t pb = ((uint64_t)b[Dk - 2] << 32) | b[Dk - 1];
        g = pa > pb;
    }
    constexpr int qtop = (Dk & 1) ? Dk / 2 - 1 : Dk / 2 - 2;
#pragma unroll
    for (int q = qtop; q >= 0; --q) {
        const uint64_t pa = ((uint64_t)a[2 * q] << 32) | a[2 * q + 1];
        const uint64_t pb = ((uint64_t)b[2 * q] << 32) | b[2 * q + 1];
        g = (pa > pb) | ((pa == pb) & g);
    }
    return g;
}

template <int D>
__device__ __forceinline__ void cex_key(uint32_t (&a)[D], uint32_t (&b)[D]) {
    const bool s = key_gt<D>(a, b);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const uint32_t x = a[d], y = b[d];
        a[d] = s ? y : x;
        b[d] = s ? x : y;
    }
}

// Odd phase across lanes: lane l's last record against lane l+1's first.
// rf/ll carry the neighbours' records between phases; the wave-edge lanes
// (63 for rf, 0 for ll) have no source lane, keep their initial all-ones /
// all-zeros records, and so never exchange.
template <int D>
__device__ __forceinline__ void cross_lane_odd(uint32_t (&first)[D], uint32_t (&last)[D],
                                               uint32_t (&rf)[D], uint32_t (&ll)[D]) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
        rf[d] = (uint32_t)__builtin_amdgcn_update_dpp((int)rf[d], (int)first[d], kDppWaveShl1,
                                                      0xF, 0xF, false);
        ll[d] = (uint32_t)__builtin_amdgcn_update_dpp((int)ll[d], (int)last[d], kDppWaveShr1,
                                                      0xF, 0xF, false);
    }
    // the same pair (lane l's last, lane l+1's first) is compared on both sides
    const bool take_right = key_gt<D>(last, rf);
    const bool take_left = key_gt<D>(ll, first);
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
// DPP row move of a double; lanes without a source lane keep `old`
__device__ __forceinline__ double dpp_f64(double old, double x, bool shl) {
    const uint64_t v = (uint64_t)__double_as_longlong(x);
    const uint64_t o = (uint64_t)__double_as_longlong(old);
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const int olo = (int)(uint32_t)o, ohi = (int)(uint32_t)(o >> 32);
    int rlo, rhi;
    if (shl) {
        rlo = __builtin_amdgcn_update_dpp(olo, lo, kDppWaveShl1, 0xF, 0xF, false);
        rhi = __builtin_amdgcn_update_dpp(ohi, hi, kDppWaveShl1, 0xF, 0xF, false);
    } else {
        rlo = __builtin_amdgcn_update_dpp(olo, lo, kDppWaveShr1, 0xF, 0xF, false);
        rhi = __builtin_amdgcn_update_dpp(ohi, hi, kDppWaveShr1, 0xF, 0xF, false);
    }
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)rhi << 32) | (uint32_t)rlo));
}

template <int K>
__device__ __forceinline__ void even_f64(double (&x)[K]) {
#pragma unroll
    for (int k = 0; k + 1 < K; k += 2) {
        const double lo = dmin(x[k], x[k + 1]), hi = dmax(x[k], x[k + 1]);
        x[k] = lo;
        x[k + 1] = hi;
    }
}

template <int K>
__device__ __forceinline__ void odd_f64(double (&x)[K], double& rf, double& ll) {
    rf = dpp_f64(rf, x[0], true);                     // right neighbour's first
    ll = dpp_f64(ll, x[K - 1], false);                // left neighbour's last
#pragma unroll
    for (int k = 1; k + 1 <= K - 2; k += 2) {
        const double lo = dmin(x[k], x[k + 1]), hi = dmax(x[k], x[k + 1]);
        x[k] = lo;
        x[k + 1] = hi;
    }
    x[K - 1] = dmin(x[K - 1], rf);
    x[0] = dmax(ll, x[0]);
}

template <int K>
__device__ __forceinline__ void phases_f64(uint32_t (&r)[K][2], int n) {
    const int nph = __builtin_amdgcn_readfirstlane(n);
    double x[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint64_t v = r[k][0] == 0xFFFFFFFFu && r[k][1] == 0xFFFFFFFFu
                               ? kF64Inf
                               : (((uint64_t)r[k][0] << 31) | r[k][1]) + kF64Bias;
        x[k] = __longlong_as_double((long long)v);
    }
    // +inf above every record, 0.0 below: the edge lanes never exchange
    double rf = __longlong_as_double((long long)kF64Inf), ll = 0.0;
    int ph = 0;
    for (; ph + 2 <= nph; ph += 2) {
        even_f64<K>(x);
        odd_f64<K>(x, rf, ll);
    }
    if (ph < nph) even_f64<K>(x);
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
__device__ __forceinline__ void even_int(uint32_t (&r)[K][D]) {
#pragma unroll
    for (int k = 0; k + 1 < K; k += 2) cex_key<D>(r[k], r[k + 1]);
}

template <int D, int K>
__device__ __forceinline__ void odd_int(uint32_t (&r)[K][D], uint32_t (&rf)[D],
                                        uint32_t (&ll)[D]) {
#pragma unroll
    for (int k = 1; k + 1 <= K - 2; k += 2) cex_key<D>(r[k], r[k + 1]);
    cross_lane_odd<D>(r[0], r[K - 1], rf, ll);
}

template <int D, int K>
__device__ __forceinline__ void phases_int(uint32_t (&r)[K][D], int n) {
    const int nph = __builtin_amdgcn_readfirstlane(n);
    uint32_t rf[D], ll[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        rf[d] = 0xFFFFFFFFu;
        ll[d] = 0u;
    }
    // pairs of phases with no branch between them, so each phase's results
    // take the next phase's registers without copies; a last even phase if n is odd
    int ph = 0;
    for (; ph + 2 <= nph; ph += 2) {
        even_int<D, K>(r);
        odd_int<D, K>(r, rf, ll);
    }
    if (ph < nph) even_int<D, K>(r);
}

// ---- tile sources: where a wave's K records per lane come from and go back to

// A tile in HBM: key lanes and index payload of bucket words [t0, t0+n).
struct HbmTile {
    gptr<uint64_t> keys;
    gptr<int32_t> perm;
    int64_t nbk;
    int t0, n;
    bool write_keys;

    template <int D, int K>
    __device__ __forceinline__ void load(uint32_t (&r)[K][D], int lane) const {
        constexpr int Dk = D - 1, W = (Dk + 1) / 2;
        const int jbase = t0 + lane * K, jend = t0 + n;
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
    }
    template <int D, int K>
    __device__ __forceinline__ void store(const uint32_t (&r)[K][D], int lane) const {
        constexpr int Dk = D - 1, W = (Dk + 1) / 2;
        const int jbase = t0 + lane * K, jend = t0 + n;
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
};

// Records in LDS are SoA dword planes of `cap` (a multiple of 64) records:
// dword d of record i sits at lds[d*cap + lsw(i)].  lsw permutes the records
// inside each row of 64 (column XOR row), so lanes that touch records a
// multiple of 2..64 apart, as tile loads (K per lane) and slot write-backs
// (E per lane) do, spread over the banks instead of a few of them.
__device__ __forceinline__ int lsw(int i) { return i ^ ((i >> 6) & 63); }

// A tile of records held in LDS, records [t0, t0+n).
struct LdsTile {
    uint32_t* lds;
    int cap;
    int t0, n;

    template <int D, int K>
    __device__ __forceinline__ void load(uint32_t (&r)[K][D], int lane) const {
        const int jbase = t0 + lane * K, jend = t0 + n;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int j = jbase + k;
#pragma unroll
            for (int d = 0; d < D; ++d) r[k][d] = j < jend ? lds[d * cap + lsw(j)] : 0xFFFFFFFFu;
        }
    }
    template <int D, int K>
    __device__ __forceinline__ void store(const uint32_t (&r)[K][D], int lane) const {
        const int jbase = t0 + lane * K, jend = t0 + n;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int j = jbase + k;
            if (j < jend) {
#pragma unroll
                for (int d = 0; d < D; ++d) lds[d * cap + lsw(j)] = r[k][d];
            }
        }
    }
};

template <int D, int K, class Src>
__device__ __forceinline__ void sort_tile(const Src& src, int n, int lane) {
    static_assert(K >= 2 && (K & 1) == 0, "K must be even");
    uint32_t r[K][D];
    src.template load<D, K>(r, lane);
    if constexpr (D == 2) {
        bool ok = true;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (lane * K + k < n && r[k][0] >= kF64KeyLimit) ok = false;
        if (__all(ok)) phases_f64<K>(r, n);
        else phases_int<D, K>(r, n);
    } else {
        phases_int<D, K>(r, n);
    }
    src.template store<D, K>(r, lane);
}

// smallest supported K >= kneed, K <= KCAP (kneed <= KCAP by construction)
template <int D, int K, int KCAP, class Src>
__device__ __forceinline__ void sort_tile_k(const Src& src, int n, int lane, int kneed) {
    if constexpr (K * 2 > KCAP) {
        sort_tile<D, K>(src, n, lane);
    } else {
        if (kneed <= K) sort_tile<D, K>(src, n, lane);
        else sort_tile_k<D, K * 2, KCAP>(src, n, lane, kneed);
    }
}

template <int D, int KCAP, class Src>
__device__ __forceinline__ void sort_tile_any(const Src& src, int n, int lane) {
    sort_tile_k<D, 2, KCAP>(src, n, lane, (n + kWave - 1) / kWave);
}

// Two-dword records compared whole (key dwords of a 5- or 6-byte word, its
// position in the sub-array in the low 16 bits of the second, which the key
// leaves zero): the exact fp64 form when the wave's records allow it, else
// the three-dword integer phases, whose key is exactly these two dwords (with
// a zero third dword in registers: the index plane in LDS stays as loaded).
// Padding records (all ones) sort last.
template <int K, class Src>
__device__ __forceinline__ void sort_tile_full2(const Src& src, int n, int lane) {
    uint32_t r[K][2];
    src.template load<2, K>(r, lane);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (lane * K + k < n && (r[k][0] >= kF64KeyLimit || r[k][1] >= 0x80000000u)) ok = false;
    if (__all(ok)) {
        phases_f64<K>(r, n);
    } else {
        uint32_t r3[K][3];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            r3[k][0] = r[k][0];
            r3[k][1] = r[k][1];
            r3[k][2] = 0u;
        }
        phases_int<3, K>(r3, n);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            r[k][0] = r3[k][0];
            r[k][1] = r3[k][1];
        }
    }
    src.template store<2, K>(r, lane);
}

// One-dword records (a 1- or 2-byte word's key in the high half, its
// position in the sub-array in the low half, which the key leaves zero),
// compared whole: a compare-exchange is one v_min_u32 and one v_max_u32.
// All-ones pads the tile and sorts last; the edge lanes' neighbours are
// all-ones (right) and zero (left), so they never exchange.
template <int K>
__device__ __forceinline__ void phases_u32(uint32_t (&x)[K], int n) {
    const int nph = __builtin_amdgcn_readfirstlane(n);
    uint32_t rf = 0xFFFFFFFFu, ll = 0u;
    int ph = 0;
    for (; ph + 2 <= nph; ph += 2) {
#pragma unroll
        for (int k = 0; k + 1 < K; k += 2) {
            const uint32_t lo = x[k] < x[k + 1] ? x[k] : x[k + 1];
            const uint32_t hi = x[k] < x[k + 1] ? x[k + 1] : x[k];
            x[k] = lo;
            x[k + 1] = hi;
        }
        rf = (uint32_t)__builtin_amdgcn_update_dpp((int)rf, (int)x[0], kDppWaveShl1, 0xF, 0xF,
                                                   false);
        ll = (uint32_t)__builtin_amdgcn_update_dpp((int)ll, (int)x[K - 1], kDppWaveShr1, 0xF,
                                                   0xF, false);
#pragma unroll
        for (int k = 1; k + 1 <= K - 2; k += 2) {
            const uint32_t lo = x[k] < x[k + 1] ? x[k] : x[k + 1];
            const uint32_t hi = x[k] < x[k + 1] ? x[k + 1] : x[k];
            x[k] = lo;
            x[k + 1] = hi;
        }
        x[K - 1] = x[K - 1] < rf ? x[K - 1] : rf;
        x[0] = ll < x[0] ? x[0] : ll;
    }
    if (ph < nph) {
#pragma unroll
        for (int k = 0; k + 1 < K; k += 2) {
            const uint32_t lo = x[k] < x[k + 1] ? x[k] : x[k + 1];
            const uint32_t hi = x[k] < x[k + 1] ? x[k + 1] : x[k];
            x[k] = lo;
            x[k + 1] = hi;
        }
    }
}

template <int K, int KCAP, class Src>
__device__ __forceinline__ void sort_tile_full1_k(const Src& src, int n, int lane, int kneed) {
    if (K * 2 > KCAP || kneed <= K) {
        uint32_t r[K][1];
        src.template load<1, K>(r, lane);
        uint32_t x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = r[k][0];
        phases_u32<K>(x, n);
#pragma unroll
        for (int k = 0; k < K; ++k) r[k][0] = x[k];
        src.template store<1, K>(r, lane);
    } else if constexpr (K * 2 <= KCAP) {
        sort_tile_full1_k<K * 2, KCAP>(src, n, lane, kneed);
    }
}

// Records of 3-byte words (key dword b0 b1 b2 0, index) in one dword when
// every first byte of the tile is below 0x80: the key's 23 significant bits
// above the record's position in the tile (9 bits: tiles of at most 512
// records), compared whole by v_min_u32/v_max_u32 like the one-dword records
// above, half the issue cost of the two-dword fp64 form.  Positions follow
// input order, so this is the (key, index) order.  The sorted dwords give
// back each key and, through the index plane at the position each carries,
// each index: the wave reads all of them before it writes any.  Padding is
// all ones; with n < 512 no record reaches it, with n = 512 there is none.
// A tile with a first byte >= 0x80 takes the two-dword phases.
template <int K>
__device__ __forceinline__ void sort_tile_pack3(const LdsTile& src, int n, int lane) {
    static_assert(K * kWave <= 512, "tile positions take 9 bits");
    uint32_t r[K][2];
    src.template load<2, K>(r, lane);
    bool ok = true;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (lane * K + k < n && r[k][0] >= 0x80000000u) ok = false;
    if (__all(ok)) {
        uint32_t x[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int j = lane * K + k;
            x[k] = j < n ? ((r[k][0] >> 8) << 9) | (uint32_t)j : 0xFFFFFFFFu;
        }
        phases_u32<K>(x, n);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (lane * K + k < n) {                    // (the store keeps these only)
                r[k][0] = (x[k] >> 9) << 8;
                r[k][1] = src.lds[src.cap + lsw(src.t0 + (int)(x[k] & 511u))];
            }
        }
    } else {
        bool f64 = true;
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (lane * K + k < n && r[k][0] >= kF64KeyLimit) f64 = false;
        if (__all(f64)) phases_f64<K>(r, n);
        else phases_int<2, K>(r, n);
    }
    src.template store<2, K>(r, lane);
}

template <int K, int KCAP>
__device__ __forceinline__ void sort_tile_pack3_k(const LdsTile& src, int n, int lane,
                                                  int kneed) {
    if constexpr (K * 2 > KCAP) {
        sort_tile_pack3<K>(src, n, lane);
    } else {
        if (kneed <= K) sort_tile_pack3<K>(src, n, lane);
        else sort_tile_pack3_k<K * 2, KCAP>(src, n, lane, kneed);
    }
}

template <int K, int KCAP, class Src>
__device__ __forceinline__ void sort_tile_full2_k(const Src& src, int n, int lane, int kneed) {
    if constexpr (K * 2 > KCAP) {
        sort_tile_full2<K>(src, n, lane);
    } else {
        if (kneed <= K) sort_tile_full2<K>(src, n, lane);
        else sort_tile_full2_k<K * 2, KCAP>(src, n, lane, kneed);
    }
}

template <int D>
__device__ __forceinline__ void run_tile(const Job* J, const TileDesc& t, bool wk, int lane) {
    HbmTile src{gp(J->keys) + t.key_off, gp(J->perm) + t.pos0, t.n_b, t.t0, t.n, wk};
    sort_tile_any<D, kmax_for(D)>(src, t.n, lane);
}

template <int D>
__global__ __launch_bounds__(256) void k_oets_tiles(const Job* __restrict__ J) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int64_t cnt = J->tile_count[D];
    if (cnt > J->tile_cap[D]) cnt = J->tile_cap[D];
    const TileDesc* tl = J->tiles[D];
    const int T = J->hbm_tile_keys[D];
    const bool tiles_only = (J->flags & kFlagTilesOnly) != 0;
    for (int64_t i = (int64_t)blockIdx.x * kTileWavesPerBlock + wv; i < cnt;
         i += (int64_t)gridDim.x * kTileWavesPerBlock) {
        const TileDesc t = tl[i];
        const bool wk = t.n_b > T && !tiles_only;   // merge-split through HBM reads keys back
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

// ---- whole sub-arrays in LDS
//
// One workgroup per sub-array of T < n <= CAP words: the sub-array is read
// into LDS once; its ceil(n/T) tiles are sorted by odd-even transposition in
// registers (one wave per tile); then the p = ceil(n/T) phases of the block
// odd-even merge-split run in LDS.  In phase s the pairs (a, a+1), a = s mod
// 2, s mod 2 + 2, ..., are merged; each thread produces up to CAP/NT
// consecutive outputs of one phase (found by a merge-path search), holds them
// in registers, and after a barrier writes them back in place.  Only the
// final index payload is written to HBM.

template <int D>
__device__ __forceinline__ void lds_rec(const uint32_t* lds, int cap, int i, uint32_t (&x)[D]) {
    const int a = lsw(i);
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = lds[d * cap + a];
}

// ---- merge-split phases inside LDS
//
// A phase pairs tiles (a, a+1), a = s&1, s&1 + 2, ...; each pair's merged
// order is written back over the pair, the lower tile receiving the smaller
// half.  Keys alone are compared and on equal keys the lower tile's record
// goes first: records of equal key keep their relative order through every
// tile sort and merge (a stable step on a contiguous window), so the lower
// tile's copies always carry the smaller indices and this is the (key,
// index) order.
//
// Work split: the outputs of a phase are cut into slots of E consecutive
// positions; 2T is a multiple of E, so a slot lies inside one pair.  A
// slot finds its start on the pair's merge path by binary search, then
// merges E outputs with one dependent LDS read each.  Each thread owns S
// slots (independent chains), stages their outputs in registers, and
// writes them after a barrier.

// The merges compare records by their key dwords (all but the last, the
// index).  FULL: by all D dwords, for records whose key and position share
// the dwords (two-dword records of 5- and 6-byte words, below).
template <int D, bool FULL = false>
__device__ __forceinline__ void lds_key(const uint32_t* lds, int cap, int i, uint32_t (&x)[D]) {
    const int a = lsw(i);
#pragma unroll
    for (int d = 0; d < (FULL ? D : D - 1); ++d) x[d] = lds[d * cap + a];
    if (!FULL) x[D - 1] = 0;
}

template <int D, bool FULL>
__device__ __forceinline__ bool rec_gt(const uint32_t (&a)[D], const uint32_t (&b)[D]) {
    if constexpr (!FULL) {
        return key_gt<D>(a, b);
    } else {
        uint32_t x[D + 1], y[D + 1];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            x[d] = a[d];
            y[d] = b[d];
        }
        x[D] = y[D] = 0;
        return key_gt<D + 1>(x, y);
    }
}

// number of the first `diag` outputs of the pair (lower tile at lo, T
// records; upper at lo+T, nb records) that come from the lower tile: the
// number of lower records i with lower[i] <= upper[diag-1-i] (this predicate
// holds on a prefix).  Shrinking-length search, a fixed trip count (T <=
// 2^logT), no branches; while len > 0 both probes lie inside their tiles.
template <int D, bool FULL = false>
__device__ __forceinline__ int lds_merge_path(const uint32_t* lds, int cap, int lo, int T,
                                              int logT, int nb, int diag) {
    int base = diag - nb > 0 ? diag - nb : 0;
    int len = (diag < T ? diag : T) - base;
    const int bq = lo + T + diag - 1;                  // upper index = bq - i
    for (int it = 0; it <= logT; ++it) {
        const int half = len >> 1;
        const int i = base + half;
        uint32_t x[D], y[D];
        lds_key<D, FULL>(lds, cap, lo + i, x);
        lds_key<D, FULL>(lds, cap, bq - i, y);
        const bool take = len > 0 && !rec_gt<D, FULL>(x, y); // lower[i] <= upper[diag-1-i]
        base = take ? i + 1 : base;
        len = take ? len - half - 1 : half;
    }
    return base;
}

// E outputs of the pair starting at output `diag`; positions are absolute:
// lower tile [lo, ea), upper tile [ea, eb), eb <= n
// (at most e <= E of them: e is uniform over the wave)
template <int D, int E, bool FULL = false>
__device__ __forceinline__ void lds_merge_slot(const uint32_t* lds, int cap, int n, int lo,
                                               int T, int logT, int nb, int diag,
                                               uint32_t (&out)[E][D], int e = E) {
    const int ia0 = lds_merge_path<D, FULL>(lds, cap, lo, T, logT, nb, diag);
    const int ea = lo + T, eb = ea + nb;
    int pa = lo + ia0, pb = ea + (diag - ia0);
    uint32_t ca[D], cb[D];
    lds_rec<D>(lds, cap, pa < n ? pa : n - 1, ca);
    lds_rec<D>(lds, cap, pb < n ? pb : n - 1, cb);
#pragma unroll
    for (int j = 0; j < E; ++j) {
        if (j < e) {
            // the lower tile's record goes first unless it is exhausted or larger
            const bool take_a = (pb >= eb) | ((pa < ea) & !rec_gt<D, FULL>(ca, cb));
            const uint32_t m = take_a ? 0xFFFFFFFFu : 0u;
#pragma unroll
            for (int d = 0; d < D; ++d) out[j][d] = cb[d] ^ ((ca[d] ^ cb[d]) & m);
            pa += take_a ? 1 : 0;
            pb += take_a ? 0 : 1;
            int nx = take_a ? pa : pb;
            nx = nx < n ? nx : n - 1;        // past the end: any record, never taken
            uint32_t x[D];
            lds_rec<D>(lds, cap, nx, x);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                ca[d] = ca[d] ^ ((x[d] ^ ca[d]) & m);
                cb[d] = x[d] ^ ((cb[d] ^ x[d]) & m);
            }
        }
    }
}

// outputs per slot: the largest power of two <= min(8, CAP/NT)
__host__ __device__ constexpr int merge_slot_outputs(int cap, int nt) {
    const int q = cap / nt;
    return q >= 8 ? 8 : q >= 4 ? 4 : 2;
}

// Count of records r[0..m) (sorted by key) that come before x: keys <= x
// when le, keys < x otherwise.  The predicate holds on a prefix, so each
// round probes the last record of 64 equal cells (one per lane) of the
// range still open and a ballot's popcount says how many whole cells lie
// inside the prefix; the next round searches the first cell that does not.
// T is a power of two >= m; rounds: ceil(log64 T), at least one.
template <int D, bool FULL = false>
__device__ __forceinline__ int wave_count_before(const uint32_t* lds, int cap, int at, int m,
                                                 int T, const uint32_t (&x)[D], bool le,
                                                 int lane) {
    auto pred = [&](int i) -> bool {
        uint32_t y[D];
        lds_key<D, FULL>(lds, cap, at + (i < m ? i : m - 1), y);
        const bool before = le ? !rec_gt<D, FULL>(y, x) : rec_gt<D, FULL>(x, y);
        return i < m && before;
    };
    int base = 0;
    for (int step = T >> 6;; step >>= 6) {                // uniform trip count
        const int st = step > 0 ? step : 1;
        base += __popcll(__ballot(pred(base + (lane + 1) * st - 1))) * st;
        if (st == 1) break;
    }
    return base;
}

// per-phase window table in LDS (merge_win_words ints), owned by the kernel
constexpr int kMaxPairs = 64;                              // 16320 / 128 / 2, rounded up
constexpr int kMergeWinWords = 4 * kMaxPairs + 1;

// WIN: trim each pair to its changing window first (two ballot searches and
// two barriers per phase; pays off where pairs are many and long)
template <int D, int NT, int CAP, bool WIN, bool FULL = false>
__device__ void lds_merge_phase(uint32_t* lds, int n, int T, int logT, int p, int s, int tid,
                                int* win) {
    constexpr int E = merge_slot_outputs(CAP, NT);        // outputs per slot
    constexpr int S = (CAP + NT * E - 1) / (NT * E);      // slots per thread
    constexpr int NW = NT / kWave;
    static_assert(CAP / 128 / 2 <= kMaxPairs, "pairs per phase");
    int* wlo = win;
    int* wna = win + kMaxPairs;
    int* wnb = win + 2 * kMaxPairs;
    int* slot0 = win + 3 * kMaxPairs;
    const int off = s & 1;
    if (p - 2 < off) return;                              // no pair in this phase (uniform)
    const int np = (p - 2 - off) / 2 + 1;                 // pairs a = off, off+2, ...
    const int lane = tid & 63, wv = tid >> 6;

    int total = NT * S + 1;                               // full pairs unless windowed
    if constexpr (WIN) {
        // 1. the window of each pair that changes: the lower tile's records above
        // the upper tile's first key and the upper tile's records below the lower
        // tile's last key (equal keys: lower tile first).  Records left of it stay.
        for (int k = wv; k < np; k += NW) {
            const int lo = (off + 2 * k) << logT;
            const int nb = n - lo - T < T ? n - lo - T : T;
            uint32_t b0[D], alast[D];
            lds_key<D, FULL>(lds, CAP, lo + T, b0);
            lds_key<D, FULL>(lds, CAP, lo + T - 1, alast);
            const int j0 = wave_count_before<D, FULL>(lds, CAP, lo, T, T, b0, true, lane);
            const int j1 = wave_count_before<D, FULL>(lds, CAP, lo + T, nb, T, alast, false, lane);
            if (lane == 0) {
                const bool moves = rec_gt<D, FULL>(alast, b0);
                wlo[k] = lo + j0;
                wna[k] = moves ? T - j0 : 0;
                wnb[k] = moves ? j1 : 0;
            }
        }
        __syncthreads();
        if (wv == 0) {                                    // slots per pair, exclusive scan
            const int w = lane < np ? wna[lane] + wnb[lane] : 0;
            const int v = (w + E - 1) / E;
            const int incl = wave_incl_scan(v, lane);
            if (lane < np) slot0[lane] = incl - v;
            if (lane == 63) slot0[np] = incl;
        }
        __syncthreads();
        total = slot0[np];
    }
    uint32_t out[S][E][D];
    int pos[S], cnt[S];

    if (total <= NT * S) {
        // 2. merge the windows only
#pragma unroll
        for (int r = 0; r < S; ++r) {
            const int q = tid + r * NT;
            cnt[r] = 0;
            pos[r] = 0;
            if (q < total) {
                int k = 0;                                // pair of slot q
                for (int h = kMaxPairs / 2; h > 0; h >>= 1)
                    if (k + h < np && slot0[k + h] <= q) k += h;
                const int na = wna[k], nbw = wnb[k];
                const int diag = (q - slot0[k]) * E;
                pos[r] = wlo[k] + diag;
                cnt[r] = na + nbw - diag < E ? na + nbw - diag : E;
                lds_merge_slot<D, E, FULL>(lds, CAP, n, wlo[k], na, logT, nbw, diag, out[r]);
            }
        }
    } else {
        // (per-pair rounding overflowed the slots: merge whole pairs)
        const int a_last = off + 2 * (np - 1);
        const int U0 = off * T;
        const int U1 = (a_last + 2) * T < n ? (a_last + 2) * T : n;
#pragma unroll
        for (int r = 0; r < S; ++r) {
            pos[r] = U0 + (tid + r * NT) * E;
            cnt[r] = U1 - pos[r] < E ? U1 - pos[r] : E;
            if (pos[r] < U1) {
                const int a = off + (((pos[r] - U0) >> (logT + 1)) << 1);   // pair's lower tile
                const int lo = a << logT;
                const int nb = n - lo - T < T ? n - lo - T : T;
                lds_merge_slot<D, E, FULL>(lds, CAP, n, lo, T, logT, nb, pos[r] - lo, out[r]);
            }
        }
    }
    __syncthreads();                                      // every read of this phase is done
#pragma unroll
    for (int r = 0; r < S; ++r) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
            if (j < cnt[r]) {
                const int a = lsw(pos[r] + j);
#pragma unroll
                for (int d = 0; d < D; ++d) lds[d * CAP + a] = out[r][j][d];
            }
        }
    }
    __syncthreads();
}

// One merge-split phase with each pair owned by one wave (tiles of at most
// kLdsMaxTile records, so a pair's window gives each lane at most
// kWaveRunMax outputs).  The wave finds the pair's window (as above), gives
// each lane an equal run of its outputs, and writes them back once all its
// lanes have read: a wave's LDS operations complete in order and pairs are
// disjoint, so one barrier ends the phase.
constexpr int kWaveRunMax = 2 * kLdsMaxTile / kWave;

template <int D, int NT, int CAP, bool FULL = false>
__device__ void lds_merge_phase_waves(uint32_t* lds, int n, int T, int logT, int p, int s,
                                      int tid) {
    constexpr int NW = NT / kWave;
    const int off = s & 1;
    if (p - 2 < off) return;                              // no pair in this phase (uniform)
    const int np = (p - 2 - off) / 2 + 1;                 // pairs a = off, off+2, ...
    const int lane = tid & 63, wv = tid >> 6;
    for (int k = wv; k < np; k += NW) {                   // uniform over the wave
        const int lo = (off + 2 * k) << logT;
        const int nb = n - lo - T < T ? n - lo - T : T;
        uint32_t b0[D], alast[D];
        lds_key<D, FULL>(lds, CAP, lo + T, b0);
        lds_key<D, FULL>(lds, CAP, lo + T - 1, alast);
        if (!rec_gt<D, FULL>(alast, b0)) continue;       // already in order across the seam
        const int j0 = wave_count_before<D, FULL>(lds, CAP, lo, T, T, b0, true, lane);
        const int j1 = wave_count_before<D, FULL>(lds, CAP, lo + T, nb, T, alast, false, lane);
        const int wlo = lo + j0, na = T - j0;
        const int m = na + j1;                            // window outputs, <= 2T
        const int e = (m + kWave - 1) / kWave;            // per lane, <= kWaveRunMax
        const int diag = lane * e;
        const int cnt = m - diag < e ? (m - diag > 0 ? m - diag : 0) : e;
        // a merge-path search range never exceeds the shorter side (>= 1
        // here): bit_length of it rounds suffice
        const int logw = 31 - __builtin_clz((unsigned)(na < j1 ? na : j1));
        uint32_t out[kWaveRunMax][D];
        if (cnt > 0) lds_merge_slot<D, kWaveRunMax, FULL>(lds, CAP, n, wlo, na, logw, j1, diag,
                                                           out, e);
#pragma unroll
        for (int j = 0; j < kWaveRunMax; ++j) {
            if (j < cnt) {
                const int a = lsw(wlo + diag + j);
#pragma unroll
                for (int d = 0; d < D; ++d) lds[d * CAP + a] = out[j][d];
            }
        }
    }
    __syncthreads();
}

// all p phases of a sub-array in LDS: pairs owned by waves in the classes
// of 8,192 words and more, slots spread over the workgroup below that
template <int D, int NT, int CAP, bool FULL = false>
__device__ __forceinline__ void lds_merge_all(uint32_t* lds, int n, int T, int logT, int p,
                                              int tid, int* win) {
    for (int s = 0; s < p; ++s) {
        if constexpr (CAP >= 8192)
            lds_merge_phase_waves<D, NT, CAP, FULL>(lds, n, T, logT, p, s, tid);
        else
            lds_merge_phase<D, NT, CAP, false, FULL>(lds, n, T, logT, p, s, tid, win);
    }
}

// One sub-array (or chunk) bk, n <= CAP words, sorted by one workgroup in
// LDS: load, tile sorts, merge-split phases, write back.  Ends with a
// barrier, so the LDS can take the next entry.
template <int D, int NT, int CAP>
__device__ __forceinline__ void lds_sort_entry(const Job* __restrict__ J, const LBucket& bk,
                                               uint32_t* lds, int* mwin, int T, int logT,
                                               bool tiles_only, int tid) {
    constexpr int NW = NT / kWave;
    constexpr int Dk = D - 1, W = (Dk + 1) / 2;
    constexpr int KCAP = kmax_for(D) < kLdsMaxTile / kWave ? kmax_for(D) : kLdsMaxTile / kWave;
    const int lane = tid & 63, wv = tid >> 6;
    const int n = bk.n_b;                              // n <= CAP (checked when listed)
    const int64_t ks = bk.stride;                      // key lane stride
    const gptr<uint64_t> keys = gp(J->keys) + bk.key_off;
    const gptr<int32_t> perm = gp(J->perm) + bk.pos0;
    // 5- and 6-byte words whose keys are not written back: a record is
    // the two key dwords with the word's position (n <= CAP < 2^16) in
    // the zero low half of the second, compared whole; the index plane
    // keeps input order and is read at that position at the end
    const bool full2 = D == 3 && bk.L <= 6 && !bk.wk;    // uniform
    // 1- and 2-byte words likewise: one dword, the key's high half and
    // the position (n <= CAP <= 2^16) in the zero low half
    const bool full1 = D == 2 && bk.L <= 2 && !bk.wk;    // uniform
#pragma unroll 4
    for (int i = tid; i < n; i += NT) {
        const int a = lsw(i);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t v = keys[w * ks + i];
            lds[(2 * w) * CAP + a] = (uint32_t)(v >> 32) | (full1 ? i : 0);
            if (2 * w + 1 < Dk) lds[(2 * w + 1) * CAP + a] = (uint32_t)v | (full2 ? i : 0);
        }
        lds[Dk * CAP + a] = (uint32_t)perm[i];     // index plane (unused by full1/2 sorts)
    }
    __syncthreads();
    const int p = (n + T - 1) / T;
    for (int t = wv; t < p; t += NW) {
        const int t0 = t * T;
        const int tn = n - t0 < T ? n - t0 : T;
        LdsTile src{lds, CAP, t0, tn};
        if constexpr (D == 3) {
            if (full2) {
                sort_tile_full2_k<2, KCAP>(src, tn, lane, (tn + kWave - 1) / kWave);
                continue;
            }
        }
        if constexpr (D == 2) {
            if (full1) {
                sort_tile_full1_k<2, KCAP>(src, tn, lane, (tn + kWave - 1) / kWave);
                continue;
            }
            if (bk.L == 3) {
                sort_tile_pack3_k<2, KCAP>(src, tn, lane, (tn + kWave - 1) / kWave);
                continue;
            }
        }
        sort_tile_any<D, KCAP>(src, tn, lane);
    }
    __syncthreads();
    if constexpr (D == 3) {
        if (full2) {
            if (!tiles_only) lds_merge_all<2, NT, CAP, true>(lds, n, T, logT, p, tid, mwin);
            // each output's index from the index plane, at the position
            // the record carries (that plane is never written while sorting)
            for (int i = tid; i < n; i += NT)
                perm[i] = (int32_t)lds[2 * CAP + lsw((int)(lds[CAP + lsw(i)] & 0xFFFFu))];
            __syncthreads();                       // LDS reused by the next sub-array
            return;
        }
    }
    if constexpr (D == 2) {
        if (full1) {
            if (!tiles_only) lds_merge_all<1, NT, CAP, true>(lds, n, T, logT, p, tid, mwin);
            // each output's index from the index plane, at the position
            // the record carries (that plane is never written while sorting)
            for (int i = tid; i < n; i += NT)
                perm[i] = (int32_t)lds[CAP + lsw((int)(lds[lsw(i)] & 0xFFFFu))];
            __syncthreads();                       // LDS reused by the next sub-array
            return;
        }
    }
    if (!tiles_only) lds_merge_all<D, NT, CAP>(lds, n, T, logT, p, tid, mwin);
    for (int i = tid; i < n; i += NT) {
        const int a = lsw(i);
        perm[i] = (int32_t)lds[Dk * CAP + a];
        if (bk.wk) {
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t hi = lds[(2 * w) * CAP + a];
                const uint64_t lo = 2 * w + 1 < Dk ? lds[(2 * w + 1) * CAP + a] : 0u;
                keys[w * ks + i] = (hi << 32) | lo;
            }
        }
    }
    __syncthreads();                                   // LDS reused by the next sub-array
}

template <int D, int NT, int CAP>
__global__ __launch_bounds__(NT) void k_bucket_lds(const Job* __restrict__ J, int list) {
    __shared__ uint32_t lds[D * CAP];
    __shared__ int mwin[1];                            // (window tables: pair merges only)
    static_assert(D * CAP * 4 <= kLdsBytes, "sub-array does not fit the LDS budget");
    static_assert(CAP % 64 == 0, "lsw permutes whole rows of 64 records");
    const int tid = threadIdx.x;
    // list < kLdsClasses: the sub-arrays of that size class; list ==
    // kLdsClasses: chunks of sub-arrays that are merged through HBM next
    // a size class's list: entries [0, front) from the front, the rest from
    // the back in reverse, taken one at a time through a counter (larger
    // sub-arrays first, each workgroup taking the next when it is free);
    // chunks merged through HBM next: strided over the grid
    int64_t cnt, front;
    const LBucket* lst;
    int32_t* take = nullptr;
    if (list < kLdsClasses) {
        const int slot = D * kLdsClasses + list;
        const int64_t nf = J->lb_count[slot], nk = J->lb_back[slot];
        front = nf < J->lb_cap ? nf : J->lb_cap;
        cnt = nf + nk < J->lb_cap ? nf + nk : J->lb_cap;
        lst = J->lbuckets + slot * J->lb_cap;
        take = J->lb_take + slot;
    } else {
        cnt = J->hc_count[D] < J->tile_cap[D] ? J->hc_count[D] : J->tile_cap[D];
        front = cnt;
        lst = J->hchunks[D];
    }
    __shared__ int next_entry;
    const bool tiles_only = (J->flags & kFlagTilesOnly) != 0;
    const bool fixed = tiles_only || (J->flags & kFlagLdsTile);
    const int T = fixed ? J->tile_keys[D] : lds_tile(J->tile_keys[D], CAP, D);
    const int logT = 31 - __builtin_clz(T);               // tile sizes are powers of two
    for (int64_t it = 0;; ++it) {
        int64_t bi;
        if (take) {                                       // uniform
            // every pass ends with a barrier, so all threads have read the
            // previous entry before thread 0 writes the next
            if (tid == 0)
                next_entry = __hip_atomic_fetch_add(gp(take), 1, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            bi = next_entry;
        } else {
            bi = blockIdx.x + it * gridDim.x;
        }
        if (bi >= cnt) break;
        const LBucket bk = lst[bi < front ? bi : J->lb_cap - 1 - (bi - front)];
        lds_sort_entry<D, NT, CAP>(J, bk, lds, mwin, T, logT, tiles_only, tid);
    }
}

// Plain per-bucket form: one launch for one sub-array sorted in LDS (one
// workgroup), or for the nchunks chunks of one sub-array merged through HBM
// (workgroup b takes chunk b: words [b*C, min(n, (b+1)*C)) of the
// sub-array), with the batched form's per-entry sort.
template <int D, int NT, int CAP>
__global__ __launch_bounds__(NT) void k_bucket_lds_one(const Job* __restrict__ J, LBucket bk,
                                                       int chunk) {
    __shared__ uint32_t lds[D * CAP];
    __shared__ int mwin[1];
    const bool tiles_only = (J->flags & kFlagTilesOnly) != 0;
    const bool fixed = tiles_only || (J->flags & kFlagLdsTile);
    const int T = fixed ? J->tile_keys[D] : lds_tile(J->tile_keys[D], CAP, D);
    const int logT = 31 - __builtin_clz(T);
    if (chunk > 0) {                                   // chunks of a sub-array merged later
        const int64_t c0 = (int64_t)blockIdx.x * chunk;
        bk.pos0 += c0;
        bk.key_off += c0;
        bk.n_b = bk.stride - c0 < chunk ? (int)(bk.stride - c0) : chunk;
    }
    lds_sort_entry<D, NT, CAP>(J, bk, lds, mwin, T, logT, tiles_only, threadIdx.x);
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

// workgroups of an in-LDS class that can be resident at once: 256 CUs times
// the workgroups whose LDS fits a CU's 160 KiB (at most 4); a larger grid
// only adds dispatches, the kernel strides over its list
template <int D, int C>
constexpr int64_t lds_resident_groups() {
    int per_cu = (160 * 1024) / (D * 4 * lds_cap(C, D));
    if (per_cu > 4) per_cu = 4;
    if (per_cu < 1) per_cu = 1;
    return 256 * per_cu;
}

template <int D, int C>
static void launch_lds_class_t(const Job* J, int64_t grid, int list, hipStream_t s) {
    if constexpr (lds_fits(D, C)) {
        constexpr int64_t gmax = lds_resident_groups<D, C>();
        int64_t g = grid < gmax ? grid : gmax;
        if (g < 1) g = 1;
        k_bucket_lds<D, lds_threads(C, D), lds_cap(C, D)><<<(unsigned)g, lds_threads(C, D), 0, s>>>(J, list);
    }
}

using LdsLauncher = void (*)(const Job*, int64_t, int, hipStream_t);
#define BSORT_LDS_ROW(D) \
    {launch_lds_class_t<D, 0>, launch_lds_class_t<D, 1>, launch_lds_class_t<D, 2>, \
     launch_lds_class_t<D, 3>, launch_lds_class_t<D, 4>}
static const LdsLauncher kLdsLaunchers[kLdsMaxD + 1][kLdsClasses] = {
    {}, {}, BSORT_LDS_ROW(2), BSORT_LDS_ROW(3), BSORT_LDS_ROW(4), BSORT_LDS_ROW(5),
    BSORT_LDS_ROW(6), BSORT_LDS_ROW(7), BSORT_LDS_ROW(8), BSORT_LDS_ROW(9)};
#undef BSORT_LDS_ROW

template <int D, int C>
static void launch_lds_one_t(const Job* J, const LBucket& bk, int nchunks, int chunk,
                             hipStream_t s) {
    if constexpr (lds_fits(D, C))
        k_bucket_lds_one<D, lds_threads(C, D), lds_cap(C, D)>
            <<<(unsigned)nchunks, lds_threads(C, D), 0, s>>>(J, bk, chunk);
}

using LdsOneLauncher = void (*)(const Job*, const LBucket&, int, int, hipStream_t);
#define BSORT_LDS_ONE_ROW(D) \
    {launch_lds_one_t<D, 0>, launch_lds_one_t<D, 1>, launch_lds_one_t<D, 2>, \
     launch_lds_one_t<D, 3>, launch_lds_one_t<D, 4>}
static const LdsOneLauncher kLdsOneLaunchers[kLdsMaxD + 1][kLdsClasses] = {
    {}, {}, BSORT_LDS_ONE_ROW(2), BSORT_LDS_ONE_ROW(3), BSORT_LDS_ONE_ROW(4),
    BSORT_LDS_ONE_ROW(5), BSORT_LDS_ONE_ROW(6), BSORT_LDS_ONE_ROW(7), BSORT_LDS_ONE_ROW(8),
    BSORT_LDS_ONE_ROW(9)};
#undef BSORT_LDS_ONE_ROW

hipError_t launch_lds_one(const Job* J, int D, int c, const LBucket& bk, int nchunks, int chunk,
                          hipStream_t s) {
    if (D < 2 || D > kLdsMaxD || c < 0 || c >= kLdsClasses || !lds_fits(D, c) || nchunks < 1)
        return hipErrorInvalidValue;
    kLdsOneLaunchers[D][c](J, bk, nchunks, chunk, s);
    return hipGetLastError();
}

hipError_t launch_lds_class(const Job* J, const Bounds& b, int D, int c, hipStream_t s) {
    if (D < 2 || D > kLdsMaxD || c < 0 || c >= kLdsClasses) return hipErrorInvalidValue;
    if (!lds_fits(D, c)) return hipSuccess;
    kLdsLaunchers[D][c](J, b.lb_cap, c, s);
    return hipGetLastError();
}

hipError_t launch_lds_buckets(const Job* J, const Bounds& b, int D, hipStream_t s) {
    for (int c = 0; c < kLdsClasses; ++c) {
        hipError_t e = launch_lds_class(J, b, D, c, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// chunks of sub-arrays merged through HBM, sorted by the in-LDS kernel of
// class b.hbm_class[D] (keys written back for the merges)
hipError_t launch_hbm_chunks(const Job* J, const Bounds& b, int D, hipStream_t s) {
    if (D < 2 || D > kLdsMaxD) return hipErrorInvalidValue;
    const int c = b.hbm_class[D];
    if (c < 0 || !lds_fits(D, c)) return hipSuccess;
    kLdsLaunchers[D][c](J, b.tile_cap, kLdsClasses, s);
    return hipGetLastError();
}

// ---- merge-split through HBM: every phase of every sub-array in one launch
//
// The work items and their order are those of merge_sched.h.  k_merge_plan
// (one workgroup) builds the order's tables from the sub-arrays the tile
// plan listed; k_merge_sched's workgroups then take items one at a time,
// wait until the items that last merged their two tiles are done (a phase
// counter per tile), merge the pair in LDS and advance both tiles' counters.

// records a pair merge of width D holds in LDS: two tiles of the HBM tile
// size (chunk size for in-LDS widths, a register tile's size otherwise)
__host__ __device__ constexpr int pair_cap(int D) {
    return 2 * (D <= kLdsMaxD ? hbm_chunk_max(D) : kWave * kmax_for(D));
}
constexpr int kPairThreads = 512;
constexpr int kPlanThreads = 1024;

// Tiles a and a+1 of sub-array m (both sorted) merged in LDS and written
// back in place, the lower tile receiving the smaller half: one phase of
// the in-LDS merge-split over a two-tile array.
template <int D>
__device__ void merge_pair_lds(const Job* __restrict__ J, const MSub& m, int a, uint32_t* lds,
                               int* sflag, int* win, int tid) {
    constexpr int CAP2 = pair_cap(D);
    static_assert(CAP2 * 4 * D <= kLdsBytes - 4 * (kMergeWinWords + 1), "pair merge LDS");
    static_assert(CAP2 % 64 == 0, "lsw permutes whole rows of 64 records");
    constexpr int Dk = D - 1, W = (Dk + 1) / 2;
    const int T = m.T;                                 // power of two, 2T <= CAP2
    const int logT = 31 - __builtin_clz(T);
    const int64_t lo = (int64_t)a * T;
    const int rest = m.n_b - (a + 1) * T;
    const int nb = rest < T ? rest : T;
    const int tot = T + nb;
    const int64_t ks = m.n_b;
    const gptr<uint64_t> keys = gp(J->keys) + m.key_off + lo;
    const gptr<int32_t> perm = gp(J->perm) + m.pos0 + lo;
    if (tid == 0) {                                    // in order across the seam: no moves
        int gt = 0;
        for (int w = 0; w < W; ++w) {
            const uint64_t x = keys[w * ks + T - 1], y = keys[w * ks + T];
            if (x != y) {
                gt = x > y;
                break;
            }
        }
        *sflag = gt;
    }
    __syncthreads();
    if (*sflag == 0) return;                           // uniform
#pragma unroll 4
    for (int i = tid; i < tot; i += kPairThreads) {
        const int q = lsw(i);
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t v = keys[w * ks + i];
            lds[(2 * w) * CAP2 + q] = (uint32_t)(v >> 32);
            if (2 * w + 1 < Dk) lds[(2 * w + 1) * CAP2 + q] = (uint32_t)v;
        }
        lds[Dk * CAP2 + q] = (uint32_t)perm[i];
    }
    __syncthreads();
    lds_merge_phase<D, kPairThreads, CAP2, true>(lds, tot, T, logT, 2, 0, tid, win);
    for (int i = tid; i < tot; i += kPairThreads) {
        const int q = lsw(i);
        perm[i] = (int32_t)lds[Dk * CAP2 + q];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t hi = lds[(2 * w) * CAP2 + q];
            const uint64_t lo32 = 2 * w + 1 < Dk ? lds[(2 * w + 1) * CAP2 + q] : 0u;
            keys[w * ks + i] = (hi << 32) | lo32;
        }
    }
}

template <int D>
__device__ __forceinline__ void merge_pair_d(const Job* J, const MSub& m, int a, uint32_t* lds,
                                             int* sflag, int* win, int tid, int d) {
    if constexpr (D <= kMaxD) {
        if (d == D) merge_pair_lds<D>(J, m, a, lds, sflag, win, tid);
        else merge_pair_d<D + 1>(J, m, a, lds, sflag, win, tid, d);
    }
}

// Exclusive running sum over n values with the whole workgroup: value i is
// get(i); put(i, sum of values before i).  Each thread takes a contiguous run
// of values.  Returns the total.  sh holds kPlanThreads/64 + 1 entries.
template <class Get, class Put>
__device__ int64_t block_scan(int64_t n, Get get, Put put, int64_t* sh) {
    constexpr int NW = kPlanThreads / kWave;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t per = (n + kPlanThreads - 1) / kPlanThreads;
    const int64_t a = (int64_t)tid * per < n ? (int64_t)tid * per : n;
    const int64_t b = a + per < n ? a + per : n;
    int64_t sum = 0;
    for (int64_t i = a; i < b; ++i) sum += get(i);
    const int64_t incl = wave_incl_scan(sum, lane);
    if (lane == kWave - 1) sh[wv] = incl;
    __syncthreads();
    if (tid == 0) {
        int64_t run = 0;
        for (int w = 0; w < NW; ++w) {
            const int64_t t = sh[w];
            sh[w] = run;
            run += t;
        }
        sh[NW] = run;
    }
    __syncthreads();
    int64_t run = sh[wv] + incl - sum;
    for (int64_t i = a; i < b; ++i) {
        const int64_t v = get(i);
        put(i, run);
        run += v;
    }
    const int64_t total = sh[NW];
    __syncthreads();                                   // sh is reused by the next scan
    return total;
}

// The order's tables (merge_sched.h) from the sub-arrays the tile plan
// listed; one workgroup.  Also clears the tile phase counters and the item
// counter.
__global__ __launch_bounds__(kPlanThreads) void k_merge_plan(const Job* __restrict__ J) {
    __shared__ int64_t sh[kPlanThreads / kWave + 1];
    const int tid = threadIdx.x;
    int64_t H = J->mcounts[0];
    H = H < J->msub_cap ? H : J->msub_cap;
    const int P = J->pmax[0] < J->phase_cap ? J->pmax[0] : J->phase_cap;
    int64_t ntiles = J->mcounts[1];
    ntiles = ntiles < J->mtile_cap ? ntiles : J->mtile_cap;
    const gptr<int32_t> cnt = gp(J->pcnt), fill = gp(J->pfill), act = gp(J->active);
    const gptr<int64_t> pe = gp(J->pe), po = gp(J->po), ps = gp(J->ps);
    const MSub* msub = J->msub;
    MSub* sorted = J->msorted;
    if (H == 0 || P < 2) {
        if (tid == 0) J->mhead[1] = 0;
        return;
    }
    for (int64_t i = tid; i < ntiles; i += kPlanThreads) J->tile_ph[i] = 0;
    for (int i = tid; i <= P + 1; i += kPlanThreads) {
        cnt[i] = 0;
        fill[i] = 0;
    }
    __syncthreads();
    // an entry's tile count, or 0 (no work) for one that does not fit the tables
    auto tiles_of = [&](const MSub& m) -> int {
        return m.p >= 2 && m.p <= P && m.tile_base >= 0 && m.tile_base + m.p <= ntiles ? m.p : 0;
    };
    for (int64_t h = tid; h < H; h += kPlanThreads) atomicAdd((int32_t*)&cnt[tiles_of(msub[h])], 1);
    __syncthreads();
    // active[s]: sub-arrays of more than s tiles (a running sum from the top)
    block_scan(P + 1, [&](int64_t j) -> int64_t { return cnt[P - j]; },
               [&](int64_t j, int64_t v) { act[P - j] = (int32_t)v; }, sh);
    // sub-arrays in order of decreasing tile count: those with more tiles first
    for (int64_t h = tid; h < H; h += kPlanThreads) {
        MSub m = msub[h];
        m.p = tiles_of(m);
        const int64_t at = act[m.p] + atomicAdd((int32_t*)&fill[m.p], 1);
        sorted[at] = m;
    }
    __syncthreads();
    const int64_t te = block_scan(H, [&](int64_t i) -> int64_t { return sorted[i].p / 2; },
                                  [&](int64_t i, int64_t v) { pe[i] = v; }, sh);
    const int64_t to = block_scan(H, [&](int64_t i) -> int64_t { return (sorted[i].p - 1) / 2; },
                                  [&](int64_t i, int64_t v) { po[i] = v; }, sh);
    if (tid == 0) {
        pe[H] = te;
        po[H] = to;
    }
    __syncthreads();
    const int64_t items = block_scan(
        P, [&](int64_t s) -> int64_t { return (s & 1) ? po[act[s]] : pe[act[s]]; },
        [&](int64_t s, int64_t v) { ps[s] = v; }, sh);
    if (tid == 0) {
        ps[P] = items;
        J->mhead[1] = items;
    }
}

// Waits until tile counter f reaches need.  The counter is polled with
// relaxed loads (no cache invalidation per poll: with an acquiring load every
// poll would invalidate the XCD's L2 under the workgroups that are merging);
// one acquire fence follows the successful poll.  Bounded: gives up (and sets
// ST_STALLED, which every other wait and every workgroup's next item then
// sees) after J->stall_ticks of the 100 MHz real-time counter, or at once when
// stall_ticks < 0 (a test setting).
__device__ bool wait_tile(const Job* J, gptr<int32_t> f, int need) {
    if (need <= 0) return true;
    if (J->stall_ticks < 0) {
        set_status(J, ST_STALLED);
        return false;
    }
    const uint64_t t0 = wall_clock64();
    // also bounded by the number of polls (each at least 1,024 clocks apart)
    const int64_t max_polls = J->stall_ticks / 8 + 1;
    for (int64_t poll = 0;; ++poll) {
        if (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return true;
        }
        if (__hip_atomic_load(gp(J->status), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
            ST_STALLED)
            return false;
        if (wall_clock64() - t0 > (uint64_t)J->stall_ticks || poll >= max_polls) {
            set_status(J, ST_STALLED);
            return false;
        }
        __builtin_amdgcn_s_sleep(16);
    }
}

// Every merge-split item of every sub-array merged through HBM.  Workgroups
// take items in the order of merge_sched.h until none is left.
__global__ __launch_bounds__(kPairThreads) void k_merge_sched(const Job* __restrict__ J) {
    extern __shared__ uint32_t lds[];
    __shared__ int sflag;
    __shared__ int mwin[kMergeWinWords];
    __shared__ int item[4];                            // phase, sub-array, lower tile, go
    const int tid = threadIdx.x;
    const int64_t N = J->mhead[1];
    if (N <= 0) return;                                // uniform
    const int P = J->pmax[0] < J->phase_cap ? J->pmax[0] : J->phase_cap;
    const gptr<int32_t> tph = gp(J->tile_ph);
    // a workgroup also stops taking items after 4 stall bounds in all, and
    // takes at most N + 1 (the last one ends it)
    const uint64_t t_start = wall_clock64();
    for (int64_t taken = 0; taken <= N; ++taken) {
        if (tid == 0) {
            int go = 0;
            const bool stalled =
                (__hip_atomic_load(gp(J->status), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                 ST_STALLED) != 0;
            if (!stalled && J->stall_ticks >= 0 &&
                wall_clock64() - t_start > 4 * (uint64_t)J->stall_ticks) {
                set_status(J, ST_STALLED);
            } else if (!stalled) {
                const int64_t q = __hip_atomic_fetch_add(gp(J->mhead), (int64_t)1,
                                                         __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                if (q < N) {
                    const MschedItem it = msched_decode(q, gp(J->ps), P, gp(J->active),
                                                        gp(J->pe), gp(J->po));
                    const int p = J->msorted[it.i].p;
                    const int64_t tb = J->msorted[it.i].tile_base;
                    go = wait_tile(J, tph + tb + it.t, (int)msched_prev(it.s, it.t, p) + 1) &&
                         wait_tile(J, tph + tb + it.t + 1,
                                   (int)msched_prev(it.s, it.t + 1, p) + 1);
                    item[0] = it.s;
                    item[1] = it.i;
                    item[2] = it.t;
                }
            }
            item[3] = go;
        }
        __syncthreads();
        if (!item[3]) break;                           // uniform: no item left, or a stall
        const int s = item[0], t = item[2];
        const MSub m = J->msorted[item[1]];
        merge_pair_d<2>(J, m, t, lds, &sflag, mwin, tid, dwords_for_len(m.L));
        // this wave's stores have reached the cache before the barrier; the
        // release below writes the cache back before the counters move
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_store(tph + m.tile_base + t, s + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(tph + m.tile_base + t + 1, s + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gp(J->mhead) + 2, (int64_t)1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Plain per-bucket form: phase s of sub-array m, workgroup b merging the
// pair whose lower tile is s%2 + 2b (the batched form's pair merge).
__global__ __launch_bounds__(kPairThreads) void k_merge_phase_one(const Job* __restrict__ J,
                                                                  MSub m, int s) {
    extern __shared__ uint32_t lds[];
    __shared__ int sflag;
    __shared__ int mwin[kMergeWinWords];
    const int t = (s & 1) + 2 * (int)blockIdx.x;
    if (t + 1 >= m.p) return;                          // uniform
    merge_pair_d<2>(J, m, t, lds, &sflag, mwin, threadIdx.x, dwords_for_len(m.L));
}

hipError_t launch_merge_phase_one(const Job* J, const MSub& m, int phase, int lds_bytes,
                                  hipStream_t s) {
    const int pairs = (m.p - (phase & 1)) / 2;
    if (pairs <= 0) return hipSuccess;
    k_merge_phase_one<<<(unsigned)pairs, kPairThreads, lds_bytes, s>>>(J, m, phase);
    return hipGetLastError();
}

int pair_merge_lds(int dmax) {
    int need = 0;
    for (int D = 2; D <= dmax && D <= kMaxD; ++D) need = std::max(need, pair_cap(D) * 4 * D);
    static bool attr = false;
    if (!attr) {
        for (const void* f : {(const void*)k_merge_sched, (const void*)k_merge_phase_one})
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                      kLdsBytes - 4 * (kMergeWinWords + 1));
        attr = true;
    }
    return need;
}

hipError_t launch_merge_sched(const Job* J, const Bounds& b, hipStream_t s) {
    k_merge_plan<<<1, kPlanThreads, 0, s>>>(J);
    // as many workgroups as stay resident (their LDS decides); each takes
    // items until none is left, so a call with few items ends quickly
    int64_t per_cu = (160 * 1024) / ((int64_t)b.pair_lds + 4 * (kMergeWinWords + 8));
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 4) per_cu = 4;
    k_merge_sched<<<(unsigned)(256 * per_cu), kPairThreads, b.pair_lds, s>>>(J);
    return hipGetLastError();
}

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
