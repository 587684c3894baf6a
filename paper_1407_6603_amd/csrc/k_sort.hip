// Sort side of the path, except the tile sort itself (k_oets.hip):
//
//   k_sort_init   zero the work-list counters
//   k_tile_plan   one wave per list: key-lane offsets of its sub-arrays, the
//                 odd-even transposition tiles of each sub-array, and the
//                 first merge-split phase's work items
//   k_pack        one thread per word: big-endian uint64 key lanes (the
//                 paper's fixed-width word slots, Section III approach two)
//                 and the initial index payload
//   k_merge_phase one workgroup per (sub-array, tile pair) of one phase of
//                 the block odd-even merge-split (Baudet and Stevenson,
//                 1978): tiles a and a+1 of a sub-array, both sorted, are
//                 merged; the lower keeps the smaller half.  p phases sort a
//                 sub-array of p tiles.  Each item also queues its
//                 successors of the next phase.
#include "bsort_internal.h"

namespace bsort {

template <typename T>
__device__ __forceinline__ T wave_incl_scan2(T v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    return v;
}

__device__ __forceinline__ void req_bounds2(const Job* J, int r, int64_t& a, int64_t& b) {
    int64_t x = J->req_start[r], y = J->req_start[r + 1];
    x = x < 0 ? 0 : (x > J->total ? J->total : x);
    y = y < x ? x : (y > J->total ? J->total : y);
    a = x;
    b = y;
}

__global__ __launch_bounds__(256) void k_sort_init(const Job* __restrict__ J) {
    for (int i = threadIdx.x; i < kNumD; i += blockDim.x) J->tile_count[i] = 0;
    for (int i = threadIdx.x; i <= J->phase_cap; i += blockDim.x) J->mcount[i] = 0;
}

__global__ __launch_bounds__(256) void k_tile_plan(const Job* __restrict__ J) {
    __shared__ int64_t kos[kTileWavesPerBlock][kMaxLen + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = blockIdx.x * kTileWavesPerBlock + wv;
    if (r >= J->R) return;
    int64_t a, b;
    req_bounds2(J, r, a, b);
    const int ml1 = J->ml1;
    const int wmax = lanes_for_len(J->max_len);
    const int32_t* cnt = J->counts + (int64_t)r * ml1;
    const int32_t* st = J->starts + (int64_t)r * (ml1 + 1);
    const bool tiles_only = (J->flags & kFlagTilesOnly) != 0;

    // uint64 offset of each sub-array's lane 0: exclusive scan of W(L)*n_L
    int64_t run = (int64_t)wmax * a;
    for (int base = 0; base < ml1; base += kWave) {
        const int L = base + lane;
        int nb = L < ml1 ? cnt[L] : 0;
        if (nb < 0) nb = 0;
        const int64_t v = (int64_t)lanes_for_len(L) * nb;
        const int64_t incl = wave_incl_scan2(v, lane);
        if (L < ml1) {
            const int64_t ko = run + incl - v;
            kos[wv][L] = ko;
            J->key_off[(int64_t)r * ml1 + L] = ko;
        }
        run += __shfl(incl, kWave - 1, kWave);
    }
    __builtin_amdgcn_wave_barrier();

    for (int L = 1; L < ml1; ++L) {                 // uniform over the wave
        const int nb = cnt[L];
        if (nb < 2) continue;                        // 0 or 1 word: already in order
        if (st[L] < 0 || (int64_t)st[L] + nb > b - a) {
            if (lane == 0) set_status(J, ST_BAD_REQ);
            continue;
        }
        const int64_t ko = kos[wv][L];
        if (ko + (int64_t)lanes_for_len(L) * nb > (int64_t)wmax * b) {   // counts inconsistent
            if (lane == 0) set_status(J, ST_BAD_REQ);
            continue;
        }
        const int D = dwords_for_len(L);
        const int T = J->tile_keys[D];
        const int nt = (nb + T - 1) / T;
        int slot = 0;
        if (lane == 0) slot = atomicAdd(&J->tile_count[D], nt);
        slot = __shfl(slot, 0, kWave);
        if ((int64_t)slot + nt > J->tile_cap[D]) {
            if (lane == 0) set_status(J, ST_OVERFLOW);
            continue;
        }
        const int64_t pos0 = a + st[L];
        for (int t = lane; t < nt; t += kWave) {
            TileDesc d;
            d.pos0 = pos0;
            d.key_off = ko;
            d.n_b = nb;
            d.t0 = t * T;
            d.n = nb - t * T < T ? nb - t * T : T;
            d.L = L;
            J->tiles[D][slot + t] = d;
        }
        if (nt >= 2 && !tiles_only) {
            const int np = nt / 2;                   // phase 0 pairs (0,1), (2,3), ...
            int s2 = 0;
            if (lane == 0) s2 = atomicAdd(&J->mcount[0], np);
            s2 = __shfl(s2, 0, kWave);
            if ((int64_t)s2 + np > J->merge_cap) {
                if (lane == 0) set_status(J, ST_OVERFLOW);
                continue;
            }
            for (int k = lane; k < np; k += kWave) {
                MergeItem m;
                m.pos0 = pos0;
                m.key_off = ko;
                m.n_b = nb;
                m.L = L;
                m.T = T;
                m.a = 2 * k;
                m.p = nt;
                m.pad = 0;
                J->mlist[0][s2 + k] = m;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_pack(const Job* __restrict__ J) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= J->total) return;
    const int R = J->R;
    const int r = upper_index(J->req_start, R, q);
    int64_t a, b;
    req_bounds2(J, r, a, b);
    if (q < a || q >= b) return;
    const int ml1 = J->ml1;
    const int32_t* cnt = J->counts + (int64_t)r * ml1;
    const int32_t* st = J->starts + (int64_t)r * (ml1 + 1);
    const int64_t local = q - a;
    if (local >= st[ml1]) return;                    // malformed words were left out
    const int32_t idx = J->order[q];
    if (idx < 0 || idx >= b - a) {
        set_status(J, ST_OVERFLOW);
        return;
    }
    const int64_t g = a + idx;
    const int64_t o0 = J->offsets[g], o1 = J->offsets[g + 1];
    const int64_t len = o1 - o0;
    if (o0 < 0 || len < 0 || len > J->max_len || o1 > J->n_bytes) {
        set_status(J, ST_BAD_OFFSETS);
        return;
    }
    const int L = (int)len;
    const int64_t j = local - st[L];
    const int nb = cnt[L];
    if (j < 0 || j >= nb) {
        set_status(J, ST_BAD_REQ);
        return;
    }
    const int64_t ko = J->key_off[(int64_t)r * ml1 + L];
    const int W = lanes_for_len(L);
    const int wmax = lanes_for_len(J->max_len);
    if (ko < (int64_t)wmax * a || ko + (int64_t)W * nb > (int64_t)wmax * b) {
        set_status(J, ST_BAD_REQ);
        return;
    }
    const uint8_t* p = J->bytes + o0;
    for (int w = 0; w < W; ++w) {
        uint64_t v = 0;
        const int k1 = L - 8 * w < 8 ? L - 8 * w : 8;
        for (int k = 0; k < k1; ++k) v |= (uint64_t)p[8 * w + k] << (56 - 8 * k);
        J->keys[ko + (int64_t)w * nb + j] = v;
    }
    J->perm[q] = idx;
}

// record x > record y, records as SoA dwords in LDS (dword d at lds[d*tot + i])
__device__ __forceinline__ bool lds_gt(const uint32_t* lds, int tot, int D, int x, int y) {
    for (int d = 0; d < D; ++d) {
        const uint32_t u = lds[d * tot + x], v = lds[d * tot + y];
        if (u != v) return u > v;
    }
    return false;
}

// Merge-split of tiles m.a and m.a+1 of one sub-array, in place.
__device__ void merge_pair(const Job* __restrict__ J, const MergeItem& m, bool last_phase,
                           uint32_t* lds, int* sflag) {
    const int D = dwords_for_len(m.L), Dk = D - 1, W = lanes_for_len(m.L);
    const int64_t lo = (int64_t)m.a * m.T;
    const int na = m.T;
    const int rest = m.n_b - (m.a + 1) * m.T;
    const int nb = rest < m.T ? rest : m.T;
    const int tot = na + nb;
    uint64_t* keys = J->keys + m.key_off;
    int32_t* perm = J->perm + m.pos0;
    const int64_t nbk = m.n_b;
    const int tid = threadIdx.x, NT = blockDim.x;

    // already in order across the seam?  then nothing moves
    if (tid == 0) {
        int in_order = -1;
        const int64_t ja = lo + na - 1, jb = lo + na;
        for (int w = 0; w < W && in_order < 0; ++w) {
            const uint64_t x = keys[w * nbk + ja], y = keys[w * nbk + jb];
            if (x != y) in_order = x < y;
        }
        if (in_order < 0) in_order = perm[ja] < perm[jb];
        *sflag = in_order;
    }
    __syncthreads();
    const bool skip = *sflag != 0;
    if (skip) return;                                // uniform

    for (int i = tid; i < tot; i += NT) {
        const int64_t j = lo + i;
        for (int w = 0; w < W; ++w) {
            const uint64_t v = keys[w * nbk + j];
            lds[(2 * w) * tot + i] = (uint32_t)(v >> 32);
            if (2 * w + 1 < Dk) lds[(2 * w + 1) * tot + i] = (uint32_t)v;
        }
        lds[Dk * tot + i] = (uint32_t)perm[j];
    }
    __syncthreads();

    const int E = (tot + NT - 1) / NT;
    const int k0 = tid * E;
    if (k0 < tot) {
        const int k1 = k0 + E < tot ? k0 + E : tot;
        // merge path: how many of the first k0 outputs come from tile a
        int lo_i = k0 - nb > 0 ? k0 - nb : 0;
        int hi_i = k0 < na ? k0 : na;
        while (lo_i < hi_i) {
            const int mid = (lo_i + hi_i) >> 1;
            if (lds_gt(lds, tot, D, na + (k0 - 1 - mid), mid)) lo_i = mid + 1;
            else hi_i = mid;
        }
        int ia = lo_i, ib = k0 - lo_i;
        for (int k = k0; k < k1; ++k) {
            const bool take_a = ib >= nb || (ia < na && lds_gt(lds, tot, D, na + ib, ia));
            const int src = take_a ? ia++ : na + ib++;
            const int64_t jo = lo + k;
            if (!last_phase) {
                for (int w = 0; w < W; ++w) {
                    const uint64_t hi = lds[(2 * w) * tot + src];
                    const uint64_t lw = (2 * w + 1 < Dk) ? lds[(2 * w + 1) * tot + src] : 0u;
                    keys[w * nbk + jo] = (hi << 32) | lw;
                }
            }
            perm[jo] = (int32_t)lds[Dk * tot + src];
        }
    }
}

__device__ __forceinline__ void push_item(const Job* J, int s1, const MergeItem& m) {
    const int slot = atomicAdd(&J->mcount[s1], 1);
    if (slot < J->merge_cap) J->mlist[s1 & 1][slot] = m;
    else set_status(J, ST_OVERFLOW);
}

__global__ __launch_bounds__(1024) void k_merge_phase(const Job* __restrict__ J, int s) {
    extern __shared__ uint32_t lds[];
    __shared__ int sflag;
    if (s >= J->phase_cap) return;
    int cnt = J->mcount[s];
    if (cnt > J->merge_cap) cnt = (int)J->merge_cap;
    const MergeItem* list = J->mlist[s & 1];
    for (int it = blockIdx.x; it < cnt; it += gridDim.x) {
        const MergeItem m = list[it];
        merge_pair(J, m, s == m.p - 1, lds, &sflag);
        if (threadIdx.x == 0 && s + 1 < m.p) {
            // successors: pair (a+1, a+2); after an odd phase also (0, 1)
            if (m.a + 2 < m.p) {
                MergeItem n = m;
                n.a = m.a + 1;
                push_item(J, s + 1, n);
            }
            if ((s & 1) && m.a == 1) {
                MergeItem n = m;
                n.a = 0;
                push_item(J, s + 1, n);
            }
        }
        __syncthreads();                            // LDS and sflag reused by the next item
    }
}

// plain form: one launch per (sub-array, phase); block x takes pair a = (s&1) + 2x
__global__ __launch_bounds__(1024) void k_merge_bucket(const Job* __restrict__ J, MergeItem m,
                                                       int s) {
    extern __shared__ uint32_t lds[];
    __shared__ int sflag;
    m.a = (s & 1) + 2 * (int)blockIdx.x;
    if (m.a + 1 >= m.p) return;
    merge_pair(J, m, s == m.p - 1, lds, &sflag);
}

static inline unsigned grid_for2(int64_t items, int per_block, int64_t cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_pack(const Job* J, const Bounds& b, hipStream_t s) {
    k_pack<<<grid_for2(b.total, 256, 0x7fffffff), 256, 0, s>>>(J);
    return hipGetLastError();
}

hipError_t launch_merge_phase(const Job* J, const Bounds& b, int phase, hipStream_t s) {
    const int64_t merge_cap = b.total / kMinTile + (int64_t)b.R * b.ml1;
    k_merge_phase<<<grid_for2(merge_cap / 2 + 1, 1, 4096), b.merge_threads, b.merge_lds, s>>>(
        J, phase);
    return hipGetLastError();
}

hipError_t launch_merge_one_bucket(const Job* J, const MergeItem& item0, int npairs, int phase,
                                   int merge_threads, int lds, hipStream_t s) {
    if (npairs <= 0) return hipSuccess;
    k_merge_bucket<<<npairs, merge_threads, lds, s>>>(J, item0, phase);
    return hipGetLastError();
}

hipError_t launch_sort_prep(const Job* J, const Bounds& b, hipStream_t s) {
    k_sort_init<<<1, 256, 0, s>>>(J);
    k_tile_plan<<<grid_for2(b.R, kTileWavesPerBlock, 0x7fffffff), 256, 0, s>>>(J);
    return launch_pack(J, b, s);
}

hipError_t launch_merges(const Job* J, const Bounds& b, hipStream_t s) {
    if (b.flags & kFlagTilesOnly) return hipSuccess;
    for (int ph = 0; ph < b.phase_bound; ++ph) {
        hipError_t e = launch_merge_phase(J, b, ph, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sort(const Job* J, const Bounds& b, hipStream_t s) {
    hipError_t e = launch_sort_prep(J, b, s);
    if (e != hipSuccess) return e;
    for (int D = 2; D <= b.dmax && D <= kMaxD; ++D) {
        e = launch_oets_tiles_one(J, b, D, s);
        if (e != hipSuccess) return e;
    }
    e = launch_merges(J, b, s);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

}  // namespace bsort
