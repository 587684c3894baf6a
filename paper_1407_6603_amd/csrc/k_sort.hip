// Sort side of the path, except the tile sort itself (k_oets.hip):
//
//   k_sort_init   zero the work-list counters
//   k_tile_plan   one wave per list, four lists per workgroup: key-lane
//                 offsets of the list's sub-arrays, its odd-even
//                 transposition tiles and the sub-arrays merged through HBM;
//                 list slots are claimed with one global atomic per
//                 workgroup and record width
//   k_pack        one wave per 1,024-word chunk: big-endian uint64 key lanes
//                 (the paper's fixed-width word slots, Section III approach
//                 two) and the initial index payload
#include "bsort_internal.h"

namespace bsort {

__global__ __launch_bounds__(256) void k_sort_init(const Job* __restrict__ J) {
    const int i0 = threadIdx.x;
    if (i0 < kNumD) J->tile_count[i0] = 0;
    if (i0 < kNumD * kLdsClasses) {
        J->lb_count[i0] = 0;
        J->lb_back[i0] = 0;
        J->lb_take[i0] = 0;
    }
    if (i0 <= kLdsMaxD) J->hc_count[i0] = 0;
    if (i0 == 0) J->pmax[0] = 0;
    if (i0 < 2) J->mcounts[i0] = 0;
    if (i0 < 3) J->mhead[i0] = 0;
}

// one wave per list; the workgroup's four waves share one global claim per
// record width D and one for the first merge phase
// device-scope add on a global counter, returning the old value
__device__ __forceinline__ int gadd(int32_t* p, int v) {
    return __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// write_ko: 0 when the bucketize pass of the same call has already written
// key_off (the same values), which its scatter may be reading meanwhile
__global__ __launch_bounds__(256) void k_tile_plan(const Job* __restrict__ J, int write_ko) {
    __shared__ int64_t kos[kTileWavesPerBlock][kMaxLen + 1];
    __shared__ int blk_tiles[kNumD];
    __shared__ int64_t blk_tile_base[kNumD];
    __shared__ int blk_msub, blk_mtiles;
    __shared__ int64_t blk_msub_base, blk_mtile_base;
    constexpr int kLb = kNumD * kLdsClasses;          // front counts, then back counts
    __shared__ int blk_lb[2 * kLb];
    __shared__ int64_t blk_lb_base[2 * kLb];
    __shared__ int blk_hc[kLdsMaxD + 1];
    __shared__ int64_t blk_hc_base[kLdsMaxD + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < kNumD) blk_tiles[tid] = 0;
    if (tid < 2 * kLb) blk_lb[tid] = 0;
    if (tid <= kLdsMaxD) blk_hc[tid] = 0;
    if (tid == 0) {
        blk_msub = 0;
        blk_mtiles = 0;
    }
    __syncthreads();

    const int r = blockIdx.x * kTileWavesPerBlock + wv;
    const bool active = r < J->R;
    const int ml1 = J->ml1;
    const int wmax = lanes_for_len(J->max_len);
    const bool tiles_only = (J->flags & kFlagTilesOnly) != 0;
    int64_t a = 0, b = 0;
    if (active) req_bounds(J, r, a, b);
    const int32_t* cnt = J->counts + (int64_t)(active ? r : 0) * ml1;
    const int32_t* st = J->starts + (int64_t)(active ? r : 0) * (ml1 + 1);

    // per length L = lane + 64*k (k = 0, 1): route, tiles, tile slot, merge slot.
    // route: 0 none, 1 one register tile, 2 whole sub-array in LDS (class lcls),
    // 3 HBM tiles merged phase by phase
    int nt[2] = {0, 0}, tslot[2] = {0, 0}, islot[2] = {0, 0}, mtslot[2] = {0, 0};
    int route[2] = {0, 0}, lcls[2] = {0, 0};
    if (active) {
        int64_t run = (int64_t)wmax * a;    // uint64 offset of each sub-array's lane 0
        for (int k = 0; k < 2; ++k) {
            const int L = lane + kWave * k;
            if (kWave * k >= ml1) break;    // uniform
            int nb = L < ml1 ? cnt[L] : 0;
            if (nb < 0) nb = 0;
            const int64_t v = (int64_t)lanes_for_len(L) * nb;
            const int64_t incl = wave_incl_scan(v, lane);
            const int64_t ko = run + incl - v;
            run += __shfl(incl, kWave - 1, kWave);
            if (L >= ml1) continue;
            kos[wv][L] = ko;
            if (write_ko) J->key_off[(int64_t)r * ml1 + L] = ko;
            if (L == 0 || nb < 2) continue;  // 0 or 1 word: already in order
            if (st[L] < 0 || (int64_t)st[L] + nb > b - a ||
                ko + (int64_t)lanes_for_len(L) * nb > (int64_t)wmax * b) {
                set_status(J, ST_BAD_REQ);  // counts/starts inconsistent with the list
                continue;
            }
            const int D = dwords_for_len(L);
            int c = -1;
            if (nb > J->tile_keys[D])
                for (int q = 0; q < kLdsClasses; ++q)
                    if (c < 0 && lds_fits(D, q) && nb <= lds_cap(q, D)) c = q;
            if (nb <= J->tile_keys[D]) {
                route[k] = 1;
                nt[k] = 1;
                tslot[k] = atomicAdd(&blk_tiles[D], 1);
            } else if (c >= 0) {
                route[k] = 2;
                lcls[k] = c;
                const bool front = lds_class_large(nb, c, D, J->tile_keys[D]);
                tslot[k] = atomicAdd(&blk_lb[(front ? 0 : kLb) + D * kLdsClasses + c], 1);
            } else {
                // merged through HBM: chunks sorted in LDS (D <= kLdsMaxD) or
                // register tiles, then nt merge-split phases
                route[k] = 3;
                const int T = J->hbm_tile_keys[D];
                nt[k] = (nb + T - 1) / T;
                if (D <= kLdsMaxD) tslot[k] = atomicAdd(&blk_hc[D], nt[k]);
                else tslot[k] = atomicAdd(&blk_tiles[D], nt[k]);
                if (nt[k] >= 2 && !tiles_only) {
                    islot[k] = atomicAdd(&blk_msub, 1);
                    mtslot[k] = atomicAdd(&blk_mtiles, nt[k]);
                    __hip_atomic_fetch_max(gp(J->pmax), nt[k], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
    }
    __syncthreads();
    if (tid < kNumD && blk_tiles[tid] > 0)
        blk_tile_base[tid] = gadd(J->tile_count + tid, blk_tiles[tid]);
    if (tid == kNumD && blk_msub > 0) blk_msub_base = gadd(J->mcounts, blk_msub);
    if (tid == kNumD + 1 && blk_mtiles > 0) blk_mtile_base = gadd(J->mcounts + 1, blk_mtiles);
    if (tid < 2 * kLb && blk_lb[tid] > 0)
        blk_lb_base[tid] = gadd(tid < kLb ? J->lb_count + tid : J->lb_back + (tid - kLb),
                                blk_lb[tid]);
    if (tid <= kLdsMaxD && blk_hc[tid] > 0)
        blk_hc_base[tid] = gadd(J->hc_count + tid, blk_hc[tid]);
    __syncthreads();
    if (!active) return;

    for (int k = 0; k < 2; ++k) {
        if (route[k] == 0) continue;
        const int L = lane + kWave * k;
        const int nb = cnt[L];
        const int D = dwords_for_len(L);
        const int64_t pos0 = a + st[L];
        const int64_t ko = kos[wv][L];
        if (route[k] == 2) {
            const int sl = D * kLdsClasses + lcls[k];
            const bool front = lds_class_large(nb, lcls[k], D, J->tile_keys[D]);
            const int64_t at0 = blk_lb_base[(front ? 0 : kLb) + sl] + tslot[k];
            const int64_t at = front ? at0 : J->lb_cap - 1 - at0;
            // front and back together hold at most 4 per list, fewer than lb_cap
            if (at0 >= J->lb_cap) {
                set_status(J, ST_OVERFLOW);
                continue;
            }
            LBucket lb;
            lb.pos0 = pos0;
            lb.key_off = ko;
            lb.n_b = nb;
            lb.L = L;
            lb.stride = nb;
            lb.wk = 0;
            J->lbuckets[sl * J->lb_cap + at] = lb;
            continue;
        }
        const int T = route[k] == 1 ? nb : J->hbm_tile_keys[D];
        const bool chunks = route[k] == 3 && D <= kLdsMaxD;
        const int64_t base = (chunks ? blk_hc_base[D] : blk_tile_base[D]) + tslot[k];
        if (base + nt[k] > J->tile_cap[D]) {
            set_status(J, ST_OVERFLOW);
            continue;
        }
        if (chunks) {
            for (int t = 0; t < nt[k]; ++t) {
                LBucket lb;
                lb.pos0 = pos0 + (int64_t)t * T;
                lb.key_off = ko + (int64_t)t * T;
                lb.n_b = nb - t * T < T ? nb - t * T : T;
                lb.L = L;
                lb.stride = nb;
                lb.wk = 1;
                J->hchunks[D][base + t] = lb;
            }
        } else for (int t = 0; t < nt[k]; ++t) {
            TileDesc d;
            d.pos0 = pos0;
            d.key_off = ko;
            d.n_b = nb;
            d.t0 = t * T;
            d.n = nb - t * T < T ? nb - t * T : T;
            d.L = L;
            J->tiles[D][base + t] = d;
        }
        if (nt[k] < 2 || tiles_only) continue;
        // a sub-array of nt tiles merged through HBM: nt merge-split phases.
        // Every claimed entry inside the list is written (p = 0, no work, if
        // its tiles do not fit the tile table), so the merge plan never reads
        // an entry of an earlier call.
        const int64_t mi = blk_msub_base + islot[k];
        const int64_t tb = blk_mtile_base + mtslot[k];
        const bool fits = tb + nt[k] <= J->mtile_cap;
        if (mi >= J->msub_cap || !fits) set_status(J, ST_OVERFLOW);
        if (mi >= J->msub_cap) continue;
        MSub m;
        m.pos0 = pos0;
        m.key_off = ko;
        m.tile_base = tb;
        m.n_b = nb;
        m.L = L;
        m.T = T;
        m.p = fits ? nt[k] : 0;
        J->msub[mi] = m;
    }
}

__global__ __launch_bounds__(256) void k_pack(const Job* __restrict__ J) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * kTileWavesPerBlock + wv;
    int r;
    int64_t a, b, gs, ge;
    if (!chunk_range(J, c, r, a, b, gs, ge)) return;
    const int ml1 = J->ml1;
    const int32_t* cnt = J->counts + (int64_t)r * ml1;
    const int32_t* st = J->starts + (int64_t)r * (ml1 + 1);
    const int64_t* ko_r = J->key_off + (int64_t)r * ml1;
    const int64_t nvalid = st[ml1];                  // malformed words were left out
    const int wmax = lanes_for_len(J->max_len);
    const int64_t first = J->offsets[0];             // nothing below it is read
    const uint8_t* blo = J->bytes + (first > 0 ? first : 0);
    const uint8_t* bhi = J->bytes + J->n_bytes;
    for (int i = 0; i < kChunkRounds; ++i) {
        const int64_t q = gs + (int64_t)i * kWave + lane;
        if (q >= ge) break;
        const int64_t local = q - a;
        if (local >= nvalid) continue;
        const int32_t idx = J->order[q];
        if (idx < 0 || idx >= b - a) {
            set_status(J, ST_OVERFLOW);
            continue;
        }
        const int64_t g = a + idx;
        const int64_t o0 = J->offsets[g], o1 = J->offsets[g + 1];
        const int64_t len = o1 - o0;
        if (o0 < 0 || len < 0 || len > J->max_len || o1 > J->n_bytes) {
            set_status(J, ST_BAD_OFFSETS);
            continue;
        }
        const int L = (int)len;
        const int64_t j = local - st[L];
        const int nb = cnt[L];
        const int64_t ko = ko_r[L];
        if (j < 0 || j >= nb || ko < (int64_t)wmax * a ||
            ko + (int64_t)lanes_for_len(L) * nb > (int64_t)wmax * b) {
            set_status(J, ST_BAD_REQ);
            continue;
        }
        if (L > 0) pack_word(blo, bhi, J->bytes + o0, L, J->keys + ko + j, nb);
        J->perm[q] = idx;
    }
}

static inline unsigned grid_for2(int64_t items, int per_block, int64_t cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t launch_pack(const Job* J, const Bounds& b, hipStream_t s) {
    k_pack<<<grid_for2(b.chunk_cap, kTileWavesPerBlock, 0x7fffffff), 256, 0, s>>>(J);
    return hipGetLastError();
}

hipError_t launch_sort_prep(const Job* J, const Bounds& b, bool after_bucketize, hipStream_t s) {
    if (!b.fused_pack) {
        hipError_t e = launch_chunk_plan(J, b, false, s);   // k_pack's chunk map
        if (e != hipSuccess) return e;
    }
    k_sort_init<<<1, 256, 0, s>>>(J);
    k_tile_plan<<<grid_for2(b.R, kTileWavesPerBlock, 0x7fffffff), 256, 0, s>>>(
        J, after_bucketize && b.fused_pack ? 0 : 1);
    // keys already written by the scatter when it packs (batched form)
    return b.fused_pack ? hipGetLastError() : launch_pack(J, b, s);
}

hipError_t launch_merges(const Job* J, const Bounds& b, hipStream_t s) {
    if (!b.hbm_merge) return hipSuccess;               // no sub-array can take this path
    for (int D = 2; D <= b.dmax && D <= kLdsMaxD; ++D) {
        if (b.hbm_class[D] < 0) continue;
        hipError_t e = launch_hbm_chunks(J, b, D, s);
        if (e != hipSuccess) return e;
    }
    if ((b.flags & kFlagTilesOnly) || !b.hbm_merge) return hipSuccess;
    return launch_merge_sched(J, b, s);
}

}  // namespace bsort
