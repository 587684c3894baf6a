// Length bucketing on the GPU: the paper's count array of words per length
// and its sub-arrays filled in input order (Section II pre-processing phase
// 2; Section III approach two's count array l[]).
//
//   k_chunk_plan    one workgroup: chunks per list, their running sum (the
//                   sort side re-runs it: its chunk map must not depend on
//                   what an earlier call left in the workspace)
//   k_chunk_hist    one wave per chunk of 1024 words: length histogram
//   k_chunk_scan    one wave per (list, length): exclusive scan over chunks
//   k_bucket_starts one wave per list: starts = exclusive scan of counts
//   k_scatter       one wave per chunk: stable placement of word indices
//
// Every word is read twice (offsets only): HBM bound, ~16 B/word read and
// 4 B/word written.  A chunk never straddles two lists.
#include "bsort_internal.h"

namespace bsort {

// length of global word g, or -1 (with a status bit) if it is malformed
__device__ __forceinline__ int word_len(const Job* J, int64_t g, uint32_t& bad) {
    const int64_t o0 = J->offsets[g], o1 = J->offsets[g + 1];
    if (o0 < 0 || o1 < o0 || o1 > J->n_bytes) {
        bad |= ST_BAD_OFFSETS;
        return -1;
    }
    if (o1 - o0 > J->max_len) {
        bad |= ST_TOO_LONG;
        return -1;
    }
    return (int)(o1 - o0);
}

__global__ void k_set_job(Job j, Job* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = j;
}

__global__ __launch_bounds__(1024) void k_chunk_plan(const Job* __restrict__ J, int clear_status) {
    __shared__ int64_t wsum[16];
    __shared__ int64_t carry;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int R = J->R;
    if (tid == 0) {
        if (clear_status && !(J->flags & kJobKeepStatus)) *J->status = 0u;
        carry = 0;
        if (J->req_start[0] != 0 || J->req_start[R] != J->total) set_status(J, ST_BAD_REQ);
    }
    __syncthreads();
    for (int base = 0; base <= R; base += 1024) {
        const int r = base + tid;
        int64_t v = 0;
        if (r < R) {
            if (J->req_start[r + 1] < J->req_start[r]) set_status(J, ST_BAD_REQ);
            int64_t a, b;
            req_bounds(J, r, a, b);
            v = (b - a + kChunk - 1) / kChunk;
        }
        const int64_t incl = wave_incl_scan(v, lane);
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        if (wv == 0) {
            int64_t x = lane < 16 ? wsum[lane] : 0;
            x = wave_incl_scan(x, lane);
            if (lane < 16) wsum[lane] = x;
        }
        __syncthreads();
        const int64_t before = carry + (wv > 0 ? wsum[wv - 1] : 0);
        if (r <= R) J->chunk_begin[r] = before + incl - v;
        __syncthreads();
        if (tid == 0) carry += wsum[15];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_chunk_hist(const Job* __restrict__ J) {
    __shared__ int hist[kTileWavesPerBlock][kMaxLen + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * kTileWavesPerBlock + wv;
    int r;
    int64_t a, b, gs, ge;
    if (!chunk_range(J, c, r, a, b, gs, ge)) return;     // whole wave; no block barriers below
    const int ml1 = J->ml1;
    for (int L = lane; L < ml1; L += kWave) hist[wv][L] = 0;
    __builtin_amdgcn_wave_barrier();
    uint32_t bad = 0;
    for (int i = 0; i < kChunkRounds; ++i) {
        const int64_t g = gs + (int64_t)i * kWave + lane;
        if (g < ge) {
            const int L = word_len(J, g, bad);
            if (L >= 0) atomicAdd(&hist[wv][L], 1);
        }
    }
    if (bad) set_status(J, bad);
    __builtin_amdgcn_wave_barrier();
    for (int L = lane; L < ml1; L += kWave) J->chunk_hist[c * ml1 + L] = hist[wv][L];
}

__global__ __launch_bounds__(256) void k_chunk_scan(const Job* __restrict__ J) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ml1 = J->ml1, R = J->R;
    const int64_t wid = (int64_t)blockIdx.x * kTileWavesPerBlock + wv;
    if (wid >= (int64_t)R * ml1) return;
    const int r = (int)(wid / ml1), L = (int)(wid % ml1);
    int64_t nch = J->chunk_begin[R];
    if (nch > J->chunk_cap) nch = J->chunk_cap;
    const int64_t c0 = J->chunk_begin[r];
    const int64_t c1 = J->chunk_begin[r + 1] < nch ? J->chunk_begin[r + 1] : nch;
    int run = 0;
    for (int64_t base = c0; base < c1; base += kWave) {
        const int64_t c = base + lane;
        const int v = c < c1 ? J->chunk_hist[c * ml1 + L] : 0;
        const int incl = wave_incl_scan(v, lane);
        if (c < c1) J->chunk_hist[c * ml1 + L] = run + incl - v;
        run += __shfl(incl, kWave - 1, kWave);
    }
    if (lane == 0) J->counts[(int64_t)r * ml1 + L] = run;
}

// starts = exclusive scan of counts; key_off = each sub-array's first key
// lane: wmax lanes per word of the list before it, then ceil(L/8) lanes per
// word of the shorter sub-arrays (the same layout the tile plan checks)
__global__ __launch_bounds__(256) void k_bucket_starts(const Job* __restrict__ J) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ml1 = J->ml1;
    const int r = blockIdx.x * kTileWavesPerBlock + wv;
    if (r >= J->R) return;
    int64_t a, b;
    req_bounds(J, r, a, b);
    const int32_t* cnt = J->counts + (int64_t)r * ml1;
    int32_t* st = J->starts + (int64_t)r * (ml1 + 1);
    int64_t* ko = J->key_off + (int64_t)r * ml1;
    int run = 0;
    int64_t krun = (int64_t)lanes_for_len(J->max_len) * a;
    for (int base = 0; base < ml1; base += kWave) {
        const int L = base + lane;
        const int v = L < ml1 ? cnt[L] : 0;
        const int incl = wave_incl_scan(v, lane);
        const int64_t kv = L < ml1 ? (int64_t)lanes_for_len(L) * v : 0;
        const int64_t kincl = wave_incl_scan(kv, lane);
        if (L < ml1) {
            st[L] = run + incl - v;
            ko[L] = krun + kincl - kv;
        }
        run += __shfl(incl, kWave - 1, kWave);
        krun += __shfl(kincl, kWave - 1, kWave);
    }
    if (lane == 0) st[ml1] = run;
}

// Stable placement by length: a word's place in its list's sub-array is the
// sub-array start, the words of that length in earlier chunks, and the
// earlier lanes of this chunk with the same length.  Writes order, or in the
// batched form (kJobFusedPack) the word's key lanes and index payload at that
// place directly.
__global__ __launch_bounds__(256) void k_scatter(const Job* __restrict__ J) {
    __shared__ int run[kTileWavesPerBlock][kMaxLen + 1];
    __shared__ int nbs[kTileWavesPerBlock][kMaxLen + 1];
    __shared__ int64_t kos[kTileWavesPerBlock][kMaxLen + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * kTileWavesPerBlock + wv;
    int r;
    int64_t a, b, gs, ge;
    if (!chunk_range(J, c, r, a, b, gs, ge)) return;
    const int ml1 = J->ml1;
    const bool fused = (J->flags & kJobFusedPack) != 0;
    const int32_t* st = J->starts + (int64_t)r * (ml1 + 1);
    for (int L = lane; L < ml1; L += kWave) {
        run[wv][L] = st[L] + J->chunk_hist[c * ml1 + L];
        if (fused) {
            nbs[wv][L] = J->counts[(int64_t)r * ml1 + L];
            kos[wv][L] = J->key_off[(int64_t)r * ml1 + L];
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int64_t nr = b - a;
    const int wmax = lanes_for_len(J->max_len);
    const int64_t first = J->offsets[0];             // nothing below it is read
    const uint8_t* blo = J->bytes + (first > 0 ? first : 0);
    const uint8_t* bhi = J->bytes + J->n_bytes;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    for (int i = 0; i < kChunkRounds; ++i) {
        const int64_t g = gs + (int64_t)i * kWave + lane;
        uint32_t bad = 0;
        const int L = g < ge ? word_len(J, g, bad) : -1;
        const bool valid = L >= 0;
        // lanes holding the same length: match the 7 bits of the length
        uint64_t m = __ballot(valid);
        const int key = valid ? L : 127;
#pragma unroll
        for (int bit = 0; bit < 7; ++bit) {
            const bool on = (key >> bit) & 1;
            const uint64_t bm = __ballot(on);
            m &= on ? bm : ~bm;
        }
        if (valid) {
            const int rank = __popcll(m & lt);          // earlier lanes, same length
            const int base = run[wv][L];
            const int64_t pos = (int64_t)base + rank;
            if (pos < 0 || pos >= nr) {
                set_status(J, ST_OVERFLOW);
            } else if (!fused) {
                J->order[a + pos] = (int32_t)(g - a);
            } else {
                const int64_t j = pos - st[L];           // place inside the sub-array
                const int nb = nbs[wv][L];
                const int64_t ko = kos[wv][L];
                if (j < 0 || j >= nb || ko < (int64_t)wmax * a ||
                    ko + (int64_t)lanes_for_len(L) * nb > (int64_t)wmax * b) {
                    set_status(J, ST_BAD_REQ);
                } else {
                    if (L > 0) pack_word(blo, bhi, J->bytes + J->offsets[g], L, J->keys + ko + j, nb);
                    J->perm[a + pos] = (int32_t)(g - a);
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (rank == 0) run[wv][L] = base + __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

static inline unsigned grid_for(int64_t items, int per_block) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 0x7fffffff) g = 0x7fffffff;
    return (unsigned)g;
}

hipError_t launch_set_job(const Job& j, Job* dst, hipStream_t s) {
    k_set_job<<<1, 64, 0, s>>>(j, dst);
    return hipGetLastError();
}

hipError_t launch_chunk_plan(const Job* J, bool clear_status, hipStream_t s) {
    k_chunk_plan<<<1, 1024, 0, s>>>(J, clear_status ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_bucketize(const Job* J, const Bounds& b, hipStream_t s) {
    k_chunk_plan<<<1, 1024, 0, s>>>(J, 1);
    k_chunk_hist<<<grid_for(b.chunk_cap, kTileWavesPerBlock), 256, 0, s>>>(J);
    k_chunk_scan<<<grid_for((int64_t)b.R * b.ml1, kTileWavesPerBlock), 256, 0, s>>>(J);
    k_bucket_starts<<<grid_for(b.R, kTileWavesPerBlock), 256, 0, s>>>(J);
    k_scatter<<<grid_for(b.chunk_cap, kTileWavesPerBlock), 256, 0, s>>>(J);
    return hipGetLastError();
}

}  // namespace bsort
