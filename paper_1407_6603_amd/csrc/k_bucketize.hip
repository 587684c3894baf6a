// Length bucketing on the GPU: the paper's count array of words per length
// and its sub-arrays filled in input order (Section II pre-processing phase
// 2; Section III approach two's count array l[]).
//
//   k_chunk_plan    one workgroup: chunks per list, their running sum (the
//                   sort side re-runs it: its chunk map must not depend on
//                   what an earlier call left in the workspace)
//   k_chunk_hist    one wave per chunk of kChunk words: length histogram,
//                   and each word's length as one byte
//   k_chunk_scan    one wave per (list, length): exclusive scan over chunks
//   k_bucket_starts one wave per list: starts = exclusive scan of counts
//   k_scatter       one wave per chunk: stable placement of word indices
//
// The offsets are read once (8 B/word, by the histogram pass); the scatter
// reads the length bytes and rebuilds each word's offset as the chunk's
// first offset plus the lengths before it (a word's bytes end where the
// next word's begin).  HBM bound.  A chunk never straddles two lists.
#include "bsort_internal.h"

namespace bsort {

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

// chunk -> list table: one wave per list writes its chunks' entries
__global__ __launch_bounds__(256) void k_chunk_lists(const Job* __restrict__ J) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = blockIdx.x * kTileWavesPerBlock + wv;
    if (r >= J->R) return;
    const gptr<const int64_t> cb = gp(J->chunk_begin);
    const int64_t c0 = cb[r];
    int64_t c1 = cb[r + 1];
    if (c1 > J->chunk_cap) c1 = J->chunk_cap;
    const gptr<int32_t> cl = gp(J->chunk_list);
    for (int64_t c = c0 + lane; c < c1; c += kWave) cl[c] = r;
}


// word length from its two offsets, or -1 (reason in bad) if malformed
// (outside [first, n_bytes], the readable bytes) or longer than max_len
__device__ __forceinline__ int word_len_o(int64_t o0, int64_t o1, int64_t first, int64_t n_bytes,
                                          int max_len, uint32_t& bad) {
    if (o0 < 0 || o0 < first || o1 < o0 || o1 > n_bytes) {
        bad |= ST_BAD_OFFSETS;
        return -1;
    }
    if (o1 - o0 > max_len) {
        bad |= ST_TOO_LONG;
        return -1;
    }
    return (int)(o1 - o0);
}

// 64-bit value of the next lane (lane 63 keeps `old`)
__device__ __forceinline__ int64_t from_next_lane64(int64_t old, int64_t v) {
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)old, (int)(uint32_t)v, 0x130, 0xF,
                                               0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)((uint64_t)old >> 32),
                                               (int)(uint32_t)((uint64_t)v >> 32), 0x130, 0xF,
                                               0xF, false);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int64_t lane0_of(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

constexpr int kHistBatch = 16;                      // rounds whose loads are in flight together

__global__ __launch_bounds__(256) void k_chunk_hist(const Job* __restrict__ J) {
    __shared__ int hist[kTileWavesPerBlock][kMaxLen + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * kTileWavesPerBlock + wv;
    int r;
    int64_t a, b, gs, ge;
    if (!chunk_range(J, c, r, a, b, gs, ge)) return;     // whole wave; no block barriers below
    const int ml1 = J->ml1, max_len = J->max_len;
    const int64_t n_bytes = J->n_bytes;
    const gptr<const int64_t> offs = gp(J->offsets);
    const gptr<uint8_t> len8 = gp(J->len8);
    const int64_t first = offs[0];
    for (int L = lane; L < ml1; L += kWave) hist[wv][L] = 0;
    __builtin_amdgcn_wave_barrier();
    uint32_t bad = 0;
    const int rounds = (int)((ge - gs + kWave - 1) / kWave);       // uniform
    for (int i0 = 0; i0 < rounds; i0 += kHistBatch) {
        // each word's first offset, once: the next word's comes from the next
        // lane, or for lane 63 from lane 0 of the next round; offsets[ge]
        // exists (offsets has total + 1 entries), so every load is in range
        int64_t o[kHistBatch];
#pragma unroll
        for (int k = 0; k < kHistBatch; ++k) {
            const int64_t g = gs + (int64_t)(i0 + k) * kWave + lane;
            o[k] = offs[g < ge ? g : ge];
        }
        const int64_t gt = gs + (int64_t)(i0 + kHistBatch) * kWave;
        const int64_t tail = offs[gt < ge ? gt : ge];
        int Ls[kHistBatch];
#pragma unroll
        for (int k = 0; k < kHistBatch; ++k) {
            const int64_t g = gs + (int64_t)(i0 + k) * kWave + lane;
            const int64_t after = k + 1 < kHistBatch ? lane0_of(o[k + 1]) : tail;
            const int64_t o1 = from_next_lane64(after, o[k]);
            Ls[k] = g < ge ? word_len_o(o[k], o1, first, n_bytes, max_len, bad) : -1;
            if (g < ge) len8[g] = (uint8_t)(Ls[k] >= 0 ? Ls[k] : 0xFF);
        }
#pragma unroll
        for (int k = 0; k < kHistBatch; ++k)
            if (Ls[k] >= 0) atomicAdd(&hist[wv][Ls[k]], 1);
    }
    if (bad) set_status(J, bad);
    __builtin_amdgcn_wave_barrier();
    const gptr<int32_t> ch = gp(J->chunk_hist);
    for (int L = lane; L < ml1; L += kWave) ch[c * ml1 + L] = hist[wv][L];
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

// Key lanes of a word of L <= 12 bytes at p: the word lies in the 16 bytes
// from the dword boundary at or below p, loaded as four dwords (a fixed
// count, so many words' loads can be in flight together); false if those
// bytes are not all inside [lo, hi).
// (the load itself is unconditional: the address is clamped into [lo, hi-16],
// which the caller guarantees is not empty, and the result only counts when
// the clamp did not move it)
__device__ __forceinline__ bool load_short_word(uintptr_t lo, uintptr_t hi, uintptr_t addr,
                                                uint32_t (&q)[4], int& sh) {
    const uintptr_t a4 = addr & ~(uintptr_t)3;
    sh = (int)(addr & 3);
    const uintptr_t top = (hi - 16) & ~(uintptr_t)3;
    const uintptr_t lo4 = (lo + 3) & ~(uintptr_t)3;
    const uintptr_t ac = a4 < lo4 ? lo4 : (a4 > top ? top : a4);
    const gptr<const uint32_t> w = (gptr<const uint32_t>)ac;
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = w[i];
    return ac == a4;
}

// big-endian key lanes (W <= 2) of the L <= 12 bytes held in q from byte sh
__device__ __forceinline__ void short_word_lanes(const uint32_t (&q)[4], int sh, int L,
                                                 uint64_t& l0, uint64_t& l1) {
    uint32_t be[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        uint32_t v = __builtin_bswap32(__builtin_amdgcn_alignbyte(q[i + 1], q[i], sh));
        const int valid = L - 4 * i;
        v = valid >= 4 ? v : (valid <= 0 ? 0u : v & (0xFFFFFFFFu << (8 * (4 - valid))));
        be[i] = v;
    }
    l0 = ((uint64_t)be[0] << 32) | be[1];
    l1 = (uint64_t)be[2] << 32;
}

// Stable placement by length: a word's place in its list's sub-array is the
// sub-array start, the words of that length in earlier chunks, and the
// earlier lanes of this chunk with the same length.  Writes order, or in the
// batched form (kJobFusedPack) the word's key lanes and index payload at that
// place directly.  Rounds are handled kScatterBatch at a time: all their
// offsets and word bytes are loaded before any of their results is stored.
constexpr int kScatterBatch = 8;

__global__ __launch_bounds__(256) void k_scatter(const Job* __restrict__ J) {
    __shared__ int run[kTileWavesPerBlock][kMaxLen + 1];
    __shared__ int sts[kTileWavesPerBlock][kMaxLen + 1];
    __shared__ int nbs[kTileWavesPerBlock][kMaxLen + 1];
    __shared__ int64_t kos[kTileWavesPerBlock][kMaxLen + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * kTileWavesPerBlock + wv;
    int r;
    int64_t a, b, gs, ge;
    if (!chunk_range(J, c, r, a, b, gs, ge)) return;
    const int ml1 = J->ml1, max_len = J->max_len;
    const bool fused = (J->flags & kJobFusedPack) != 0;
    // the four-dword word loads need at least 16 readable bytes
    const bool short_words = max_len <= 12;
    const int64_t n_bytes = J->n_bytes;
    const int64_t nr = b - a;
    const int wmax = lanes_for_len(max_len);
    {
        const gptr<const int32_t> st = gp(J->starts) + (int64_t)r * (ml1 + 1);
        const gptr<const int32_t> cnt = gp(J->counts) + (int64_t)r * ml1;
        const gptr<const int64_t> ko_r = gp(J->key_off) + (int64_t)r * ml1;
        const gptr<const int32_t> ch = gp(J->chunk_hist) + c * ml1;
        for (int L = lane; L < ml1; L += kWave) {
            const int s0 = st[L];
            run[wv][L] = s0 + ch[L];
            sts[wv][L] = s0;
            nbs[wv][L] = fused ? cnt[L] : 0;
            // a sub-array whose key lanes would leave the list's range is
            // never written (marked by a negative offset)
            const int64_t ko = fused ? ko_r[L] : 0;
            const bool kok = !fused || (ko >= (int64_t)wmax * a &&
                                        ko + (int64_t)lanes_for_len(L) * cnt[L] <= (int64_t)wmax * b);
            kos[wv][L] = kok ? ko : -1;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const gptr<const int64_t> offs = gp(J->offsets);
    const gptr<const uint8_t> bytes = gp(J->bytes);
    const gptr<uint64_t> keys = gp(J->keys);
    const gptr<int32_t> perm = gp(J->perm);
    const gptr<int32_t> order = gp(J->order);
    const int64_t first = offs[0];                   // nothing below it is read
    const gptr<const uint8_t> blo = bytes + (first > 0 ? first : 0);
    const gptr<const uint8_t> bhi = bytes + n_bytes;
    const bool short_ok = short_words && (uintptr_t)bhi >= (uintptr_t)blo + 32;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    // bits that tell lengths 0..max_len and "no word" (all ones) apart
    const int nbits = 32 - __builtin_clz((unsigned)ml1);
    const int none = (1 << nbits) - 1;
    uint32_t err = 0;
    const gptr<const uint8_t> len8 = gp(J->len8);
    // the first offset of the batch's next word: the chunk's first offset,
    // then the running sum of the lengths (a malformed word counts as empty:
    // the call has failed, and the range checks below keep every read in
    // bounds)
    int64_t run_off = offs[gs];
    const int rounds = (int)((ge - gs + kWave - 1) / kWave);       // uniform
    for (int i0 = 0; i0 < rounds; i0 += kScatterBatch) {
        // 1. lengths (and for short words the bytes) of the batch's words
        int Ls[kScatterBatch];
        int64_t o0[kScatterBatch];
        uint32_t q[kScatterBatch][4];
        int shs[kScatterBatch];
        bool qok[kScatterBatch];
        uint32_t lb[kScatterBatch];
#pragma unroll
        for (int k = 0; k < kScatterBatch; ++k) {
            const int64_t g = gs + (int64_t)(i0 + k) * kWave + lane;
            lb[k] = g < ge ? (uint32_t)len8[g] : 0xFFu;
        }
#pragma unroll
        for (int k = 0; k < kScatterBatch; ++k) {
            const int L = lb[k] == 0xFFu ? -1 : (int)lb[k];
            const int v = L > 0 ? L : 0;
            const int incl = wave_incl_scan(v, lane);
            o0[k] = run_off + (incl - v);
            run_off += __builtin_amdgcn_readlane(incl, kWave - 1);
            // the rebuilt range must lie in the readable bytes
            Ls[k] = (L >= 0 && o0[k] >= first && o0[k] + L <= n_bytes) ? L : -1;
            qok[k] = false;
            shs[k] = 0;
        }
        // key lanes of the whole batch before any of its stores: the
        // vector-memory counter also counts stores, so a load consumed after
        // a store has been issued would wait for that store as well
        uint64_t l0s[kScatterBatch], l1s[kScatterBatch];
        if (fused && short_ok) {
#pragma unroll
            for (int k = 0; k < kScatterBatch; ++k) {
                const int64_t oc = o0[k] >= 0 && o0[k] <= n_bytes ? o0[k] : 0;
                const bool in = load_short_word((uintptr_t)blo, (uintptr_t)bhi,
                                                (uintptr_t)(bytes + oc), q[k], shs[k]);
                qok[k] = Ls[k] > 0 && in;
            }
#pragma unroll
            for (int k = 0; k < kScatterBatch; ++k)
                short_word_lanes(q[k], shs[k], Ls[k], l0s[k], l1s[k]);
        }
        // 2. places, in round order (each round's counters feed the next)
#pragma unroll
        for (int k = 0; k < kScatterBatch; ++k) {
            const int64_t g = gs + (int64_t)(i0 + k) * kWave + lane;
            const int L = Ls[k];
            const bool valid = L >= 0;
            const int key = valid ? L : none;
            uint64_t m = ~0ull;                        // lanes holding the same length
            for (int bit = 0; bit < nbits; ++bit) {
                const bool on = (key >> bit) & 1;
                const uint64_t bm = __ballot(on);
                m &= on ? bm : ~bm;
            }
            const int Lc = valid ? L : 0;
            const int rank = __popcll(m & lt);         // earlier lanes, same length
            const int base = run[wv][Lc];
            const int pos = base + rank;
            const int j = pos - sts[wv][Lc];           // place inside the sub-array
            const int nb = nbs[wv][Lc];
            const int64_t ko = kos[wv][Lc];
            const bool in_list = pos >= 0 && pos < nr;
            const bool ok = valid && in_list && (!fused || (j >= 0 && j < nb && ko >= 0));
            err |= (valid && !in_list) ? ST_OVERFLOW : ((valid && !ok) ? ST_BAD_REQ : 0u);
            if (ok) {
                if (!fused) {
                    order[a + pos] = (int32_t)(g - a);
                } else {
                    const gptr<uint64_t> out = keys + ko + j;
                    if (qok[k]) {
                        out[0] = l0s[k];
                        if (L > 8) out[nb] = l1s[k];
                    } else if (L > 0) {
                        pack_word(blo, bhi, bytes + o0[k], L, out, nb);
                    }
                    perm[a + pos] = (int32_t)(g - a);
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (valid && rank == 0) run[wv][L] = base + __popcll(m);
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (err) set_status(J, err);
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

hipError_t launch_chunk_plan(const Job* J, const Bounds& b, bool clear_status, hipStream_t s) {
    k_chunk_plan<<<1, 1024, 0, s>>>(J, clear_status ? 1 : 0);
    if (b.R > 1) k_chunk_lists<<<grid_for(b.R, kTileWavesPerBlock), 256, 0, s>>>(J);
    return hipGetLastError();
}

hipError_t launch_bucket_starts(const Job* J, const Bounds& b, hipStream_t s) {
    hipError_t e = launch_chunk_plan(J, b, true, s);
    if (e != hipSuccess) return e;
    k_chunk_hist<<<grid_for(b.chunk_cap, kTileWavesPerBlock), 256, 0, s>>>(J);
    k_chunk_scan<<<grid_for((int64_t)b.R * b.ml1, kTileWavesPerBlock), 256, 0, s>>>(J);
    k_bucket_starts<<<grid_for(b.R, kTileWavesPerBlock), 256, 0, s>>>(J);
    return hipGetLastError();
}

hipError_t launch_scatter(const Job* J, const Bounds& b, hipStream_t s) {
    k_scatter<<<grid_for(b.chunk_cap, kTileWavesPerBlock), 256, 0, s>>>(J);
    return hipGetLastError();
}

hipError_t launch_bucketize(const Job* J, const Bounds& b, hipStream_t s) {
    hipError_t e = launch_bucket_starts(J, b, s);
    return e != hipSuccess ? e : launch_scatter(J, b, s);
}

}  // namespace bsort
