// Data-structure ablation (Section III: approach one keeps the words as
// vectors of strings, approach two as one fixed-width character array per
// length; Tables 2 and 3 time the same sort on both).  The GPU counterpart
// sorts each sub-array of one list the same way with its words held two
// ways, one workgroup per sub-array running odd-even transposition sort over
// the whole sub-array (n phases, no tiles, no merge-split):
//   packed  each word's key as big-endian dwords in LDS beside its position
//           (the fixed-width array: a compare reads LDS dwords);
//   text    positions only in LDS; a compare reads both words' bytes from
//           the text through order and offsets (the vector of strings: two
//           dependent global reads, then the bytes).
// Both swap only a strictly greater left word, so equal words keep input
// order and both give the library's result.
#include "../../include/bsort.h"
#include "bsort_internal.h"

namespace bsort {
namespace {

constexpr int kLayThreads = 1024;
constexpr int kLayLds = 144 * 1024;               // bytes of LDS per sub-array

struct LayArgs {
    const uint8_t* bytes;
    int64_t n_bytes;
    int32_t n_words;
    const int64_t* offsets;
    const int32_t* counts;
    const int32_t* starts;
    const int32_t* order;
    int32_t* perm;
    int32_t* status;
    int32_t max_len;
};

__global__ void k_lay_clear(int32_t* status) { *gp(status) = 0; }

// big-endian dword q of a word of L bytes at p (zero past its end)
__device__ __forceinline__ uint32_t key_dword(gptr<const uint8_t> p, int L, int q) {
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int j = 4 * q + k;
        v = (v << 8) | (j < L ? (uint32_t)p[j] : 0u);
    }
    return v;
}

// the L bytes of the word at position k of the sub-array, or null (and a
// status bit) if order or offsets point outside the words or the text
__device__ __forceinline__ gptr<const uint8_t> word_at(const LayArgs& A, int start, int L, int k) {
    const int32_t w = gp(A.order)[start + k];
    if (w >= 0 && w < A.n_words) {
        const int64_t o = gp(A.offsets)[w];
        if (o >= 0 && o + L <= A.n_bytes) return gp(A.bytes) + o;
    }
    __hip_atomic_fetch_or(gp(A.status), 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return nullptr;
}

// word at position a of the sub-array is greater than the one at b, reading
// both from the text
__device__ __forceinline__ bool text_gt(const LayArgs& A, int start, int L, int a, int b) {
    const gptr<const uint8_t> pa = word_at(A, start, L, a);
    const gptr<const uint8_t> pb = word_at(A, start, L, b);
    if (!pa || !pb) return false;
    for (int j = 0; j < L; ++j) {
        const uint32_t x = pa[j], y = pb[j];
        if (x != y) return x > y;
    }
    return false;
}

template <bool TEXT>
__global__ __launch_bounds__(kLayThreads) void k_layout_oets(LayArgs A) {
    extern __shared__ uint32_t lds[];
    const int L = blockIdx.x;                      // one workgroup per length
    if (L > A.max_len) return;
    const int n = gp(A.counts)[L];
    const int start = gp(A.starts)[L];
    const int Dk = (L + 3) / 4;                     // key dwords
    const int per = TEXT ? 1 : Dk + 1;              // LDS dwords per word
    if (n < 0 || start < 0 || (int64_t)start + n > A.n_words) {   // buckets not from these words
        if (threadIdx.x == 0)
            __hip_atomic_fetch_or(gp(A.status), 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    if (n < 2) {
        for (int k = threadIdx.x; k < n; k += kLayThreads)
            gp(A.perm)[start + k] = gp(A.order)[start + k];
        return;
    }
    if ((int64_t)n * per * 4 > kLayLds) {           // does not fit: report, sort nothing
        if (threadIdx.x == 0)
            __hip_atomic_fetch_or(gp(A.status), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    // plane d of word k at lds[d * n + k]; the last plane is the position
    for (int k = threadIdx.x; k < n; k += kLayThreads) {
        if (!TEXT) {
            const gptr<const uint8_t> p = word_at(A, start, L, k);
            for (int q = 0; q < Dk; ++q) lds[q * n + k] = p ? key_dword(p, L, q) : 0u;
        }
        lds[(per - 1) * n + k] = (uint32_t)k;
    }
    __syncthreads();
    for (int ph = 0; ph < n; ++ph) {
        for (int i = 2 * threadIdx.x + (ph & 1); i + 1 < n; i += 2 * kLayThreads) {
            bool gt;
            if (TEXT) {
                gt = text_gt(A, start, L, (int)lds[i], (int)lds[i + 1]);
            } else {
                gt = false;
                for (int q = 0; q < Dk; ++q) {
                    const uint32_t x = lds[q * n + i], y = lds[q * n + i + 1];
                    if (x != y) {
                        gt = x > y;
                        break;
                    }
                }
            }
            if (gt)
                for (int d = 0; d < per; ++d) {
                    const uint32_t t = lds[d * n + i];
                    lds[d * n + i] = lds[d * n + i + 1];
                    lds[d * n + i + 1] = t;
                }
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < n; k += kLayThreads)
        gp(A.perm)[start + k] = gp(A.order)[start + (int)lds[(per - 1) * n + k]];
}

}  // namespace

hipError_t launch_layout_oets(const uint8_t* bytes, int64_t n_bytes, const int64_t* offsets,
                              int32_t n_words, int32_t max_len, const int32_t* counts,
                              const int32_t* starts, const int32_t* order, int32_t* perm,
                              int32_t layout, int32_t* status, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void*)k_layout_oets<false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kLayLds);
        (void)hipFuncSetAttribute((const void*)k_layout_oets<true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kLayLds);
        attr = true;
    }
    LayArgs A{bytes, n_bytes, n_words, offsets, counts, starts, order, perm, status, max_len};
    k_lay_clear<<<1, 1, 0, s>>>(status);
    if (layout == BSORT_LAYOUT_TEXT)
        k_layout_oets<true><<<max_len + 1, kLayThreads, kLayLds, s>>>(A);
    else
        k_layout_oets<false><<<max_len + 1, kLayThreads, kLayLds, s>>>(A);
    return hipGetLastError();
}

}  // namespace bsort
