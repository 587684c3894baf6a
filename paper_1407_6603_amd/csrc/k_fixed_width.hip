// Fixed-width keys for the unbucketed ablation (Section II, Table 1 rows
// 2-3: the whole file bubble-sorted by alphabetic order, or by word length,
// with no sub-arrays).  Every word becomes a key of the same width, so the
// sorting calls see one sub-array per list and run the same odd-even
// transposition sort and merge-split over the whole list:
//   bytes only         the word's bytes, zero-padded (alphabetic order:
//                      a prefix sorts first; zero bytes inside words tie
//                      with the padding, which the letter workloads never
//                      have);
//   length only        one byte, the word's length;
//   length then bytes  the length byte, then the padded bytes: the order of
//                      the bucketed sort, reached without buckets.
// One thread per output byte; HBM-bound.
#include "../../include/bsort.h"
#include "bsort_internal.h"

namespace bsort {
namespace {

constexpr int kFwThreads = 256;

__global__ void k_fw_clear(int32_t* status) { *gp(status) = 0; }

// out[i*width + k] for every word i and key byte k; offsets_out[i] = i*width
__global__ __launch_bounds__(kFwThreads) void k_fixed_width(
    const uint8_t* __restrict__ bytes, int64_t n_bytes, const int64_t* __restrict__ offsets,
    int64_t n_words, int32_t width, int32_t mode, uint8_t* __restrict__ out,
    int64_t* __restrict__ offsets_out, int32_t* __restrict__ status) {
    const gptr<const int64_t> off = gp(offsets);
    const gptr<const uint8_t> b = gp(bytes);
    const int64_t total = n_words * (int64_t)width;
    for (int64_t e = (int64_t)blockIdx.x * kFwThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kFwThreads) {
        const int64_t i = e / width;
        const int k = (int)(e - i * width);
        const int64_t a = off[i];
        const int64_t end = off[i + 1];
        const bool valid = a >= 0 && end >= a && end <= n_bytes;   // else nothing is read
        const int64_t len = valid ? end - a : 0;
        const int lead = mode == BSORT_KEY_BYTES ? 0 : 1;     // the length byte
        uint8_t v = 0;
        if (mode == BSORT_KEY_LENGTH) {
            v = (uint8_t)len;
        } else if (k < lead) {
            v = (uint8_t)len;
        } else if (k - lead < len) {
            v = b[a + (k - lead)];
        }
        gp(out)[e] = v;
        if (k == 0) {
            gp(offsets_out)[i] = e;
            const bool fits = mode == BSORT_KEY_LENGTH ? len <= 255 : len + lead <= width &&
                                                                      (lead == 0 || len <= 255);
            if (!fits || !valid)
                __hip_atomic_fetch_or(gp(status), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) gp(offsets_out)[n_words] = total;
}

}  // namespace

hipError_t launch_fixed_width(const uint8_t* bytes, int64_t n_bytes, const int64_t* offsets,
                              int64_t n_words,
                              int32_t width, int32_t mode, uint8_t* out, int64_t* offsets_out,
                              int32_t* status, hipStream_t s) {
    const int64_t total = n_words * (int64_t)width;
    int64_t g = (total + kFwThreads - 1) / kFwThreads;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    k_fw_clear<<<1, 1, 0, s>>>(status);
    k_fixed_width<<<(unsigned)g, kFwThreads, 0, s>>>(bytes, n_bytes, offsets, n_words, width,
                                                      mode, out, offsets_out, status);
    return hipGetLastError();
}

}  // namespace bsort
