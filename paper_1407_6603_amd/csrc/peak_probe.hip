// Throughput probes for the rooflines that bound libbsort's kernels on this
// GPU: the vector ALU forms of a compare-exchange (exact fp64 min/max, 32-bit
// unsigned min/max, 64-bit compare plus selects), the cross-lane row move,
// LDS reads and writes, and HBM reads and copies.  Each probe runs on every
// CU with independent instruction chains (or conflict-free streams), so its
// rate is an issue or bandwidth ceiling, not a latency.  See
// include/bsort_probe.h.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bsort_probe.h"

namespace {

constexpr int kThreads = 1024;          // 16 waves per workgroup
constexpr int kChains = 8;              // independent chains per lane

// a DPP row move, lane i reading lane i+1 (the library's odd-phase exchange)
constexpr int kDppWaveShl1 = 0x130;

template <int KIND>
__global__ __launch_bounds__(kThreads) void k_valu(int64_t iters, uint32_t* sink) {
    const uint32_t t = threadIdx.x + blockIdx.x * kThreads;
    if constexpr (KIND == BSORT_PROBE_F64_MINMAX) {
        double a[kChains], b[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            a[c] = (double)(t + c);
            b[c] = (double)(t ^ (c * 977));
        }
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                double lo, hi;
                asm volatile("v_min_f64 %0, %2, %3\n\tv_max_f64 %1, %2, %3"
                             : "=&v"(lo), "=&v"(hi) : "v"(a[c]), "v"(b[c]));
                a[c] = hi;
                b[c] = lo;
            }
        }
        double s = 0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) s += a[c] - b[c];
        if (s == -1.0) sink[t] = 1u;
    } else if constexpr (KIND == BSORT_PROBE_U32_MINMAX || KIND == BSORT_PROBE_U32_ADD) {
        uint32_t a[kChains], b[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            a[c] = t * 2654435761u + c;
            b[c] = t ^ (c * 977u);
        }
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                uint32_t lo, hi;
                if constexpr (KIND == BSORT_PROBE_U32_MINMAX)
                    asm volatile("v_min_u32 %0, %2, %3\n\tv_max_u32 %1, %2, %3"
                                 : "=&v"(lo), "=&v"(hi) : "v"(a[c]), "v"(b[c]));
                else
                    asm volatile("v_add_u32 %0, %2, %3\n\tv_add_u32 %1, %2, %0"
                                 : "=&v"(lo), "=&v"(hi) : "v"(a[c]), "v"(b[c]));
                a[c] = hi;
                b[c] = lo;
            }
        }
        uint32_t s = 0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) s ^= a[c] ^ b[c];
        if (s == 0x9E3779B9u) sink[t] = s;
    } else if constexpr (KIND == BSORT_PROBE_U64_CMP_SELECT) {
        // compare two 64-bit keys and select both 32-bit halves of both records
        uint64_t a[kChains], b[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            a[c] = ((uint64_t)t << 32) | (t * 2654435761u + c);
            b[c] = ((uint64_t)(t ^ c) << 32) | (t * 40503u);
        }
        for (int64_t i = 0; i < iters; ++i) {
            uint64_t lo[kChains], hi[kChains];
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                // the library's integer compare-exchange: one 64-bit compare, four selects
                const bool g = a[c] > b[c];
                lo[c] = g ? b[c] : a[c];
                hi[c] = g ? a[c] : b[c];
            }
            // the next step pairs one chain's larger record with the next chain's
            // smaller one, so no order between them is known in advance
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                a[c] = hi[c];
                b[c] = lo[(c + 1) % kChains];
            }
        }
        uint64_t s = 0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) s ^= a[c] ^ b[c];
        if (s == 0x9E3779B97F4A7C15ull) sink[t] = 1u;
    } else if constexpr (KIND == BSORT_PROBE_DPP_MOVE) {
        int a[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) a[c] = (int)(t + c);
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                a[c] = __builtin_amdgcn_update_dpp(a[c], a[c] + c, kDppWaveShl1, 0xF, 0xF,
                                                   false);
        }
        int s = 0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) s ^= a[c];
        if (s == 0x12345678) sink[t] = 1u;
    }
}

// LDS: each lane moves 16 bytes per access, consecutive lanes consecutive
// 16-byte words (no bank conflicts); 64 KiB per workgroup.
constexpr int kLdsWords = 64 * 1024 / 16;

template <bool WRITE>
__global__ __launch_bounds__(kThreads) void k_lds(int64_t iters, uint32_t* sink) {
    __shared__ uint4 buf[kLdsWords];
    const int tid = threadIdx.x;
    for (int i = tid; i < kLdsWords; i += kThreads) buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < kLdsWords / kThreads; ++r) {
            const int i = (tid + r * kThreads + (int)it * 64) & (kLdsWords - 1);
            if constexpr (WRITE) {
                buf[i] = make_uint4((uint32_t)it, r, tid, 7);
            } else {
                const uint4 v = buf[i];
                acc.x ^= v.x;
                acc.y += v.y;
                acc.z ^= v.z;
                acc.w += v.w;
            }
        }
        if constexpr (WRITE) __syncthreads();
    }
    if constexpr (WRITE) acc = buf[(tid * 7) & (kLdsWords - 1)];
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x5A5A5A5Au) sink[blockIdx.x * kThreads + tid] = 1u;
}

// HBM: every lane streams 16-byte words, grid-stride (read, or read + write)
template <bool COPY>
__global__ __launch_bounds__(256) void k_hbm(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                             int64_t n16, uint32_t* sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint4 acc = make_uint4(0, 0, 0, 0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const uint4 v = src[i];
        if constexpr (COPY) {
            dst[i] = v;
        } else {
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
    }
    if (!COPY && (acc.x & acc.y & acc.z & acc.w) == 0xFFFFFFFFu) sink[0] = 1u;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t init() {
        hipError_t e = hipEventCreate(&a);
        return e == hipSuccess ? hipEventCreate(&b) : e;
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" {

int bsort_probe_run(int probe, int64_t iters, void* scratch, size_t scratch_bytes, double* ms,
                    double* units, void* stream) {
    if (!ms || !units || iters < 1 || !scratch || scratch_bytes < (64u << 20)) return 1;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 2;
    uint32_t* sink = (uint32_t*)scratch;                 // first 32 MiB: sinks
    Timer tm;
    if (tm.init() != hipSuccess) return 2;
    const unsigned grid = (unsigned)cus * 2;             // two 1024-thread workgroups per CU
    const double lanes = (double)grid * kThreads;
    if (hipEventRecord(tm.a, s) != hipSuccess) return 2;
    switch (probe) {
        case BSORT_PROBE_F64_MINMAX:
            k_valu<BSORT_PROBE_F64_MINMAX><<<grid, kThreads, 0, s>>>(iters, sink);
            *units = lanes * iters * kChains * 2;
            break;
        case BSORT_PROBE_U32_MINMAX:
            k_valu<BSORT_PROBE_U32_MINMAX><<<grid, kThreads, 0, s>>>(iters, sink);
            *units = lanes * iters * kChains * 2;
            break;
        case BSORT_PROBE_U32_ADD:
            k_valu<BSORT_PROBE_U32_ADD><<<grid, kThreads, 0, s>>>(iters, sink);
            *units = lanes * iters * kChains * 2;
            break;
        case BSORT_PROBE_U64_CMP_SELECT:
            k_valu<BSORT_PROBE_U64_CMP_SELECT><<<grid, kThreads, 0, s>>>(iters, sink);
            *units = lanes * iters * kChains;          // compare-exchanges
            break;
        case BSORT_PROBE_DPP_MOVE:
            k_valu<BSORT_PROBE_DPP_MOVE><<<grid, kThreads, 0, s>>>(iters, sink);
            *units = lanes * iters * kChains * 2;      // the add and the row move
            break;
        case BSORT_PROBE_LDS_READ:
            k_lds<false><<<grid, kThreads, 0, s>>>(iters, sink);
            *units = (double)grid * iters * kLdsWords * 16.0;
            break;
        case BSORT_PROBE_LDS_WRITE:
            k_lds<true><<<grid, kThreads, 0, s>>>(iters, sink);
            *units = (double)grid * iters * kLdsWords * 16.0;
            break;
        case BSORT_PROBE_HBM_READ:
        case BSORT_PROBE_HBM_COPY: {
            // the scratch past its first 32 MiB, halves as source and destination
            char* base = (char*)scratch + (32u << 20);
            const size_t half = ((scratch_bytes - (32u << 20)) / 2) & ~(size_t)255;
            const int64_t n16 = (int64_t)(half / 16);
            const unsigned g = (unsigned)cus * 8;
            for (int64_t r = 0; r < iters; ++r) {
                if (probe == BSORT_PROBE_HBM_READ)
                    k_hbm<false><<<g, 256, 0, s>>>((const uint4*)base, nullptr, n16, sink);
                else
                    k_hbm<true><<<g, 256, 0, s>>>((const uint4*)base, (uint4*)(base + half),
                                                  n16, sink);
            }
            *units = (double)iters * half * (probe == BSORT_PROBE_HBM_COPY ? 2.0 : 1.0);
            break;
        }
        default:
            return 1;
    }
    if (hipGetLastError() != hipSuccess) return 2;
    if (hipEventRecord(tm.b, s) != hipSuccess) return 2;
    if (hipEventSynchronize(tm.b) != hipSuccess) return 2;
    float f = 0.f;
    if (hipEventElapsedTime(&f, tm.a, tm.b) != hipSuccess) return 2;
    *ms = f;
    return 0;
}

}  // extern "C"
