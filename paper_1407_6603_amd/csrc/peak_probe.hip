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
constexpr int kChains = 16;             // independent chains per lane

// a DPP row move, lane i reading lane i+1 (the library's odd-phase exchange)
constexpr int kDppWaveShl1 = 0x130;

// Every ALU probe issues 2*kChains instructions per loop trip, in two rounds
// of kChains independent instructions; an instruction of the second round
// reads the result of the first round's instruction of its chain, kChains
// instructions earlier, so no instruction waits on the one just before it.
// The instructions are written in inline asm, each as the only instruction
// of its statement, so the loop issues exactly these (plus the loop's own
// scalar counter); the operands are registers that stay live.
template <int KIND>
__global__ __launch_bounds__(kThreads) void k_valu(int64_t iters, uint32_t* sink) {
    const uint32_t t = threadIdx.x + blockIdx.x * kThreads;
    if constexpr (KIND == BSORT_PROBE_F64_MINMAX) {
        double x[kChains], y[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            x[c] = 1.0 + (double)(t & 1023) + c;        // positive normal doubles
            y[c] = 2.0 + (double)((t * 7u) & 1023);
        }
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                asm volatile("v_min_f64 %0, %0, %1" : "+v"(x[c]) : "v"(y[c]));
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                asm volatile("v_max_f64 %0, %0, %1" : "+v"(y[c]) : "v"(x[c]));
        }
        double s = 0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) s += x[c] - y[c];
        if (s == 1.0) sink[t] = 1u;
    } else if constexpr (KIND == BSORT_PROBE_U32_MINMAX || KIND == BSORT_PROBE_U32_ADD) {
        uint32_t x[kChains], y[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            x[c] = t * 2654435761u + c;
            y[c] = t ^ (c * 977u);
        }
        for (int64_t i = 0; i < iters; ++i) {
            if constexpr (KIND == BSORT_PROBE_U32_MINMAX) {
#pragma unroll
                for (int c = 0; c < kChains; ++c)
                    asm volatile("v_min_u32 %0, %0, %1" : "+v"(x[c]) : "v"(y[c]));
#pragma unroll
                for (int c = 0; c < kChains; ++c)
                    asm volatile("v_max_u32 %0, %0, %1" : "+v"(y[c]) : "v"(x[c]));
            } else {
#pragma unroll
                for (int c = 0; c < kChains; ++c)
                    asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[c]) : "v"(y[c]));
#pragma unroll
                for (int c = 0; c < kChains; ++c)
                    asm volatile("v_add_u32 %0, %0, %1" : "+v"(y[c]) : "v"(x[c]));
            }
        }
        uint32_t s = 0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) s ^= x[c] ^ y[c];
        if (s == 0x9E3779B9u) sink[t] = s;
    } else if constexpr (KIND == BSORT_PROBE_U64_CMP_SELECT) {
        // compare two 64-bit keys and select both 32-bit halves of both records
        // (the compiler's own form of the library's integer compare-exchange)
        uint64_t a[kChains / 2], b[kChains / 2];
#pragma unroll
        for (int c = 0; c < kChains / 2; ++c) {
            a[c] = ((uint64_t)t << 32) | (t * 2654435761u + c);
            b[c] = ((uint64_t)(t ^ c) << 32) | (t * 40503u);
        }
        for (int64_t i = 0; i < iters; ++i) {
            uint64_t lo[kChains / 2], hi[kChains / 2];
#pragma unroll
            for (int c = 0; c < kChains / 2; ++c) {
                const bool g = a[c] > b[c];
                lo[c] = g ? b[c] : a[c];
                hi[c] = g ? a[c] : b[c];
            }
            // the next step pairs one chain's larger record with the next chain's
            // smaller one, so no order between them is known in advance
#pragma unroll
            for (int c = 0; c < kChains / 2; ++c) {
                a[c] = hi[c];
                b[c] = lo[(c + 1) % (kChains / 2)];
            }
        }
        uint64_t s = 0;
#pragma unroll
        for (int c = 0; c < kChains / 2; ++c) s ^= a[c] ^ b[c];
        if (s == 0x9E3779B97F4A7C15ull) sink[t] = 1u;
    } else if constexpr (KIND == BSORT_PROBE_DPP_MOVE) {
        // row moves alone: x <- y of the next lane, then y <- x of the next lane
        int x[kChains], y[kChains];
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            x[c] = (int)(t + c);
            y[c] = (int)(t ^ c);
        }
        for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                x[c] = __builtin_amdgcn_update_dpp(x[c], y[c], kDppWaveShl1, 0xF, 0xF, false);
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                y[c] = __builtin_amdgcn_update_dpp(y[c], x[c], kDppWaveShl1, 0xF, 0xF, false);
        }
        int s = 0;
#pragma unroll
        for (int c = 0; c < kChains; ++c) s ^= x[c] ^ y[c];
        if (s == 0x12345678) sink[t] = 1u;
    }
}

// LDS: each lane moves 16 bytes per access, consecutive lanes consecutive
// 16-byte words (no bank conflicts); 64 KiB per workgroup.  A loop trip makes
// four accesses at immediate offsets 16 KiB apart from one base address,
// which changes once per trip; a read's four dwords are folded into two
// running three-input XORs (two VALU instructions per 1 KiB a wave reads);
// a write stores one register quad.
constexpr int kLdsWords = 64 * 1024 / 16;
constexpr int kXor3 = 0x96;             // v_bitop3_b32 truth table of a ^ b ^ c

template <bool WRITE>
__global__ __launch_bounds__(kThreads) void k_lds(int64_t iters, uint32_t* sink) {
    __shared__ uint4 buf[kLdsWords];
    const int tid = threadIdx.x;
    for (int i = tid; i < kLdsWords; i += kThreads) buf[i] = make_uint4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    uint32_t a0 = 0, a1 = 0;
    const uint4 w = make_uint4(tid, tid + 1, tid * 3, 7);
    for (int64_t it = 0; it < iters; ++it) {
        // tid XOR a value below 64 permutes each group of 64 lanes: still
        // consecutive 16-byte words per group of 16 lanes
        const int b = tid ^ ((int)it & 63);
#pragma unroll
        for (int r = 0; r < kLdsWords / kThreads; ++r) {
            if constexpr (WRITE) {
                buf[b + r * kThreads] = w;
            } else {
                const uint4 v = buf[b + r * kThreads];
                a0 = __builtin_amdgcn_bitop3_b32(a0, v.x, v.y, kXor3);
                a1 = __builtin_amdgcn_bitop3_b32(a1, v.z, v.w, kXor3);
            }
        }
    }
    if constexpr (WRITE) {
        __syncthreads();
        const uint4 v = buf[(tid * 7) & (kLdsWords - 1)];
        a0 = v.x ^ v.y;
        a1 = v.z ^ v.w;
    }
    if ((a0 ^ a1) == 0x5A5A5A5Au) sink[blockIdx.x * kThreads + tid] = 1u;
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
            *units = lanes * iters * (kChains / 2);    // compare-exchanges
            break;
        case BSORT_PROBE_DPP_MOVE:
            k_valu<BSORT_PROBE_DPP_MOVE><<<grid, kThreads, 0, s>>>(iters, sink);
            *units = lanes * iters * kChains * 2;      // row moves
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
