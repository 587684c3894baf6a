/*
 * bsort_probe -- throughput probes for the rooflines that bound libbsort's
 * kernels on the GPU they run on (libbsort_probe.so, built beside
 * libbsort.so).  Not part of the sort: they measure the ceilings the sort's
 * kernels are priced against.
 *
 * The compare-exchange of odd-even transposition sort (the data-parallel
 * form of the paper's bubble sort, Section I and "Bubble sort as parallel":
 * n(n-1)/2 compare-exchanges) is issued by libbsort in three vector forms:
 * exact fp64 min/max on records packed as doubles, 32-bit unsigned min/max
 * on one-dword records, and a 64-bit compare plus four dword selects.  The
 * probes time each form, the row move that carries records across lanes, LDS
 * reads and writes, and HBM reads and copies, on every CU of the device.
 */
#ifndef BSORT_PROBE_H
#define BSORT_PROBE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSORT_PROBE_F64_MINMAX 0      /* v_min_f64, v_max_f64; unit: lane instructions */
#define BSORT_PROBE_U32_MINMAX 1      /* v_min_u32, v_max_u32; unit: lane instructions */
#define BSORT_PROBE_U64_CMP_SELECT 2  /* 64-bit compare and four dword selects (as the compiler
                                         forms them); unit: compare-exchanges per lane */
#define BSORT_PROBE_DPP_MOVE 3        /* v_mov_b32 DPP row moves; unit: lane instructions */
#define BSORT_PROBE_U32_ADD 4         /* v_add_u32; unit: lane instructions */
#define BSORT_PROBE_LDS_READ 5        /* 16-byte LDS reads, no bank conflicts; unit: bytes */
#define BSORT_PROBE_LDS_WRITE 6       /* 16-byte LDS writes, no bank conflicts; unit: bytes */
#define BSORT_PROBE_HBM_READ 7        /* 16-byte global loads streaming HBM; unit: bytes */
#define BSORT_PROBE_HBM_COPY 8        /* read + write streams; unit: bytes read plus written */

/*
 * The ALU probes issue, per loop trip and lane, 32 instructions of their
 * kind in two rounds of 16 independent chains (an instruction depends on its
 * chain's instruction 16 earlier), so the rate is the issue ceiling, not a
 * latency; the LDS probes make four 16-byte accesses per trip at immediate
 * offsets with two VALU instructions per read.
 *
 * Runs probe `probe` on the current device, on `stream` (a hipStream_t as
 * void*), and waits for it.  iters: loop trips per lane (ALU and LDS probes)
 * or passes over the buffer (HBM probes).
 * scratch: caller-owned device memory of scratch_bytes >= 64 MiB (the HBM
 * probes stream its part past the first 32 MiB, as two halves).  Writes the
 * probe's device time in milliseconds (HIP events around the launches) to
 * *ms and the work it did, in the probe's unit, to *units; rate = units /
 * (ms / 1000).  Returns 0, 1 for a bad argument, 2 for a HIP error.
 */
int bsort_probe_run(int probe, int64_t iters, void *scratch, size_t scratch_bytes, double *ms,
                    double *units, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BSORT_PROBE_H */
