/* zippel_microbench.h — throughput probes that set the roofline of the integer
 * Zippel path on gfx950 (measured, not assumed: no int32-multiply rate is
 * published for MI355X).  Not part of the reconstruction itself.
 *
 * zr_microbench(kind, blocks, iters, bytes, stream, &ms, &ops):
 *   Launches `blocks` workgroups of 256 lanes; each lane runs `iters`
 *   iterations of 8 independent instances of the probed operation (kinds
 *   below).  The first launch warms up; the second is timed with HIP events
 *   on `stream`.  *ms = duration of the timed launch, *ops = number of probed
 *   operations it executed (lanes x iters x 8), or bytes moved for COPY
 *   (reads + writes of a `bytes`-long buffer, 16-byte vector accesses), or
 *   bytes delivered to lanes for the LDS kinds (lanes x iters x 8 x 8).
 *   Returns 0, -1 for an unknown kind, -7 if allocation fails, -8 on a HIP error.
 *   Allocates and frees its own device memory.
 */
#ifndef ZIPPEL_MICROBENCH_H
#define ZIPPEL_MICROBENCH_H
#include <stdint.h>
#include <hip/hip_runtime_api.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  ZR_MB_MAD_U64_U32 = 0, /* v_mad_u64_u32: 32x32 -> 64-bit product plus 64-bit addend */
  ZR_MB_MUL_LO_U32 = 1,  /* v_mul_lo_u32 */
  ZR_MB_MUL_HI_U32 = 2,  /* v_mul_hi_u32 */
  ZR_MB_ADD_U32 = 3,     /* v_add_u32 (full-rate reference) */
  ZR_MB_MAC192 = 4,      /* the library's 64x64 -> 192-bit multiply-accumulate */
  ZR_MB_SHOUP = 5,       /* the library's Shoup product by a fixed multiplier */
  ZR_MB_COPY = 6,        /* streaming device-to-device copy */
  ZR_MB_LDS_READ = 7,    /* 8-byte LDS reads at lane-consecutive addresses */
  ZR_MB_LDS_BCAST = 8    /* 8-byte LDS reads, one address per wave (broadcast) */
};

int zr_microbench(int kind, uint32_t blocks, uint32_t iters, uint64_t bytes, hipStream_t stream, double* ms,
                  double* ops);

#ifdef __cplusplus
}
#endif
#endif
