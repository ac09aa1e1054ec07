// Throughput microbenchmarks for the roofline of the integer path on gfx950:
// independent streams of one VALU instruction per lane, at full occupancy, plus
// the library's 64x64 multiply-accumulate and Shoup product, LDS reads, and a
// streaming copy for the HBM bandwidth and the traffic-counter calibration.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/zippel_microbench.h"
#include "field.hpp"

namespace {

constexpr int kChains = 8;

__global__ void __launch_bounds__(256) k_mad_u64_u32(uint32_t iters, uint32_t seed, uint64_t* sink) {
  uint64_t acc[kChains];
  uint32_t a[kChains];
  const uint32_t b = seed | 1u;
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    acc[i] = threadIdx.x + i;
    a[i] = seed * (i + 3) + threadIdx.x;
  }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      uint64_t carry;
      asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(acc[i]), "=s"(carry) : "v"(a[i]), "v"(b));
    }
  }
  uint64_t x = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) x ^= acc[i];
  if (x == 0x123456789ull) sink[0] = x;
}

__global__ void __launch_bounds__(256) k_mul_lo_u32(uint32_t iters, uint32_t seed, uint64_t* sink) {
  uint32_t x[kChains];
  const uint32_t c = seed | 1u;
#pragma unroll
  for (int i = 0; i < kChains; ++i) x[i] = threadIdx.x * 7 + i + 1;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) r ^= x[i];
  if (r == 0x1234567u) sink[0] = r;
}

__global__ void __launch_bounds__(256) k_mul_hi_u32(uint32_t iters, uint32_t seed, uint64_t* sink) {
  uint32_t x[kChains];
  const uint32_t c = 0xFFFFFFFFu ^ (seed & 1u);
#pragma unroll
  for (int i = 0; i < kChains; ++i) x[i] = threadIdx.x * 7 + i + 1 + seed;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) r ^= x[i];
  if (r == 0x1234567u) sink[0] = r;
}

__global__ void __launch_bounds__(256) k_add_u32(uint32_t iters, uint32_t seed, uint64_t* sink) {
  uint32_t x[kChains];
  const uint32_t c = seed | 1u;
#pragma unroll
  for (int i = 0; i < kChains; ++i) x[i] = threadIdx.x * 7 + i + 1;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
  }
  uint32_t r = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) r ^= x[i];
  if (r == 0x1234567u) sink[0] = r;
}

// The library's exact 192-bit multiply-accumulate of two 64-bit values.
__global__ void __launch_bounds__(256) k_mac192(uint32_t iters, uint32_t seed, uint64_t* sink) {
  zr_acc192 acc[kChains];
  uint64_t q[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) {
    zr_acc_zero(acc[i]);
    q[i] = (uint64_t)seed * 0x9E3779B97F4A7C15ull + threadIdx.x + i;
  }
  const uint64_t v = ((uint64_t)seed << 32) | 0x89abcdefu;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) {
      zr_acc_mac(acc[i], q[i], v);
      q[i] += v;
    }
  }
  uint64_t x = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) x ^= acc[i].lo ^ acc[i].hi ^ acc[i].top;
  if (x == 0x123456789ull) sink[0] = x;
}

// Shoup product by a fixed multiplier (the synthetic-division chain step).
__global__ void __launch_bounds__(256) k_shoup(zr_mod M, uint32_t iters, uint32_t seed, uint64_t* sink) {
  uint64_t x[kChains];
  const uint64_t w = (((uint64_t)seed << 32) | 12345u) % M.p;
  const uint64_t wp = zr_shoup_pre(M, w);
#pragma unroll
  for (int i = 0; i < kChains; ++i) x[i] = (threadIdx.x * 1315423911ull + i) % M.p;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) x[i] = zr_shoup(M, x[i], w, wp);
  }
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) r ^= x[i];
  if (r == 0x123456789ull) sink[0] = r;
}

// LDS reads of 8 bytes per lane: at lane-consecutive addresses (the
// consumers' read of q) or, with BCAST, at one address per wave (a broadcast).
// The reads are volatile so that every one is issued; the addresses move with
// the iteration and stay inside the 16 KB array.
template <bool BCAST>
__global__ void __launch_bounds__(256) k_lds_read(uint32_t iters, uint32_t seed, uint64_t* sink) {
  __shared__ uint64_t buf[2048];
  for (uint32_t i = threadIdx.x; i < 2048; i += blockDim.x) buf[i] = (uint64_t)seed * (i + 1);
  __syncthreads();
  typedef const volatile __attribute__((address_space(3))) uint64_t lds_u64;
  lds_u64* lds = (lds_u64*)buf;  // LDS reads proper, not flat ones
  const uint32_t lane = BCAST ? 0 : (threadIdx.x & 63), wave = threadIdx.x >> 6;
  uint64_t x[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) x[i] = 0;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) x[i] += lds[(lane + 64 * ((wave + i + it) & 31)) & 2047];
  }
  uint64_t r = 0;
#pragma unroll
  for (int i = 0; i < kChains; ++i) r ^= x[i];
  if (r == 0x123456789ull) sink[0] = r;
}

__global__ void __launch_bounds__(256) k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" int zr_microbench(int kind, uint32_t blocks, uint32_t iters, uint64_t bytes, hipStream_t s,
                             double* ms_out, double* ops_out) {
  uint64_t* sink = nullptr;
  if (hipMalloc(&sink, 64) != hipSuccess) return -7;
  void* a = nullptr;
  void* b = nullptr;
  const uint32_t threads = 256;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double ops = 0;
  int rc = 0;
  const zr_mod M = zr_mod_make((1ull << 63) - 25);
  if (kind == ZR_MB_COPY) {
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) rc = -7;
    if (!rc) {
      (void)hipMemsetAsync(a, 1, bytes, s);
      hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(threads), 0, s, (const uint4*)a, (uint4*)b, bytes / 16);
    }
  }
  if (!rc) {
    // warm-up launch of the same kind, then the timed one
    for (int rep = 0; rep < 2; ++rep) {
      if (rep == 1) (void)hipEventRecord(e0, s);
      switch (kind) {
        case ZR_MB_MAD_U64_U32:
          hipLaunchKernelGGL(k_mad_u64_u32, dim3(blocks), dim3(threads), 0, s, iters, 7u, sink);
          break;
        case ZR_MB_MUL_LO_U32:
          hipLaunchKernelGGL(k_mul_lo_u32, dim3(blocks), dim3(threads), 0, s, iters, 7u, sink);
          break;
        case ZR_MB_MUL_HI_U32:
          hipLaunchKernelGGL(k_mul_hi_u32, dim3(blocks), dim3(threads), 0, s, iters, 7u, sink);
          break;
        case ZR_MB_ADD_U32:
          hipLaunchKernelGGL(k_add_u32, dim3(blocks), dim3(threads), 0, s, iters, 7u, sink);
          break;
        case ZR_MB_MAC192:
          hipLaunchKernelGGL(k_mac192, dim3(blocks), dim3(threads), 0, s, iters, 7u, sink);
          break;
        case ZR_MB_SHOUP:
          hipLaunchKernelGGL(k_shoup, dim3(blocks), dim3(threads), 0, s, M, iters, 7u, sink);
          break;
        case ZR_MB_COPY:
          hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(threads), 0, s, (const uint4*)a, (uint4*)b, bytes / 16);
          break;
        case ZR_MB_LDS_READ:
          hipLaunchKernelGGL(k_lds_read<false>, dim3(blocks), dim3(threads), 0, s, iters, 7u, sink);
          break;
        case ZR_MB_LDS_BCAST:
          hipLaunchKernelGGL(k_lds_read<true>, dim3(blocks), dim3(threads), 0, s, iters, 7u, sink);
          break;
        default:
          rc = -1;
      }
      if (rc) break;
    }
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) rc = -8;
  }
  float ms = 0;
  if (!rc) (void)hipEventElapsedTime(&ms, e0, e1);
  if (kind == ZR_MB_COPY) ops = 2.0 * (double)(bytes / 16) * 16;
  else if (kind == ZR_MB_LDS_READ || kind == ZR_MB_LDS_BCAST)
    ops = (double)blocks * threads * (double)iters * kChains * 8;  // bytes delivered to lanes
  else ops = (double)blocks * threads * (double)iters * kChains;
  if (ms_out) *ms_out = ms;
  if (ops_out) *ops_out = ops;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return rc;
}
