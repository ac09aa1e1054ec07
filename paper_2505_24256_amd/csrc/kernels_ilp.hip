// The product-tree convolution, whose time goes to dependent-instruction
// latency at one wave per SIMD.  This file is compiled with LLVM's
// latency-aware (iterative-ilp) machine scheduler, which measured faster on
// it; the integer-VALU solve kernels in kernels.hip keep the default
// scheduler, under which they use fewer registers and keep more waves per SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.hpp"
#include "kernels.hpp"
#include "kernels_dev.hpp"

namespace zr {

__global__ void __launch_bounds__(64) k_master_conv(zr_mod M, uint32_t t, uint32_t half, uint32_t IC, uint32_t nic,
                                                    const uint64_t* __restrict__ cur, const uint4* __restrict__ limbs,
                                                    uint64_t* __restrict__ part, uint64_t* __restrict__ nxt,
                                                    uint4* __restrict__ limbs_nxt) {
  extern __shared__ uint64_t win[];  // 64 + IC + 8 words
  master_conv_body(M, t, half, IC, nic, blockIdx.x * 64, blockIdx.y, cur, limbs, part, t, nxt, limbs_nxt, win);
}

// four waves sharing one window, for factors of degree half >= 128
__global__ void __launch_bounds__(256) k_master_conv4(zr_mod M, uint32_t t, uint32_t half, uint32_t IC, uint32_t nic,
                                                      const uint64_t* __restrict__ cur, const uint4* __restrict__ limbs,
                                                      uint64_t* __restrict__ part, uint64_t* __restrict__ nxt,
                                                      uint4* __restrict__ limbs_nxt) {
  extern __shared__ uint64_t win[];  // 256 + IC + 8 words
  master_conv_body<4>(M, t, half, IC, nic, blockIdx.x * 256, blockIdx.y, cur, limbs, part, t, nxt, limbs_nxt, win);
}

// One level of the product tree: for half >= 128 four waves share each
// window (at IC = 4096 a one-wave window of 33 KB left one wave per SIMD; a
// four-wave window of 35 KB leaves four).
void launch_master_conv(hipStream_t s, const zr_mod& M, uint32_t t, uint32_t half, uint32_t IC, uint32_t nic,
                        const uint64_t* cur, const uint4* limbs, uint64_t* part, uint64_t* nxt, uint4* limbs_nxt) {
  if (half >= 128)
    hipLaunchKernelGGL(k_master_conv4, dim3(cdiv(t, 256), nic), dim3(256), (256 + IC + 8) * 8, s, M, t, half, IC, nic,
                       cur, limbs, part, nxt, limbs_nxt);
  else
    hipLaunchKernelGGL(k_master_conv, dim3(cdiv(t, 64), nic), dim3(64), (64 + IC + 8) * 8, s, M, t, half, IC, nic,
                       cur, limbs, part, nxt, limbs_nxt);
}

}  // namespace zr
