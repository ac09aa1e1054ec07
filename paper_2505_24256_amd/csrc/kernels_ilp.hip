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

void launch_master_conv(dim3 grid, size_t shmem, hipStream_t s, const zr_mod& M, uint32_t t, uint32_t half,
                        uint32_t IC, uint32_t nic, const uint64_t* cur, const uint4* limbs, uint64_t* part,
                        uint64_t* nxt, uint4* limbs_nxt) {
  hipLaunchKernelGGL(k_master_conv, grid, dim3(64), shmem, s, M, t, half, IC, nic, cur, limbs, part, nxt, limbs_nxt);
}

}  // namespace zr
