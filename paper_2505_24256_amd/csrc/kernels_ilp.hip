// Kernels whose time goes to dependent-instruction latency at one or two
// waves per SIMD: the matrix-core dot-product pass (two modular chains per
// lane beside 256 accumulator registers) and the product-tree convolution.
// This file is compiled with LLVM's latency-aware (iterative-ilp) machine
// scheduler, which measured faster on both; the integer-VALU solve kernels in
// kernels.hip keep the default scheduler, under which they use fewer
// registers and keep two waves per SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.hpp"
#include "kernels.hpp"
#include "kernels_dev.hpp"

namespace zr {

template <int NT, bool LAZY>
__global__ void __launch_bounds__(64) k_vs_mfma(VsArgs a, const uint32_t* __restrict__ Dg, uint32_t tp, uint32_t RT) {
  if (blockIdx.z == 0) vs_mfma_body<NT, true, LAZY>(a, Dg, tp, RT, blockIdx.x, blockIdx.y, 0);
  else vs_mfma_body<NT, false, LAZY>(a, Dg, tp, RT, blockIdx.x, blockIdx.y, blockIdx.z);
}

typedef void (*MfKernel)(VsArgs, const uint32_t*, uint32_t, uint32_t);
static MfKernel mf_kernel(uint32_t NT, bool lazy) {
  static const MfKernel table[2][kMfMaxNT + 1] = {
      {nullptr, k_vs_mfma<1, false>, k_vs_mfma<2, false>, k_vs_mfma<3, false>, k_vs_mfma<4, false>,
       k_vs_mfma<5, false>, k_vs_mfma<6, false>, k_vs_mfma<7, false>, k_vs_mfma<8, false>},
      {nullptr, k_vs_mfma<1, true>, k_vs_mfma<2, true>, k_vs_mfma<3, true>, k_vs_mfma<4, true>, k_vs_mfma<5, true>,
       k_vs_mfma<6, true>, k_vs_mfma<7, true>, k_vs_mfma<8, true>}};
  return NT >= 1 && NT <= kMfMaxNT ? table[lazy ? 1 : 0][NT] : nullptr;
}

hipError_t launch_vs_mfma(uint32_t NT, bool lazy, dim3 grid, hipStream_t s, const VsArgs& a, const uint32_t* Dg,
                          uint32_t tp, uint32_t RT) {
  MfKernel km = mf_kernel(NT, lazy);
  if (!km) return hipErrorInvalidValue;
  hipLaunchKernelGGL(km, grid, dim3(64), 0, s, a, Dg, tp, RT);
  return hipGetLastError();
}

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
