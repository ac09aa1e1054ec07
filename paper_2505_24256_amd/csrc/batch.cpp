// vandermonde_solve_batch: many transposed Vandermonde systems (§1, §2.2;
// the "several expressions" solved at once by the multi-prime routine of §2.2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/zippel.h"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"

namespace zr {

static void solve_batch(size_t nsys, uint64_t p, const uint64_t* h_sys_off, const uint64_t* d_mono,
                        const uint32_t* h_nrhs, const uint64_t* h_rhs_off, const uint64_t* d_rhs, uint64_t* d_out,
                        int32_t* d_status, hipStream_t s) {
  const zr_mod M = zr_mod_make(p);
  DevArena A(s);
  check(fill_i32(d_status, 0, nsys, s));
  uint64_t tmax = 0;
  size_t wmax = 0;
  for (size_t i = 0; i < nsys; ++i) {
    const uint64_t t = h_sys_off[i + 1] - h_sys_off[i];
    tmax = std::max(tmax, t);
    if (t && h_nrhs[i]) wmax = std::max(wmax, vsolve_workspace_words(vsolve_plan((uint32_t)t, h_nrhs[i], device_cus())));
  }
  uint64_t* Mc = A.alloc<uint64_t>(std::max<uint64_t>(tmax, 1));
  uint64_t* tmp = A.alloc<uint64_t>(master_tmp_words((uint32_t)std::max<uint64_t>(tmax, 1)));
  uint64_t* work = A.alloc<uint64_t>(std::max<size_t>(wmax, 1));
  for (size_t i = 0; i < nsys; ++i) {
    const uint32_t t = (uint32_t)(h_sys_off[i + 1] - h_sys_off[i]);
    const uint32_t R = h_nrhs[i];
    if (t == 0 || R == 0) continue;
    const uint64_t* mono = d_mono + h_sys_off[i];
    check(master_poly(M, t, mono, Mc, tmp, s));
    const VsolvePlan plan = vsolve_plan(t, R, device_cus());
    check(vsolve(M, plan, mono, Mc, d_rhs + h_rhs_off[i], t, d_out + h_rhs_off[i], t, work, d_status + i, s));
  }
}

}  // namespace zr

extern "C" zr_status vandermonde_solve_batch(size_t nsys, uint64_t p, const uint64_t* d_sys_off,
                                             const uint64_t* h_sys_off, const uint64_t* d_mono,
                                             const uint32_t* h_nrhs, const uint64_t* d_rhs_off,
                                             const uint64_t* h_rhs_off, const uint64_t* d_rhs, uint64_t* d_out,
                                             int32_t* d_status, hipStream_t stream) {
  (void)d_sys_off;
  (void)d_rhs_off;
  if (nsys == 0) return ZR_OK;
  if (p < 3 || p >= ((uint64_t)1 << 63) || !h_sys_off || !h_nrhs || !h_rhs_off || !d_status) return ZR_EINVAL;
  if (!zr::is_prime_u64(p)) return ZR_ENOTPRIME;
  for (size_t i = 0; i < nsys; ++i) {
    if (h_sys_off[i + 1] < h_sys_off[i]) return ZR_EINVAL;
    const uint64_t t = h_sys_off[i + 1] - h_sys_off[i];
    if (t >= ((uint64_t)1 << 31)) return ZR_EINVAL;
    if (h_rhs_off[i + 1] - h_rhs_off[i] != t * h_nrhs[i]) return ZR_EINVAL;
  }
  if (h_sys_off[nsys] && (!d_mono || !d_rhs || !d_out)) return ZR_EINVAL;
  try {
    zr::solve_batch(nsys, p, h_sys_off, d_mono, h_nrhs, h_rhs_off, d_rhs, d_out, d_status, stream);
    return ZR_OK;
  } catch (const zr::Error& e) {
    return (zr_status)e.code;
  }
}
