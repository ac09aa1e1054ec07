// One transposed Vandermonde solve that allocates nothing: the master
// polynomial's levels and the solve's workspace live in one fixed device array
// of this file, sized at build time, instead of in memory taken from the
// allocator.  For callers that cannot allocate device memory (code under
// stream capture, tight serving loops).  The kernels and their arguments are
// those of zr_vandermonde_solve; only where the workspace comes from differs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/zippel.h"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"
#include "kernels_dev.hpp"

namespace zr {

// 64 MiB of workspace per GPU, held from the library's load until the process
// ends.  Each device holds its own copy at its own address.
constexpr size_t kScratchWords = (size_t)8 << 20;
static __device__ __align__(256) uint64_t scratch[kScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device
// (the array's name is a host-side stand-in that no kernel may be given).
uint64_t* scratch_on_current_device() {
  int dev = -1;
  check(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    note_error("device ordinal %d outside the %d devices the no-allocation solve tracks", dev, kMaxDevices);
    throw Error(ZR_EDEVICE);
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      note_error("hipGetSymbolAddress(scratch) on device %d failed: %s", dev, hipGetErrorString(e));
      (void)hipGetLastError();
      throw Error(ZR_EDEVICE);
    }
    g_scratch_dev[dev] = (uint64_t*)p;
  }
  return g_scratch_dev[dev];
}

size_t round_words(size_t w) { return (w + 31) & ~(size_t)31; }  // 256-byte boundaries

// The plan of vsolve_plan, cut down until its workspace fits max_words: for
// the producer/consumer pass first fewer partial-sum slots (the same chunks in
// more launches), then fewer chunks; false when even one chunk does not fit.
// Every cut changes only the speed.
bool vsolve_plan_within(uint32_t t, uint32_t R, uint32_t num_cus, size_t max_words, VsolvePlan* out) {
  const VsolvePlan Q = vsolve_plan(t, R, num_cus);
  if (vsolve_workspace_words(Q) <= max_words) {
    *out = Q;
    return true;
  }
  const size_t per_slot = std::max<size_t>((size_t)Q.Rg * t, 1);
  if (Q.pc) {
    VsolvePlan P = Q;
    P.Sd = 1;
    const size_t w1 = vsolve_workspace_words(P);
    if (w1 <= max_words) {
      const uint32_t sd = (uint32_t)std::min<size_t>(Q.S, 1 + (max_words - w1) / per_slot);
      P.Sd = cdiv(P.S, cdiv(P.S, sd));
      *out = P;
      return true;
    }
  }
  // one chunk, then as many as fit: each adds 3 t words of chunk state, and
  // R t of partial sums unless the slots are shared (producer/consumer pass)
  VsolvePlan P = Q;
  P.S = P.Sd = 1;
  P.L = std::max<uint32_t>(1, t);
  const size_t base = vsolve_workspace_words(P);
  if (base > max_words) return false;
  const size_t per_chunk = 3 * (size_t)t + (Q.pc ? 0 : per_slot);
  const uint32_t smax = (uint32_t)std::min<size_t>(Q.S, 1 + (max_words - base) / std::max<size_t>(per_chunk, 1));
  P.L = std::max<uint32_t>(1, cdiv(t, smax));
  P.S = std::max<uint32_t>(1, cdiv(t, P.L));
  P.Sd = Q.pc ? 1 : P.S;
  if (vsolve_workspace_words(P) > max_words) return false;
  *out = P;
  return true;
}

}  // namespace
}  // namespace zr

using namespace zr;

extern "C" zr_status zr_vandermonde_solve_noalloc(uint64_t p, uint32_t t, uint32_t R, const uint64_t* d_mono,
                                                  const uint64_t* d_rhs, uint64_t* d_out, int32_t* d_status,
                                                  hipStream_t stream) {
  if (p < 3 || p >= ((uint64_t)1 << 63) || !d_status || t >= ((uint32_t)1 << 31)) return ZR_EINVAL;
  if (t && R && (!d_mono || !d_rhs || !d_out)) return ZR_EINVAL;
  if (!is_prime_u64(p)) return ZR_ENOTPRIME;
  try {
    // the fixed layout: master polynomial | its level buffers | solve workspace
    const size_t o_tmp = round_words(t);
    const size_t o_work = o_tmp + round_words(t ? master_tmp_words(t) : 0);
    VsolvePlan plan{};
    if (t && R) {
      if (o_work >= kScratchWords ||
          !vsolve_plan_within(t, R, device_cus(), kScratchWords - o_work, &plan)) {
        note_error("zr_vandermonde_solve_noalloc: t = %u, R = %u needs more than the %zu MiB workspace", t, R,
                   kScratchWords * 8 >> 20);
        return ZR_EINVAL;
      }
    }
    uint64_t* base = scratch_on_current_device();
    check(fill_i32(d_status, 0, 1, stream));
    if (t == 0 || R == 0) return ZR_OK;
    const zr_mod M = zr_mod_make(p);
    check(master_poly(M, t, d_mono, base, base + o_tmp, stream));
    check(vsolve(M, plan, d_mono, base, d_rhs, t, d_out, t, base + o_work, d_status, stream));
    return ZR_OK;
  } catch (const Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    return ZR_ENOMEM;
  } catch (...) {
    return ZR_EDEVICE;
  }
}
