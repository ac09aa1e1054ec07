// Zippel reconstruction without known degree bounds (Introduction: a result
// is accepted when further probes reproduce it).  Each stage samples x_k at
// its anchor and then at further nodes, a batch at a time (one master
// polynomial per stage, one solve per batch); after each batch
// every term's divided differences of the new orders,
//   b_m = sum_{i<=m} f_i / prod_{j<=m, j!=i} (x_i - x_j),
// are formed on the device and counted where nonzero.  The stage stops at the
// first order m whose last `confirm` orders vanish for every term; its degree
// is D = m - confirm and the terms are lifted over x_0..x_D as in the
// fixed-bound path.  The batch size changes only how many samples are drawn
// beyond the stop, never the stop itself.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "../../include/zippel.h"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"
#include "kernels_dev.hpp"

namespace zr {

// Nonzero divided differences of orders m0..m1-1 over the terms: one thread
// per term, exact 192-bit sums of the weighted values; per order, one atomic
// per wave of the wave's count.
__global__ void __launch_bounds__(256) k_ddiff_count(zr_mod M, uint32_t t, uint32_t m0, uint32_t m1, uint32_t ldw,
                                                     const uint64_t* __restrict__ wtab,
                                                     const uint64_t* __restrict__ vals, uint32_t* __restrict__ nz) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = l < t;
  for (uint32_t m = m0; m < m1; ++m) {
    bool nonzero = false;
    if (live) {
      zr_acc192 acc;
      zr_acc_zero(acc);
      for (uint32_t i = 0; i <= m; ++i) zr_acc_mac(acc, wtab[(size_t)m * ldw + i], vals[(size_t)i * t + l]);
      nonzero = zr_acc_reduce(M, acc) != 0;
    }
    const uint64_t b = __ballot(nonzero);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&nz[m], (uint32_t)__popcll(b));
  }
}

namespace {

// Nodes per black-box call and solve: 16 at a time.  Each solve reruns the
// synthetic-division chain (about eight right-hand sides' worth of work), so
// fewer, wider solves cost less; batches of 16 keep the samples drawn beyond
// a stage's stop below 16 and take the producer/consumer pass.  A stage's
// first batch is as wide as the previous stage's degree plus the confirming
// orders (at most kBatchGuess, one producer/consumer pass), so that a
// polynomial of even degrees needs one solve per stage.
constexpr uint32_t kBatchFirst = 16, kBatchMax = 16, kBatchGuess = 63;

// w[m][i] = 1 / prod_{j<=m, j!=i} (x_i - x_j) for m < X.size(), i <= m.
std::vector<uint64_t> ddiff_weights(const zr_mod& M, const std::vector<uint64_t>& X) {
  const size_t n = X.size();
  std::vector<uint64_t> den(n * n, 0), w(n * n, 0);
  for (size_t m = 0; m < n; ++m) {
    uint64_t dm = 1 % M.p;
    for (size_t i = 0; i < m; ++i) {
      den[m * n + i] = zr_mul(M, den[(m - 1) * n + i], zr_sub(M, X[i], X[m]));
      dm = zr_mul(M, dm, zr_sub(M, X[m], X[i]));
    }
    den[m * n + m] = dm;
    for (size_t i = 0; i <= m; ++i) w[m * n + i] = zr_inv(M, den[m * n + i]);
  }
  return w;
}

// Newton matrix limbs and powers of y for a lift over D1 nodes of variable v,
// laid out as the fixed-bound path's stage constants.
struct LiftConsts {
  uint32_t* W = nullptr;
  uint64_t* ypow = nullptr;
};
LiftConsts lift_consts(const Params& P, uint32_t v, const std::vector<uint64_t>& X, uint32_t D1, DevArena& A,
                       hipStream_t s) {
  std::vector<uint64_t> Xs(X.begin(), X.begin() + D1);
  std::vector<uint32_t> W = newton_matrix_limbs(P.M, Xs);
  W.resize(W.size() + 3 * 8 + 2, 0);  // the lift kernel fetches whole limb groups ahead of use
  std::vector<uint64_t> yp(2 * (size_t)D1);
  uint64_t acc = 1 % P.p;
  for (uint32_t d = 0; d < D1; ++d) {
    yp[d] = acc;
    yp[D1 + d] = zr_shoup_pre(P.M, acc);
    acc = zr_mul(P.M, acc, P.y[v]);
  }
  LiftConsts C;
  C.W = A.alloc<uint32_t>(W.size());
  C.ypow = A.alloc<uint64_t>(yp.size());
  h2d(C.W, W.data(), W.size() * 4, s);
  h2d(C.ypow, yp.data(), yp.size() * 8, s);
  check(hipStreamSynchronize(s));  // the host vectors go out of scope
  return C;
}

void reconstruct_adaptive(const zr_params* params, uint32_t confirm, zr_blackbox_fn bb, void* ctx, hipStream_t s,
                          zr_poly* out, uint32_t* deg_found) {
  if (!params || !bb || !params->deg || confirm == 0 || confirm > 8 || params->nvars == 0 || params->nvars > 64)
    throw Error(ZR_EINVAL);
  if ((params->last_stage && params->last_stage != params->nvars) || params->first_stage > 1 || params->deg_den)
    throw Error(ZR_EINVAL);
  const uint32_t n = params->nvars;
  // the schedule needs cap + confirm nodes per variable
  std::vector<uint32_t> need(n);
  for (uint32_t v = 0; v < n; ++v) need[v] = params->deg[v] + confirm;
  zr_params pm = *params;
  pm.deg = need.data();
  Params P(&pm, false);
  zr_counters& C = counters();
  C = zr_counters{};
  DevArena keep(s);
  std::vector<std::unique_ptr<DevArena>> arenas;
  int32_t* d_status = keep.alloc<int32_t>(1);
  check(fill_i32(d_status, 0, 1, s));
  Skeleton cur;
  cur.alloc(keep, n, 1);  // the empty monomial
  check(fill_u64(cur.mono, 1 % P.p, 1, s));
  check(fill_u64(cur.coef, 1 % P.p, 1, s));
  check(fill_u64((uint64_t*)cur.exps, 0, (n * 2 + 7) / 8, s));
  int32_t* h = host_scratch();
  uint32_t prevD = 0;  // degree found in the previous stage
  for (uint32_t k = 1; k <= n; ++k) {
    const uint32_t kv = k - 1, t = cur.t, maxm = need[kv];  // orders 1..maxm
    const std::vector<uint64_t> X = P.node_list(kv, maxm + 1);
    const std::vector<uint64_t> w = ddiff_weights(P.M, X);
    DevArena* kp = new DevArena(s);
    arenas.emplace_back(kp);
    Skeleton nxt;
    {
      DevArena A(s);
      const size_t tt = std::max<uint32_t>(t, 1);
      uint64_t* vals = A.alloc<uint64_t>((size_t)(maxm + 1) * tt);
      uint64_t* d_w = A.alloc<uint64_t>(w.size());
      uint32_t* d_nz = A.alloc<uint32_t>(maxm + 1);
      h2d(d_w, w.data(), w.size() * 8, s);
      check(fill_i32((int32_t*)d_nz, 0, maxm + 1, s));
      if (k == 1) call_bb(bb, ctx, P, 1, 1, P.y.data(), X.data(), 1, vals, s);
      else check(copy_u64(vals, cur.coef, t, s));
      // one master polynomial for all of the stage's solves
      uint64_t* Mc = nullptr;
      if (k >= 2 && t) {
        Mc = A.alloc<uint64_t>(t);
        uint64_t* tmp = A.alloc<uint64_t>(master_tmp_words(t));
        check(master_poly(P.M, t, cur.mono, Mc, tmp, s));
        C.mulmods += (uint64_t)t * (t - 1) / 2;
      }
      uint32_t m = 0, run = 0, stop = 0;
      uint32_t batch = k >= 2 ? std::min(std::max(kBatchFirst, prevD + confirm), kBatchGuess) : kBatchFirst;
      std::vector<uint32_t> nz(maxm + 1);
      while (!stop) {
        if (m == maxm) {
          note_error("stage %u: no %u vanishing orders within %u nodes", k, confirm, maxm);
          throw Error(ZR_EPROBE);
        }
        const uint32_t B = std::min(batch, maxm - m);
        batch = kBatchMax;
        uint64_t* rows = vals + (size_t)(m + 1) * t;
        call_bb(bb, ctx, P, k, k == 1 ? 1 : t, P.y.data(), X.data() + m + 1, B, rows, s);
        if (k >= 2 && t) {
          // rows m+1..m+B in place
          DevArena W(s);
          const VsolvePlan plan = vsolve_plan(t, B, device_cus());
          uint64_t* work = W.alloc<uint64_t>(vsolve_workspace_words(plan));
          check(vsolve(P.M, plan, cur.mono, Mc, rows, t, rows, t, work, d_status, s));
          count_solve(t, B);
          C.mulmods -= (uint64_t)t * (t - 1) / 2;  // the master polynomial is counted once per stage
        }
        if (t)
          hipLaunchKernelGGL(k_ddiff_count, dim3(cdiv(t, 256)), dim3(256), 0, s, P.M, t, m + 1, m + 1 + B,
                             (uint32_t)X.size(), d_w, vals, d_nz);
        check(hipGetLastError());
        check(hipMemcpyAsync(nz.data() + m + 1, d_nz + m + 1, B * 4, hipMemcpyDeviceToHost, s));
        check(hipMemcpyAsync(&h[0], d_status, 4, hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
        if (h[0] != 0) throw Error(h[0]);
        for (uint32_t o = m + 1; o <= m + B && !stop; ++o) {
          run = nz[o] == 0 ? run + 1 : 0;
          if (run == confirm) stop = o;
        }
        m += B;
      }
      const uint32_t D = stop - confirm;
      if (deg_found) deg_found[kv] = D;
      prevD = D;
      const LiftConsts L = lift_consts(P, kv, X, D + 1, A, s);
      lift_stage(P, kv, cur, vals, D + 1, L.W, L.ypow, *kp, nxt, s, d_status);
    }
    if (arenas.size() > 1) arenas.erase(arenas.begin());
    cur = nxt;
    C.stages = k;
  }
  if (P.nprobes) check_probes(P, bb, ctx, cur, nullptr, s);
  download(cur, s, out);
}

}  // namespace
}  // namespace zr

using namespace zr;

extern "C" zr_status zippel_reconstruct_adaptive(const zr_params* params, uint32_t confirm, zr_blackbox_fn bb,
                                                 void* ctx, hipStream_t stream, zr_poly* out, uint32_t* deg_found) {
  if (!out) return ZR_EINVAL;
  *out = zr_poly{};
  try {
    reconstruct_adaptive(params, confirm, bb, ctx, stream, out, deg_found);
    return ZR_OK;
  } catch (const Error& e) {
    zr_poly_free(out);
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    zr_poly_free(out);
    return ZR_ENOMEM;
  } catch (...) {
    zr_poly_free(out);
    return ZR_EDEVICE;
  }
}
