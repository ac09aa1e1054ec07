// Host driver of balanced Zippel for rational functions f = P/Q (§1, §2.2).
//
// Stage 1: Thiele in x_1 (eq. 2) gives N_1/D_1 scaled so that the lowest
// nonzero coefficient of D_1 is 1; this fixes one unknown common factor C with
// N_1 = C P(x_1, anchors), D_1 = C Q(x_1, anchors).
// Stage k: for each slice i = 1..T (T = max(t_N, t_D)), Thiele in x_k at
// x_{<k} = y^i gives A_i/B_i = h_i P/h_i Q with an unknown h_i.  The balancing
// factor beta_i = N_{k-1}(y^i)/A_i(c_k) = C/h_i (falling back to the
// denominator when either factor vanishes) makes beta_i A_i(x_k^(j)) and
// beta_i B_i(x_k^(j)) the values of C P and C Q, so numerator and denominator
// are each lifted by the polynomial Zippel step.  Finally D(0) is scaled to 1.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "../../include/zippel.h"
#include "batch.hpp"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"

namespace zr {

// Download a device int32 array.
static std::vector<int32_t> d2h_i32(const int32_t* d, size_t n, hipStream_t s) {
  std::vector<int32_t> h(n);
  d2h_sync(h.data(), d, n * 4, s);
  return h;
}

// Build a univariate skeleton (in variable 0) from host coefficients c[0..deg].
// Host arrays of the stage-1 skeleton with coefficients c (c_r of x_1^r):
// the nonzero r in order, exponents in the variable-0 row of the SoA layout,
// monomial values y_1^r.  Returns the term count.
uint32_t stage1_skeleton_host(const Params& P, const std::vector<uint64_t>& c, std::vector<uint16_t>& exps,
                              std::vector<uint64_t>& coef, std::vector<uint64_t>& mono) {
  std::vector<uint32_t> idx;
  for (uint32_t r = 0; r < c.size(); ++r)
    if (c[r]) idx.push_back(r);
  const uint32_t t = (uint32_t)idx.size();
  exps.assign((size_t)P.nvars * std::max<uint32_t>(t, 1), 0);
  coef.assign(std::max<uint32_t>(t, 1), 0);
  mono.assign(std::max<uint32_t>(t, 1), 0);
  for (uint32_t l = 0; l < t; ++l) {
    exps[l] = (uint16_t)idx[l];
    coef[l] = c[idx[l]];
    mono[l] = zr_pow(P.M, P.y[0], idx[l]);
  }
  return t;
}

void host_skeleton(const Params& P, const std::vector<uint64_t>& c, DevArena& keep, Skeleton& S,
                          hipStream_t s) {
  std::vector<uint16_t> exps;
  std::vector<uint64_t> coef, mono;
  const uint32_t t = stage1_skeleton_host(P, c, exps, coef, mono);
  S.alloc(keep, P.nvars, t);
  if (t) {
    h2d(S.exps, exps.data(), (size_t)P.nvars * t * 2, s);
    h2d(S.coef, coef.data(), (size_t)t * 8, s);
    h2d(S.mono, mono.data(), (size_t)t * 8, s);
  }
  check(hipStreamSynchronize(s));
}

// Combine the per-slice statuses and degrees like the definition: the most
// negative slice status first, then the slices must agree on (deg A, deg B)
// and respect the bounds.
void check_slices(const std::vector<int32_t>& st, const std::vector<int32_t>& dA,
                         const std::vector<int32_t>& dB, uint32_t bn, uint32_t bd, int32_t& rhoN, int32_t& rhoD) {
  int32_t worst = 0;
  for (int32_t v : st) worst = std::min(worst, v);
  if (worst) throw Error(worst);
  if (dA.empty()) {
    rhoN = rhoD = 0;
    return;
  }
  rhoN = dA[0];
  rhoD = dB[0];
  for (size_t i = 0; i < dA.size(); ++i)
    if (dA[i] != rhoN || dB[i] != rhoD) throw Error(ZR_EDEGEN);
  if (rhoN > (int32_t)bn || rhoD > (int32_t)bd) throw Error(ZR_EDEGEN);
}

// Stage 1: Thiele in x_1 from the anchor and the first nodes (eq. 2); the
// numerator and denominator become univariate skeletons in `keep`.
void balanced_stage1(const Params& P, zr_blackbox_fn bb, void* ctx, DevArena& keep, Skeleton& SN, Skeleton& SD,
                     hipStream_t s) {
  const uint32_t n1 = P.nnodes[0] + 1;
  std::vector<uint64_t> X = P.node_list(0, n1);
  DevArena A(s);
  uint64_t* F = A.alloc<uint64_t>(n1);
  uint64_t* dX = A.alloc<uint64_t>(n1);
  uint64_t* dA = A.alloc<uint64_t>(n1 + 1);
  uint64_t* dB = A.alloc<uint64_t>(n1 + 1);
  int32_t* dg = A.alloc<int32_t>(3);
  const size_t sw = thiele_scratch_words(1, n1);
  uint64_t* scr = sw ? A.alloc<uint64_t>(sw) : nullptr;
  h2d(dX, X.data(), n1 * 8, s);
  call_bb(bb, ctx, P, 1, 1, P.y.data(), X.data(), n1, F, s);
  check(thiele_slices(P.M, 1, n1, dX, F, dA, dB, dg, dg + 1, dg + 2, scr, s));
  std::vector<int32_t> g = d2h_i32(dg, 3, s);
  int32_t rn, rd;
  check_slices({g[2]}, {g[0]}, {g[1]}, P.deg[0], P.deg_den[0], rn, rd);
  std::vector<uint64_t> ca(rn + 1), cb(rd + 1);
  d2h_sync(ca.data(), dA, (rn + 1) * 8, s);
  d2h_sync(cb.data(), dB, (rd + 1) * 8, s);
  host_skeleton(P, ca, keep, SN, s);
  host_skeleton(P, cb, keep, SD, s);
}

// After the last stage: scale so that D(0) = 1 (ZR_ENORM if D has no constant
// term), check the probes, download.
void balanced_finish(const Params& P, zr_blackbox_fn bb, void* ctx, Skeleton& SN, Skeleton& SD, hipStream_t s,
                     zr_poly* num, zr_poly* den) {
  if (P.last == P.nvars) {
    uint64_t c0 = 0;
    if (SD.t) {
      std::vector<uint16_t> e0(P.nvars);
      for (uint32_t v = 0; v < P.nvars; ++v) d2h_sync(&e0[v], SD.exps + (size_t)v * SD.t, 2, s);
      bool zero = true;
      for (uint16_t e : e0) zero &= e == 0;
      if (zero) d2h_sync(&c0, SD.coef, 8, s);
    }
    if (c0 == 0) throw Error(ZR_ENORM);
    const uint64_t ci = zr_inv(P.M, c0);
    check(scale_u64(P.M, SN.coef, SN.t, ci, s));
    check(scale_u64(P.M, SD.coef, SD.t, ci, s));
    if (P.nprobes) check_probes(P, bb, ctx, SN, &SD, s);
  }
  download(SN, s, num);
  download(SD, s, den);
}

static void reconstruct_balanced(const zr_params* params, zr_blackbox_fn bb, void* ctx, hipStream_t s, zr_poly* num,
                                 zr_poly* den) {
  Params P(params, true);
  counters() = zr_counters{};
  DevArena keep(s);
  int32_t* d_status = keep.alloc<int32_t>(1);
  check(fill_i32(d_status, 0, 1, s));
  std::vector<std::unique_ptr<DevArena>> arenas;
  Skeleton SN, SD;
  {
    auto* kp = new DevArena(s);
    arenas.emplace_back(kp);
    balanced_stage1(P, bb, ctx, *kp, SN, SD, s);
  }
  counters().stages = 1;
  // ---- stages k >= 2 ---------------------------------------------------------
  for (uint32_t k = 2; k <= P.last; ++k) {
    const uint32_t kvar = k - 1;
    const uint32_t tN = SN.t, tD = SD.t, T = std::max(tN, tD);
    const uint32_t nk = P.nnodes[kvar] + 1;
    std::vector<uint64_t> X = P.node_list(kvar, nk);
    auto* kp = new DevArena(s);
    arenas.emplace_back(kp);
    Skeleton nN, nD;
    {
      DevArena A(s);
      uint64_t* dX = A.alloc<uint64_t>(nk);
      h2d(dX, X.data(), nk * 8, s);
      uint64_t* F = A.alloc<uint64_t>((size_t)nk * std::max<uint32_t>(T, 1));
      call_bb(bb, ctx, P, k, T, P.y.data(), X.data(), nk, F, s);
      uint64_t* cA = A.alloc<uint64_t>((size_t)(nk + 1) * std::max<uint32_t>(T, 1));
      uint64_t* cB = A.alloc<uint64_t>((size_t)(nk + 1) * std::max<uint32_t>(T, 1));
      const uint32_t T1 = std::max<uint32_t>(T, 1);
      int32_t* dgA = A.alloc<int32_t>(3 * (size_t)T1);  // degrees of A, of B, slice statuses
      int32_t* dgB = dgA + T1;
      int32_t* dst = dgB + T1;
      const size_t sw = thiele_scratch_words(T, nk);
      uint64_t* scr = sw ? A.alloc<uint64_t>(sw) : nullptr;
      check(thiele_slices(P.M, T, nk, dX, F, cA, cB, dgA, dgB, dst, scr, s));
      // previous numerator and denominator at the Zippel points y^i, i = 1..T
      uint64_t* nprev = A.alloc<uint64_t>(T1);
      uint64_t* dprev = A.alloc<uint64_t>(T1);
      const size_t ww = std::max(vapply_work_words(tN, T), vapply_work_words(tD, T));
      uint64_t* wk = A.alloc<uint64_t>(ww);
      check(vapply(P.M, tN, SN.mono, SN.coef, T, nprev, wk, ww, s));
      check(vapply(P.M, tD, SD.mono, SD.coef, T, dprev, wk, ww, s));
      counters().mulmods += (uint64_t)T * (tN + tD);
      // one read-back of every slice's degrees and status
      int32_t* h = host_words(3 * (size_t)T1);
      check(hipMemcpyAsync(h, dgA, 3 * (size_t)T1 * 4, hipMemcpyDeviceToHost, s));
      check(hipStreamSynchronize(s));
      int32_t rhoN = 0, rhoD = 0;
      check_slices(std::vector<int32_t>(h + 2 * (size_t)T1, h + 2 * (size_t)T1 + T),
                   std::vector<int32_t>(h, h + T), std::vector<int32_t>(h + T1, h + T1 + T), P.deg[kvar],
                   P.deg_den[kvar], rhoN, rhoD);
      // balanced right-hand sides into the Newton value arrays; a slice without
      // a balancing factor marks the reconstruction degenerate (read back with
      // the lift's statuses)
      const uint32_t D1N = (uint32_t)rhoN + 1, D1D = (uint32_t)rhoD + 1;
      uint64_t* valsN = A.alloc<uint64_t>((size_t)D1N * std::max<uint32_t>(tN, 1));
      uint64_t* valsD = A.alloc<uint64_t>((size_t)D1D * std::max<uint32_t>(tD, 1));
      check(copy_u64(valsN, SN.coef, tN, s));
      check(copy_u64(valsD, SD.coef, tD, s));
      check(fill_i32(dst, 0, T, s));
      check(balance_rhs(P.M, T, nk, dX, cA, cB, dgA, dgB, nprev, dprev, tN, rhoN, valsN + tN, tN, tD, rhoD,
                        valsD + tD, tD, dst, A.alloc<uint64_t>(T1), s));
      check(fold_status(dst, T, d_status, ZR_EDEGEN, s));
      solve_stage(P, SN, valsN, (uint32_t)rhoN, s, d_status);
      solve_stage(P, SD, valsD, (uint32_t)rhoD, s, d_status);
      // Newton matrices (built on the device) and the lifts of N and D, one read-back
      uint64_t* cwN = A.alloc<uint64_t>(newton_W_words(D1N) / 2 + 2 + 2 * (size_t)D1N);
      uint64_t* cwD = A.alloc<uint64_t>(newton_W_words(D1D) / 2 + 2 + 2 * (size_t)D1D);
      const std::vector<ConstsJob> cj{
          ConstsJob{D1N, X.data(), P.y[kvar], (uint32_t*)cwN, cwN + newton_W_words(D1N) / 2 + 1},
          ConstsJob{D1D, X.data(), P.y[kvar], (uint32_t*)cwD, cwD + newton_W_words(D1D) / 2 + 1}};
      batched_consts(P.M, cj, s);
      const std::vector<LiftJob> lj{
          LiftJob{kvar, D1N, &SN, valsN, cj[0].Wl, cj[0].ypow, d_status, &nN},
          LiftJob{kvar, D1D, &SD, valsD, cj[1].Wl, cj[1].ypow, d_status, &nD}};
      for (int32_t v : batched_lift(P.M, lj, *kp, s))
        if (v) throw Error(v);
    }
    arenas.erase(arenas.begin());
    SN = nN;
    SD = nD;
    counters().stages = k;
  }
  balanced_finish(P, bb, ctx, SN, SD, s, num, den);
}

}  // namespace zr

extern "C" zr_status zippel_balanced_reconstruct(const zr_params* params, zr_blackbox_fn bb, void* ctx,
                                                 hipStream_t stream, zr_poly* num, zr_poly* den) {
  if (!num || !den || !bb) return ZR_EINVAL;
  *num = zr_poly{0, 0, nullptr, nullptr};
  *den = zr_poly{0, 0, nullptr, nullptr};
  try {
    zr::reconstruct_balanced(params, bb, ctx, stream, num, den);
    return ZR_OK;
  } catch (const zr::Error& e) {
    zr_poly_free(num);
    zr_poly_free(den);
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    zr_poly_free(num);
    zr_poly_free(den);
    return ZR_ENOMEM;
  }
}

extern "C" zr_status zr_thiele_slices(uint64_t p, uint32_t T, uint32_t nk, const uint64_t* d_X, const uint64_t* d_F,
                                      uint64_t* d_A, uint64_t* d_B, int32_t* d_degA, int32_t* d_degB,
                                      int32_t* d_status, hipStream_t stream) {
  if (T == 0) return ZR_OK;
  if (p < 3 || p >= ((uint64_t)1 << 63) || nk == 0 || !d_X || !d_F || !d_A || !d_B || !d_degA || !d_degB ||
      !d_status)
    return ZR_EINVAL;
  if (!zr::is_prime_u64(p)) return ZR_ENOTPRIME;
  try {
    const zr_mod M = zr_mod_make(p);
    zr::DevArena A(stream);  // blocks return to a cache ordered on `stream`: no synchronisation
    const size_t sw = zr::thiele_scratch_words(T, nk);
    uint64_t* scr = sw ? A.alloc<uint64_t>(sw) : nullptr;
    check(zr::thiele_slices(M, T, nk, d_X, d_F, d_A, d_B, d_degA, d_degB, d_status, scr, stream));
    return ZR_OK;
  } catch (const zr::Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    return ZR_ENOMEM;
  }
}
