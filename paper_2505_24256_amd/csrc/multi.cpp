// Several expressions reconstructed together over one skeleton (§2.2: the
// solve serves several expressions of various degrees at once; its cost grows
// with the square of the system size plus the size times the number of
// right-hand sides).  All expressions are sampled at the same points; stage k
// solves ONE transposed Vandermonde system on the union U of the expressions'
// stage-(k-1) skeletons, with sum_e D_k^(e) right-hand sides.  A monomial of U
// absent from expression e has coefficient zero in e at every node, so the
// union costs nothing in exactness.  Each expression is then lifted by its own
// Newton interpolation (D_k^(e) + 1 nodes, the first ones of the shared node
// list), and the next union keeps (l, d) when any expression has a nonzero
// coefficient there.  State on the device: the union's exponents and monomial
// values, and a coefficient matrix [E][|U|] with zeros where a term is absent.
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

constexpr uint32_t kMaxExpr = 64;

struct MultiExpr {
  uint32_t E;               // expressions
  uint32_t Dmax1;           // max over e of D1[e]
  uint32_t D1[kMaxExpr];    // Newton nodes of expression e at this stage (D_k^(e) + 1)
  uint64_t goff[kMaxExpr];  // offset (words) of expression e's g [D1[e]][t] in the packed G
};

// Terms (l, d) of the next union per l: d < Dmax1 with a nonzero g_e[d][l] in some e.
__global__ void k_multi_count(uint32_t t, MultiExpr X, const uint64_t* __restrict__ G, uint32_t* __restrict__ cnt) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t) return;
  uint32_t c = 0;
  for (uint32_t d = 0; d < X.Dmax1; ++d) {
    bool any = false;
    for (uint32_t e = 0; e < X.E && !any; ++e) any = d < X.D1[e] && G[X.goff[e] + (size_t)d * t + l] != 0;
    c += any ? 1 : 0;
  }
  cnt[l] = c;
}

// Next union in lexicographic order (l-major, d ascending), its monomial
// values m_l y_k^d and every expression's coefficient (0 where absent).
__global__ void k_multi_expand(zr_mod M, uint32_t t, MultiExpr X, uint32_t kvar, uint32_t nvars,
                               const uint16_t* __restrict__ exps_old, const uint64_t* __restrict__ mono_old,
                               const uint64_t* __restrict__ G, const uint32_t* __restrict__ off,
                               const uint64_t* __restrict__ ypow, const uint64_t* __restrict__ ypowp,
                               uint16_t* __restrict__ exps_new, uint64_t* __restrict__ mono_new,
                               uint64_t* __restrict__ coef_new, uint32_t ld_new) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t) return;
  uint32_t pos = off[l];
  const uint64_t m = mono_old[l];
  for (uint32_t d = 0; d < X.Dmax1; ++d) {
    bool any = false;
    for (uint32_t e = 0; e < X.E && !any; ++e) any = d < X.D1[e] && G[X.goff[e] + (size_t)d * t + l] != 0;
    if (!any) continue;
    for (uint32_t v = 0; v < nvars; ++v)
      exps_new[(size_t)v * ld_new + pos] = v == kvar ? (uint16_t)d : exps_old[(size_t)v * t + l];
    mono_new[pos] = zr_shoup(M, m, ypow[d], ypowp[d]);
    for (uint32_t e = 0; e < X.E; ++e)
      coef_new[(size_t)e * ld_new + pos] = d < X.D1[e] ? G[X.goff[e] + (size_t)d * t + l] : 0;
    ++pos;
  }
}

namespace {

struct Union {
  uint32_t t = 0;
  uint16_t* exps = nullptr;  // [nvars][t]
  uint64_t* mono = nullptr;  // [t]
  uint64_t* coef = nullptr;  // [E][t]
};

// All expressions' right-hand sides in one solve over the union skeleton: one
// master polynomial, and one chain pass and inversion for all (vsolve takes
// more than kPcMaxR right-hand sides in groups).
void solve_groups(const Params& P, const Union& U, uint64_t* rhs, uint32_t R, hipStream_t s, int32_t* d_status) {
  const uint32_t t = U.t;
  if (t == 0 || R == 0) return;
  DevArena A(s);
  uint64_t* Mc = A.alloc<uint64_t>(t);
  uint64_t* tmp = A.alloc<uint64_t>(master_tmp_words(t));
  check(master_poly(P.M, t, U.mono, Mc, tmp, s));
  const VsolvePlan plan = vsolve_plan(t, R, device_cus());
  uint64_t* work = A.alloc<uint64_t>(vsolve_workspace_words(plan));
  check(vsolve(P.M, plan, U.mono, Mc, rhs, t, rhs, t, work, d_status, s));
  count_solve(t, R);
}

void call_box_multi(zr_blackbox_fn bb, void* ctx, const Params& P, uint32_t E, uint32_t k, uint64_t ni,
                    const uint64_t* y, const uint64_t* xk, uint64_t nj, uint64_t* d_vals, hipStream_t s) {
  zr_points pts;
  pts.nvars = P.nvars;
  pts.k = k;
  pts.i_first = 1;
  pts.ni = ni;
  pts.nj = nj;
  pts.y = y;
  pts.anchor = P.anchor.data();
  pts.xk = xk;
  pts.p = P.p;
  pts.nexpr = E;
  if (ni == 0 || nj == 0) return;
  if (bb(ctx, &pts, d_vals, s) != 0) throw Error(ZR_EBLACKBOX);
}

// Newton per expression and the next union.  vals_e [D1_e][t] per expression
// (row 0: the coefficients at the anchor node); K[e] holds expression e's
// Newton matrices, Kmax the powers of y up to the largest degree.
Union lift_multi(const Params& P, uint32_t kvar, const Union& U, const std::vector<uint64_t*>& vals,
                 const std::vector<uint32_t>& D1, const std::vector<std::unique_ptr<StageConsts>>& K,
                 const StageConsts& Kmax, DevArena& keep, hipStream_t s, int32_t* d_status) {
  const uint32_t E = (uint32_t)D1.size(), t = U.t;
  DevArena A(s);
  MultiExpr X{};
  X.E = E;
  size_t gw = 0;
  for (uint32_t e = 0; e < E; ++e) {
    X.D1[e] = D1[e];
    X.Dmax1 = std::max(X.Dmax1, D1[e]);
    X.goff[e] = gw;
    gw += (size_t)D1[e] * t;
  }
  uint64_t* G = A.alloc<uint64_t>(std::max<size_t>(gw, 1));
  uint32_t* cnt = A.alloc<uint32_t>(std::max<uint32_t>(t, 1));
  uint32_t* off = A.alloc<uint32_t>((size_t)t + 1);
  uint32_t* tmp = A.alloc<uint32_t>(scan_tmp_words(t));
  for (uint32_t e = 0; e < E; ++e) {
    check(newton_lift(P.M, t, D1[e], vals[e], K[e]->W(kvar), G + X.goff[e], cnt, s));
    count_newton(t, D1[e]);
  }
  if (t) hipLaunchKernelGGL(k_multi_count, dim3(cdiv(t, 256)), dim3(256), 0, s, t, X, G, cnt);
  check(hipGetLastError());
  if (t == 0) check(fill_i32((int32_t*)off, 0, 1, s));
  else check(exclusive_scan(t, cnt, off, tmp, s));
  int32_t* h = host_scratch();
  check(hipMemcpyAsync(&h[0], off + t, 4, hipMemcpyDeviceToHost, s));
  check(hipMemcpyAsync(&h[1], d_status, 4, hipMemcpyDeviceToHost, s));
  check(hipStreamSynchronize(s));
  if (h[1] != 0) throw Error(h[1]);
  Union N;
  N.t = (uint32_t)h[0];
  const size_t tn = std::max<uint32_t>(N.t, 1);
  N.exps = keep.alloc<uint16_t>((size_t)P.nvars * tn);
  N.mono = keep.alloc<uint64_t>(tn);
  N.coef = keep.alloc<uint64_t>((size_t)E * tn);
  const uint64_t* yp = Kmax.ypow(kvar);
  if (t)
    hipLaunchKernelGGL(k_multi_expand, dim3(cdiv(t, 256)), dim3(256), 0, s, P.M, t, X, kvar, P.nvars, U.exps,
                       U.mono, G, off, yp, yp + X.Dmax1, N.exps, N.mono, N.coef, (uint32_t)tn);
  check(hipGetLastError());
  return N;
}

void check_probes_multi(const Params& P, uint32_t E, zr_blackbox_fn bb, void* ctx, const Union& U, hipStream_t s) {
  DevArena A(s);
  const uint32_t np = P.nprobes, nv = P.nvars;
  uint32_t ld = 1;
  for (uint32_t v = 0; v < nv; ++v) ld = std::max(ld, P.deg[v] + 1);
  std::vector<uint64_t> tab((size_t)np * nv * ld, 0);
  for (uint32_t q = 0; q < np; ++q)
    for (uint32_t v = 0; v < nv; ++v) {
      uint64_t acc = 1 % P.p;
      for (uint32_t d = 0; d < ld; ++d) {
        tab[((size_t)q * nv + v) * ld + d] = acc;
        acc = zr_mul(P.M, acc, P.probes[(size_t)q * nv + v]);
      }
    }
  uint64_t* d_tab = A.alloc<uint64_t>(tab.size());
  uint64_t* d_box = A.alloc<uint64_t>((size_t)np * E);
  uint64_t* d_val = A.alloc<uint64_t>((size_t)np * E);
  uint64_t* d_part = A.alloc<uint64_t>((size_t)np * E * kPolyEvalBlocks);
  h2d(d_tab, tab.data(), tab.size() * 8, s);
  for (uint32_t q = 0; q < np; ++q) {
    const uint64_t* pt = P.probes.data() + (size_t)q * nv;
    call_box_multi(bb, ctx, P, E, nv, 1, pt, pt + (nv - 1), 1, d_box + (size_t)q * E, s);
    for (uint32_t e = 0; e < E; ++e) {
      uint64_t* res = d_val + (size_t)q * E + e;
      if (U.t)
        check(poly_eval_point(P.M, U.t, nv, U.exps, U.t, U.coef + (size_t)e * U.t, d_tab + (size_t)q * nv * ld, ld,
                              res, d_part + ((size_t)q * E + e) * kPolyEvalBlocks, s));
      else check(fill_u64(res, 0, 1, s));
    }
  }
  std::vector<uint64_t> a((size_t)np * E), b((size_t)np * E);
  check(hipMemcpyAsync(a.data(), d_box, a.size() * 8, hipMemcpyDeviceToHost, s));
  d2h_sync(b.data(), d_val, b.size() * 8, s);
  if (a != b) throw Error(ZR_EPROBE);
}

void reconstruct_multi(const zr_params* params, uint32_t E, const uint32_t* degs, zr_blackbox_fn bb, void* ctx,
                       hipStream_t s, zr_poly* out) {
  if (!params || !degs || !bb || E == 0 || E > kMaxExpr || params->nvars == 0 || params->nvars > 64)
    throw Error(ZR_EINVAL);
  if ((params->last_stage && params->last_stage != params->nvars) || params->first_stage > 1 || params->deg_den)
    throw Error(ZR_EINVAL);
  const uint32_t n = params->nvars;
  // the schedule and the validation see the largest bound of each variable
  std::vector<uint32_t> dmax(n, 0);
  for (uint32_t e = 0; e < E; ++e)
    for (uint32_t v = 0; v < n; ++v) dmax[v] = std::max(dmax[v], degs[(size_t)e * n + v]);
  zr_params pm = *params;
  pm.deg = dmax.data();
  Params P(&pm, false);
  zr_counters& C = counters();
  C = zr_counters{};
  DevArena keep(s);
  std::vector<std::unique_ptr<DevArena>> arenas;
  int32_t* d_status = keep.alloc<int32_t>(1);
  check(fill_i32(d_status, 0, 1, s));
  std::vector<std::unique_ptr<StageConsts>> K(E);
  for (uint32_t e = 0; e < E; ++e) {
    std::vector<uint32_t> D1s(n);
    for (uint32_t v = 0; v < n; ++v) D1s[v] = degs[(size_t)e * n + v] + 1;
    K[e].reset(new StageConsts(P, keep, D1s, s));
  }
  std::vector<uint32_t> D1max(n);
  for (uint32_t v = 0; v < n; ++v) D1max[v] = dmax[v] + 1;
  StageConsts Kmax(P, keep, D1max, s);
  auto D1_of = [&](uint32_t kvar) {
    std::vector<uint32_t> d(E);
    for (uint32_t e = 0; e < E; ++e) d[e] = degs[(size_t)e * n + kvar] + 1;
    return d;
  };
  // stage 1: the one-term root skeleton, Newton in x_1 per expression
  Union root;
  root.t = 1;
  root.exps = keep.alloc<uint16_t>(n);
  root.mono = keep.alloc<uint64_t>(1);
  check(fill_u64((uint64_t*)root.exps, 0, (n * 2 + 7) / 8, s));
  check(fill_u64(root.mono, 1 % P.p, 1, s));
  Union cur;
  {
    const std::vector<uint32_t> D1 = D1_of(0);
    const std::vector<uint64_t> X = P.node_list(0, D1max[0]);
    DevArena A(s);
    uint64_t* box = A.alloc<uint64_t>((size_t)E * D1max[0]);
    call_box_multi(bb, ctx, P, E, 1, 1, P.y.data(), X.data(), D1max[0], box, s);
    std::vector<uint64_t*> vals(E);
    for (uint32_t e = 0; e < E; ++e) vals[e] = box + (size_t)e * D1max[0];  // first D1[e] samples of expression e
    DevArena* kp = new DevArena(s);
    arenas.emplace_back(kp);
    cur = lift_multi(P, 0, root, vals, D1, K, Kmax, *kp, s, d_status);
  }
  C.stages = 1;
  for (uint32_t k = 2; k <= n; ++k) {
    const uint32_t kvar = k - 1, t = cur.t, Dm = dmax[kvar];
    const std::vector<uint32_t> D1 = D1_of(kvar);
    const std::vector<uint64_t> X = P.node_list(kvar, D1max[kvar]);
    uint32_t R = 0;
    for (uint32_t e = 0; e < E; ++e) R += D1[e] - 1;
    DevArena* kp = new DevArena(s);
    arenas.emplace_back(kp);
    {
      DevArena A(s);
      const size_t tt = std::max<uint32_t>(t, 1);
      // samples of every expression at the Dm nodes beyond the anchor: [E][Dm][t]
      uint64_t* box = A.alloc<uint64_t>((size_t)E * std::max<uint32_t>(Dm, 1) * tt);
      call_box_multi(bb, ctx, P, E, k, t, P.y.data(), X.data() + 1, Dm, box, s);
      // right-hand sides: expression e's first D_e node rows, packed [R][t]
      uint64_t* rhs = A.alloc<uint64_t>((size_t)std::max<uint32_t>(R, 1) * tt);
      uint32_t r0 = 0;
      for (uint32_t e = 0; e < E; ++e) {
        if (D1[e] > 1 && t)
          check(hipMemcpyAsync(rhs + (size_t)r0 * t, box + (size_t)e * Dm * t, (size_t)(D1[e] - 1) * t * 8,
                               hipMemcpyDeviceToDevice, s));
        r0 += D1[e] - 1;
      }
      solve_groups(P, cur, rhs, R, s, d_status);
      // per expression [D1_e][t]: the previous coefficients, then its solved rows
      std::vector<uint64_t*> vals(E);
      r0 = 0;
      for (uint32_t e = 0; e < E; ++e) {
        vals[e] = A.alloc<uint64_t>((size_t)D1[e] * tt);
        if (t) {
          check(copy_u64(vals[e], cur.coef + (size_t)e * t, t, s));
          if (D1[e] > 1)
            check(hipMemcpyAsync(vals[e] + t, rhs + (size_t)r0 * t, (size_t)(D1[e] - 1) * t * 8,
                                 hipMemcpyDeviceToDevice, s));
        }
        r0 += D1[e] - 1;
      }
      cur = lift_multi(P, kvar, cur, vals, D1, K, Kmax, *kp, s, d_status);
    }
    arenas.erase(arenas.begin());
    C.stages = k;
  }
  if (P.nprobes) check_probes_multi(P, E, bb, ctx, cur, s);
  // results: each expression's nonzero terms of the union, in its order
  const uint32_t t = cur.t;
  std::vector<uint16_t> ex((size_t)n * t);
  std::vector<uint64_t> co((size_t)E * t);
  if (t) {
    check(hipMemcpyAsync(ex.data(), cur.exps, ex.size() * 2, hipMemcpyDeviceToHost, s));
    check(hipMemcpyAsync(co.data(), cur.coef, co.size() * 8, hipMemcpyDeviceToHost, s));
  }
  check(hipStreamSynchronize(s));
  for (uint32_t e = 0; e < E; ++e) {
    uint32_t cnt = 0;
    for (uint32_t l = 0; l < t; ++l) cnt += co[(size_t)e * t + l] != 0;
    zr_poly& o = out[e];
    o.nvars = n;
    o.nterms = cnt;
    o.exps = (uint16_t*)malloc(sizeof(uint16_t) * std::max<size_t>((size_t)cnt * n, 1));
    o.coeffs = (uint64_t*)malloc(sizeof(uint64_t) * std::max<uint32_t>(cnt, 1));
    if (!o.exps || !o.coeffs) throw Error(ZR_ENOMEM);
    uint32_t j = 0;
    for (uint32_t l = 0; l < t; ++l) {
      const uint64_t c = co[(size_t)e * t + l];
      if (!c) continue;
      for (uint32_t v = 0; v < n; ++v) o.exps[(size_t)j * n + v] = ex[(size_t)v * t + l];
      o.coeffs[j++] = c;
    }
  }
}

}  // namespace
}  // namespace zr

using namespace zr;

extern "C" zr_status zippel_reconstruct_multi(const zr_params* params, uint32_t nexpr, const uint32_t* deg,
                                              zr_blackbox_fn bb, void* ctx, hipStream_t stream, zr_poly* out) {
  if (!out || nexpr == 0 || nexpr > kMaxExpr) return ZR_EINVAL;
  for (uint32_t e = 0; e < nexpr; ++e) out[e] = zr_poly{};
  try {
    reconstruct_multi(params, nexpr, deg, bb, ctx, stream, out);
    return ZR_OK;
  } catch (const Error& e) {
    for (uint32_t i = 0; i < nexpr; ++i) zr_poly_free(&out[i]);
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    for (uint32_t i = 0; i < nexpr; ++i) zr_poly_free(&out[i]);
    return ZR_ENOMEM;
  } catch (...) {
    for (uint32_t i = 0; i < nexpr; ++i) zr_poly_free(&out[i]);
    return ZR_EDEVICE;
  }
}
