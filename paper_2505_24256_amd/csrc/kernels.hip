// gfx950 kernels of the polynomial Zippel path: master polynomial, the fused
// transposed Vandermonde solve, Newton lift, skeleton expansion, probes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "field.hpp"
#include "kernels.hpp"

namespace zr {

static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// ============================================================================
// Transposed Vandermonde solve.
//
// For row l (one lane per row):   q_{t-1} = 1,  q_{r-1} = M_r + m_l q_r,
//   s^(j) = sum_r q_r v^(j)_{r+1}   (192-bit exact sums, one reduction),
//   delta = sum_r q_r m_l^r = q_l(m_l) (Horner),   a^(j) = s^(j) / (m_l delta).
// The right-hand sides are packed as VT[r][ldv] so that the R values used at
// step r are contiguous and identical for every lane: they are loaded once
// per wave through the scalar cache.  The length-t vector q_l is never stored.
// ============================================================================

VsolvePlan vsolve_plan(uint32_t t, uint32_t R, uint32_t target_waves) {
  VsolvePlan P;
  P.t = t;
  P.R = R;
  const uint32_t kMaxRT = 32;
  P.ntile = R == 0 ? 1 : cdiv(R, kMaxRT);
  uint32_t rt = R == 0 ? 2 : cdiv(R, P.ntile);
  P.RT = (rt + 1) & ~1u;
  P.ldv = P.RT * P.ntile;
  const uint32_t row_waves = std::max<uint32_t>(1, cdiv(t, 64));
  uint32_t S = std::max<uint32_t>(1, cdiv(target_waves, row_waves * P.ntile));
  const uint32_t minL = 48;
  S = std::min<uint32_t>(S, std::max<uint32_t>(1, t / minL));
  S = std::min<uint32_t>(S, 256);
  P.L = std::max<uint32_t>(1, cdiv(t, S));
  P.S = std::max<uint32_t>(1, cdiv(t, P.L));
  return P;
}

// workspace layout: VT [t][ldv] | mono_p [t] | Bc [S][t] | qstart [S][t] | mL [t] |
//                   spart [S][R][t] | hpart [S][t]
size_t vsolve_workspace_words(const VsolvePlan& P) {
  const size_t t = P.t, S = P.S;
  return t * P.ldv + t + 2 * S * t + t + S * (size_t)P.R * t + S * t + 64;
}

struct VsArgs {
  zr_mod M;
  uint32_t t, L, S, R, ldv;
  const uint64_t* mono;
  const uint64_t* mono_p;
  const uint64_t* Mc;
  const uint64_t* VT;
  const uint64_t* qstart;
  uint64_t* Bc;
  uint64_t* spart;
  uint64_t* hpart;
};

__device__ __forceinline__ void chunk_range(uint32_t t, uint32_t L, uint32_t c, uint32_t& lo, uint32_t& hi) {
  hi = t - c * L;
  lo = hi > L ? hi - L : 0;
}

__global__ void k_pack(uint32_t t, uint32_t R, uint32_t ldv, const uint64_t* __restrict__ rhs, size_t ld_rhs,
                       uint64_t* __restrict__ VT, const uint64_t* __restrict__ mono, uint64_t* __restrict__ mono_p,
                       zr_mod M) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)t * ldv;
  if (idx < total) {
    const uint32_t r = (uint32_t)(idx / ldv), j = (uint32_t)(idx % ldv);
    VT[idx] = j < R ? rhs[(size_t)j * ld_rhs + r] : 0;
  }
  if (idx < t) mono_p[idx] = zr_shoup_pre(M, mono[idx]);
}

// Pass 1: chain only, from 0, over chunk c < S-1: B_c = sum_r M_r m^(r-lo).
__global__ void __launch_bounds__(256) k_vs_chain(VsArgs a) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t c = blockIdx.y;
  if (l >= a.t) return;
  uint32_t lo, hi;
  chunk_range(a.t, a.L, c, lo, hi);
  const uint64_t m = a.mono[l], mp = a.mono_p[l];
  uint64_t x = 0;
  for (uint32_t r = hi; r-- > lo;) x = zr_add(a.M, zr_shoup(a.M, x, m, mp), a.Mc[r]);
  a.Bc[(size_t)c * a.t + l] = x;
}

// Per-row scan over chunks: qstart[0] = 1, qstart[c] = m^L qstart[c-1] + B_{c-1}.
__global__ void k_vs_scan(VsArgs a, uint64_t* __restrict__ qstart, uint64_t* __restrict__ mL_out) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.t) return;
  const uint64_t m = a.mono[l];
  const uint64_t mL = zr_pow(a.M, m, a.L), mLp = zr_shoup_pre(a.M, mL);
  mL_out[l] = mL;
  uint64_t q = 1 % a.M.p;
  qstart[l] = q;
  for (uint32_t c = 1; c < a.S; ++c) {
    q = zr_add(a.M, zr_shoup(a.M, q, mL, mLp), a.Bc[(size_t)(c - 1) * a.t + l]);
    qstart[(size_t)c * a.t + l] = q;
  }
}

// Pass 2: chain + Horner + RT right-hand-side dot products over one chunk.
template <int RT>
__global__ void __launch_bounds__(256) k_vs_dots(VsArgs a) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t c = blockIdx.y;
  const uint32_t tile = blockIdx.z;
  if (l >= a.t) return;
  uint32_t lo, hi;
  chunk_range(a.t, a.L, c, lo, hi);
  const zr_mod M = a.M;
  const uint64_t m = a.mono[l], mp = a.mono_p[l];
  uint64_t q = a.qstart ? a.qstart[(size_t)c * a.t + l] : 1 % M.p;
  uint64_t h = 0;
  zr_acc192 acc[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) zr_acc_zero(acc[j]);
  const uint64_t* __restrict__ VT = a.VT + (size_t)tile * RT;
  for (uint32_t r = hi; r-- > lo;) {
    const uint64_t* __restrict__ v = VT + (size_t)r * a.ldv;
#pragma unroll
    for (int j = 0; j < RT; ++j) zr_acc_mac(acc[j], q, v[j]);
    h = zr_add(M, zr_shoup(M, h, m, mp), q);
    q = zr_add(M, zr_shoup(M, q, m, mp), a.Mc[r]);
  }
  const uint32_t j0 = tile * RT;
#pragma unroll
  for (int j = 0; j < RT; ++j)
    if (j0 + j < a.R) a.spart[((size_t)c * a.R + j0 + j) * a.t + l] = zr_acc_reduce(M, acc[j]);
  if (tile == 0) a.hpart[(size_t)c * a.t + l] = h;
}

// Combine chunks: delta by Horner over chunk partials, s by sums, a = s / (m delta).
__global__ void k_vs_finish(VsArgs a, const uint64_t* __restrict__ mLv, uint64_t* __restrict__ out, size_t ld_out,
                            int32_t* __restrict__ status) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.t) return;
  const zr_mod M = a.M;
  const uint64_t m = a.mono[l];
  uint64_t delta = a.hpart[l];
  if (a.S > 1) {
    const uint64_t mL = mLv[l];
    const uint32_t len_last = a.t - (a.S - 1) * a.L;
    const uint64_t mlast = zr_pow(M, m, len_last);
    for (uint32_t c = 1; c < a.S; ++c) {
      const uint64_t w = (c + 1 < a.S) ? mL : mlast;
      delta = zr_add(M, zr_mul(M, delta, w), a.hpart[(size_t)c * a.t + l]);
    }
  }
  const uint64_t w = zr_mul(M, m, delta);
  if (w == 0) {
    atomicExch(status, -3);  // ZR_ESINGULAR
    for (uint32_t j = 0; j < a.R; ++j) out[(size_t)j * ld_out + l] = 0;
    return;
  }
  const uint64_t wi = zr_inv(M, w), wip = zr_shoup_pre(M, wi);
  for (uint32_t j = 0; j < a.R; ++j) {
    uint64_t s = a.spart[(size_t)j * a.t + l];
    for (uint32_t c = 1; c < a.S; ++c) s = zr_add(M, s, a.spart[((size_t)c * a.R + j) * a.t + l]);
    out[(size_t)j * ld_out + l] = zr_shoup(M, s, wi, wip);
  }
}

typedef void (*DotsKernel)(VsArgs);
template <int RT>
static DotsKernel dots_ptr() {
  return k_vs_dots<RT>;
}
static DotsKernel dots_kernel(uint32_t RT) {
  switch (RT) {
    case 2: return dots_ptr<2>();
    case 4: return dots_ptr<4>();
    case 6: return dots_ptr<6>();
    case 8: return dots_ptr<8>();
    case 10: return dots_ptr<10>();
    case 12: return dots_ptr<12>();
    case 14: return dots_ptr<14>();
    case 16: return dots_ptr<16>();
    case 18: return dots_ptr<18>();
    case 20: return dots_ptr<20>();
    case 22: return dots_ptr<22>();
    case 24: return dots_ptr<24>();
    case 26: return dots_ptr<26>();
    case 28: return dots_ptr<28>();
    case 30: return dots_ptr<30>();
    case 32: return dots_ptr<32>();
    default: return nullptr;
  }
}

hipError_t vsolve(const zr_mod& M, const VsolvePlan& P, const uint64_t* mono, const uint64_t* Mc, const uint64_t* rhs,
                  size_t ld_rhs, uint64_t* out, size_t ld_out, uint64_t* work, int32_t* status, hipStream_t s) {
  if (P.t == 0) return hipSuccess;
  const size_t t = P.t, S = P.S;
  uint64_t* VT = work;
  uint64_t* mono_p = VT + t * P.ldv;
  uint64_t* Bc = mono_p + t;
  uint64_t* qstart = Bc + S * t;
  uint64_t* mL = qstart + S * t;
  uint64_t* spart = mL + t;
  uint64_t* hpart = spart + S * (size_t)P.R * t;
  VsArgs a;
  a.M = M;
  a.t = P.t;
  a.L = P.L;
  a.S = P.S;
  a.R = P.R;
  a.ldv = P.ldv;
  a.mono = mono;
  a.mono_p = mono_p;
  a.Mc = Mc;
  a.VT = VT;
  a.qstart = S > 1 ? qstart : nullptr;
  a.Bc = Bc;
  a.spart = spart;
  a.hpart = hpart;
  {
    const size_t total = std::max<size_t>(t * P.ldv, t);
    TimedLaunch tl("vs_pack", s);
    hipLaunchKernelGGL(k_pack, dim3(cdiv(total, 256)), dim3(256), 0, s, P.t, P.R, P.ldv, rhs, ld_rhs, VT, mono,
                       mono_p, M);
  }
  if (S > 1) {
    {
      TimedLaunch tl("vs_chain", s);
      hipLaunchKernelGGL(k_vs_chain, dim3(cdiv(t, 256), P.S - 1), dim3(256), 0, s, a);
    }
    {
      TimedLaunch tl("vs_scan", s);
      hipLaunchKernelGGL(k_vs_scan, dim3(cdiv(t, 256)), dim3(256), 0, s, a, qstart, mL);
    }
  }
  DotsKernel kd = dots_kernel(P.RT);
  if (!kd) return hipErrorInvalidValue;
  {
    TimedLaunch tl("vs_dots", s);
    hipLaunchKernelGGL(kd, dim3(cdiv(t, 64), P.S, P.ntile), dim3(64), 0, s, a);
  }
  {
    TimedLaunch tl("vs_finish", s);
    hipLaunchKernelGGL(k_vs_finish, dim3(cdiv(t, 256)), dim3(256), 0, s, a, mL, out, ld_out, status);
  }
  return hipGetLastError();
}

// ============================================================================
// Master polynomial by a product tree.  Level s multiplies pairs of monic
// factors of degree <= 2^s; every level stores the non-leading coefficients
// of all its factors in one array of length t (factor [a, b) at [a, b)).
// ============================================================================

__global__ void k_master_leaf(zr_mod M, uint32_t t, const uint64_t* __restrict__ mono, uint64_t* __restrict__ cur) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < t) cur[l] = zr_neg(M, mono[l] % M.p);
}

__global__ void k_master_level(zr_mod M, uint32_t t, uint32_t half, const uint64_t* __restrict__ cur,
                               uint64_t* __restrict__ nxt) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= t) return;
  const uint32_t a = (g / (2 * half)) * (2 * half);
  const uint32_t n1 = std::min(half, t - a);
  const uint32_t n2 = std::min(half, t - a - n1);
  const uint32_t k = g - a;
  const uint64_t* Lc = cur + a;
  const uint64_t* Rc = cur + a + n1;
  zr_acc192 acc;
  zr_acc_zero(acc);
  // sum_{i+j=k} L_i R_j, i in [max(0, k-n2+1), min(k, n1-1)]
  if (n2 > 0) {
    const uint32_t ilo = k + 1 > n2 ? k + 1 - n2 : 0;
    const uint32_t ihi = std::min(k, n1 - 1);
    for (uint32_t i = ilo; i <= ihi; ++i) zr_acc_mac(acc, Lc[i], Rc[k - i]);
  }
  if (k >= n1) zr_acc_mac(acc, 1, Rc[k - n1]);
  if (k >= n2) zr_acc_mac(acc, 1, Lc[k - n2]);
  nxt[g] = zr_acc_reduce(M, acc);
}

hipError_t master_poly(const zr_mod& M, uint32_t t, const uint64_t* mono, uint64_t* Mc, uint64_t* tmp,
                       hipStream_t s) {
  if (t == 0) return hipSuccess;
  TimedLaunch tl("master", s);
  // count levels so that the final level lands in Mc
  uint32_t levels = 0;
  for (uint32_t half = 1; half < t; half *= 2) ++levels;
  uint64_t* bufs[2] = {Mc, tmp};
  uint64_t* cur = bufs[levels % 2];
  hipLaunchKernelGGL(k_master_leaf, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, mono, cur);
  uint32_t lev = 0;
  for (uint32_t half = 1; half < t; half *= 2, ++lev) {
    uint64_t* nxt = bufs[(levels - lev - 1) % 2];
    hipLaunchKernelGGL(k_master_level, dim3(cdiv(t, 128)), dim3(128), 0, s, M, t, half, cur, nxt);
    cur = nxt;
  }
  return hipGetLastError();
}

// ============================================================================
// Newton lift (eq. 1): per term, values at nodes x_0..x_{D} -> divided
// differences -> monomial coefficients.  Node constants are uniform (Shoup
// multipliers shared by all lanes); per-lane arrays live in LDS.
// ============================================================================

constexpr int kNewtonBlock = 64;

__global__ void __launch_bounds__(kNewtonBlock) k_newton(zr_mod M, uint32_t t, uint32_t D1,
                                                         const uint64_t* __restrict__ vals,
                                                         const uint64_t* __restrict__ consts,
                                                         uint64_t* __restrict__ g, uint32_t* __restrict__ cnt) {
  extern __shared__ uint64_t sh[];
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t) return;
  uint64_t* c = sh + threadIdx.x;  // c[i] at c[i * kNewtonBlock]
  const uint64_t* x = consts;
  const uint64_t* xp = consts + D1;
  const uint64_t* invd = consts + 2 * D1;
  const uint64_t* invdp = invd + (size_t)D1 * D1;
  for (uint32_t i = 0; i < D1; ++i) c[i * kNewtonBlock] = vals[(size_t)i * t + l];
  for (uint32_t j = 1; j < D1; ++j)
    for (uint32_t i = D1 - 1; i >= j; --i) {
      const uint64_t d = zr_sub(M, c[i * kNewtonBlock], c[(i - 1) * kNewtonBlock]);
      c[i * kNewtonBlock] = zr_shoup(M, d, invd[j * D1 + i], invdp[j * D1 + i]);
    }
  // expand the nested form from the inside; position q holds the coefficient
  // of z^(q-i) of the partial polynomial after step i
  for (uint32_t i = D1 - 1; i-- > 0;)
    for (uint32_t q = i; q + 1 < D1; ++q) {
      const uint64_t u = zr_shoup(M, c[(q + 1) * kNewtonBlock], x[i], xp[i]);
      c[q * kNewtonBlock] = zr_sub(M, c[q * kNewtonBlock], u);
    }
  uint32_t n = 0;
  for (uint32_t i = 0; i < D1; ++i) {
    const uint64_t v = c[i * kNewtonBlock];
    g[(size_t)i * t + l] = v;
    n += v != 0;
  }
  cnt[l] = n;
}

hipError_t newton_lift(const zr_mod& M, uint32_t t, uint32_t D1, const uint64_t* vals, const uint64_t* consts,
                       uint64_t* g, uint32_t* cnt, hipStream_t s) {
  if (t == 0) return hipSuccess;
  TimedLaunch tl("newton", s);
  const size_t shmem = (size_t)D1 * kNewtonBlock * sizeof(uint64_t);
  hipLaunchKernelGGL(k_newton, dim3(cdiv(t, kNewtonBlock)), dim3(kNewtonBlock), shmem, s, M, t, D1, vals, consts, g,
                     cnt);
  return hipGetLastError();
}

// ============================================================================
// Exclusive scan (three launches: block sums, scan of block sums, apply).
// ============================================================================

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;

__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off *= 2) {
    uint32_t add = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  total = sh[kScanThreads - 1];
  uint32_t incl = sh[tid];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(uint32_t n, const uint32_t* __restrict__ cnt,
                                                            uint32_t* __restrict__ sums) {
  __shared__ uint32_t sh[kScanThreads];
  const size_t base = (size_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  uint32_t v = 0;
  for (int e = 0; e < kScanPer; ++e)
    if (base + e < n) v += cnt[base + e];
  uint32_t total;
  block_exclusive_scan(v, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_top(uint32_t nb, uint32_t* __restrict__ sums,
                                                           uint32_t* __restrict__ total_out) {
  __shared__ uint32_t sh[kScanThreads];
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nb; base += kScanThreads) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t v = i < nb ? sums[i] : 0;
    uint32_t total;
    const uint32_t ex = block_exclusive_scan(v, sh, total);
    if (i < nb) sums[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(uint32_t n, const uint32_t* __restrict__ cnt,
                                                             const uint32_t* __restrict__ sums,
                                                             uint32_t* __restrict__ off) {
  __shared__ uint32_t sh[kScanThreads];
  const size_t base = (size_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
  uint32_t loc[kScanPer];
  uint32_t v = 0;
  for (int e = 0; e < kScanPer; ++e) {
    loc[e] = base + e < n ? cnt[base + e] : 0;
    v += loc[e];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan(v, sh, total) + sums[blockIdx.x];
  for (int e = 0; e < kScanPer; ++e) {
    if (base + e < n) off[base + e] = ex;
    ex += loc[e];
  }
}

size_t scan_tmp_words(uint32_t n) { return cdiv(std::max<uint32_t>(n, 1), kScanBlock) + 1; }

hipError_t exclusive_scan(uint32_t n, const uint32_t* cnt, uint32_t* off, uint32_t* tmp, hipStream_t s) {
  TimedLaunch tl("scan", s);
  const uint32_t nb = cdiv(std::max<uint32_t>(n, 1), kScanBlock);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(kScanThreads), 0, s, n, cnt, tmp);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, nb, tmp, off + n);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, n, cnt, tmp, off);
  return hipGetLastError();
}

// ============================================================================
// Skeleton expansion: terms (e_l, d) with nonzero coefficient, lex order kept.
// ============================================================================

__global__ void k_expand(zr_mod M, uint32_t t, uint32_t D1, uint32_t kvar, uint32_t nvars,
                         const uint16_t* __restrict__ exps_old, const uint64_t* __restrict__ mono_old,
                         const uint64_t* __restrict__ g, const uint32_t* __restrict__ off,
                         const uint64_t* __restrict__ ypow, const uint64_t* __restrict__ ypowp,
                         uint16_t* __restrict__ exps_new, uint64_t* __restrict__ coef_new,
                         uint64_t* __restrict__ mono_new, uint32_t ld_new) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t) return;
  uint32_t pos = off[l];
  const uint64_t m = mono_old[l];
  for (uint32_t d = 0; d < D1; ++d) {
    const uint64_t c = g[(size_t)d * t + l];
    if (c == 0) continue;
    for (uint32_t v = 0; v < nvars; ++v)
      exps_new[(size_t)v * ld_new + pos] = v == kvar ? (uint16_t)d : exps_old[(size_t)v * t + l];
    coef_new[pos] = c;
    mono_new[pos] = zr_shoup(M, m, ypow[d], ypowp[d]);
    ++pos;
  }
}

hipError_t expand(const zr_mod& M, uint32_t t, uint32_t D1, uint32_t kvar, uint32_t nvars, const uint16_t* exps_old,
                  const uint64_t* mono_old, const uint64_t* g, const uint32_t* off, const uint64_t* ypow,
                  const uint64_t* ypowp, uint16_t* exps_new, uint64_t* coef_new, uint64_t* mono_new, uint32_t ld_new,
                  hipStream_t s) {
  if (t == 0) return hipSuccess;
  TimedLaunch tl("expand", s);
  hipLaunchKernelGGL(k_expand, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, D1, kvar, nvars, exps_old, mono_old, g, off,
                     ypow, ypowp, exps_new, coef_new, mono_new, ld_new);
  return hipGetLastError();
}

// ============================================================================
// Probe: value of the sparse polynomial at one point (power tables per
// variable; partial sums per thread, wave and block reductions mod p).
// ============================================================================

__global__ void __launch_bounds__(256) k_poly_eval(zr_mod M, uint32_t t, uint32_t nvars,
                                                   const uint16_t* __restrict__ exps, uint32_t ld,
                                                   const uint64_t* __restrict__ coef,
                                                   const uint64_t* __restrict__ tab, uint32_t ldtab,
                                                   uint64_t* __restrict__ result) {
  __shared__ uint64_t sh[256];
  uint64_t acc = 0;
  for (uint32_t l = threadIdx.x; l < t; l += blockDim.x) {
    uint64_t v = coef[l];
    for (uint32_t j = 0; j < nvars; ++j) v = zr_mul(M, v, tab[(size_t)j * ldtab + exps[(size_t)j * ld + l]]);
    acc = zr_add(M, acc, v);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = zr_add(M, sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *result = sh[0];
}

hipError_t poly_eval_point(const zr_mod& M, uint32_t t, uint32_t nvars, const uint16_t* exps, uint32_t ld,
                           const uint64_t* coef, const uint64_t* tab, uint32_t ldtab, uint64_t* result,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_poly_eval, dim3(1), dim3(256), 0, s, M, t, nvars, exps, ld, coef, tab, ldtab, result);
  return hipGetLastError();
}

// ============================================================================
// helpers
// ============================================================================

__global__ void k_fill_u64(uint64_t* p, uint64_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int32_t v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_copy_u64(uint64_t* d, const uint64_t* s, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

hipError_t fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(cdiv(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t copy_u64(uint64_t* d, const uint64_t* src, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_u64, dim3(cdiv(n, 256)), dim3(256), 0, s, d, src, n);
  return hipGetLastError();
}

// ============================================================================
// kernel timing
// ============================================================================

struct TimingState {
  std::mutex mu;
  bool on = false;
  struct Pending {
    std::string name;
    hipEvent_t e0, e1;
  };
  std::vector<Pending> pending;
  std::unordered_map<std::string, std::pair<uint64_t, double>> totals;
  void resolve() {
    for (auto& p : pending) {
      (void)hipEventSynchronize(p.e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, p.e0, p.e1);
      auto& e = totals[p.name];
      e.first += 1;
      e.second += ms;
      (void)hipEventDestroy(p.e0);
      (void)hipEventDestroy(p.e1);
    }
    pending.clear();
  }
};
static TimingState g_timing;

TimedLaunch::TimedLaunch(const char* n, hipStream_t st) : name(n), s(st), e0(nullptr), e1(nullptr), on(false) {
  if (!g_timing.on) return;
  on = true;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  (void)hipEventRecord(e0, s);
}

TimedLaunch::~TimedLaunch() {
  if (!on) return;
  (void)hipEventRecord(e1, s);
  std::lock_guard<std::mutex> g(g_timing.mu);
  g_timing.pending.push_back({name, e0, e1});
}

}  // namespace zr

extern "C" {
void zr_timing_enable(int on) {
  std::lock_guard<std::mutex> g(zr::g_timing.mu);
  zr::g_timing.on = on != 0;
}
void zr_timing_reset(void) {
  std::lock_guard<std::mutex> g(zr::g_timing.mu);
  zr::g_timing.resolve();
  zr::g_timing.totals.clear();
}
uint64_t zr_timing_get(const char* kernel, double* total_ms) {
  std::lock_guard<std::mutex> g(zr::g_timing.mu);
  zr::g_timing.resolve();
  auto it = zr::g_timing.totals.find(kernel);
  if (it == zr::g_timing.totals.end()) {
    if (total_ms) *total_ms = 0;
    return 0;
  }
  if (total_ms) *total_ms = it->second.second;
  return it->second.first;
}
}
