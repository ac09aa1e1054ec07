// Kernels of the multi-prime step (§1: the reconstruction modulo large primes
// ends with the recovery of rational numbers; §2.2: the multi-prime Zippel
// routine).  With the term set fixed by the first prime, each further prime
// needs the coefficients of t known monomials: one transposed Vandermonde
// system with a single right-hand side, solved here in its correlation form,
//   a_l = W(m_l) / (m_l M'(m_l)),   W(z) = sum_d w_d z^d,
//   w_d = sum_{r=0}^{t-1-d} M_{r+d+1} v_{r+1}   (M_t = 1),
// which is sum_r q_{l,r} v_{r+1} regrouped by powers of m_l (q_l = M/(z - m_l)).
// The residues of every term over the primes used so far are then combined by
// the Chinese remainder theorem (Garner's mixed radix) and turned into a
// fraction by Wang's rational reconstruction, one lane per term, in exact
// multiword integers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"
#include "kernels_dev.hpp"
#include "multiprime.hpp"

namespace zr {

// ---- correlation ---------------------------------------------------------------

// Steps of the correlation per LDS window.
constexpr uint32_t kCorrWin = 256;

// Part c of w_d for the 64 values d of block db: the terms r of chunk c,
// [c LC, min((c+1) LC, t - d)), as an exact six-column sum reduced once.  The
// lane-varying M_{r+d+1} comes from an LDS window of kCorrWin + 64
// coefficients (zero beyond M_t = 1, which also ends each lane's sum); the
// uniform v_{r+1} is read through the scalar cache.
__global__ void __launch_bounds__(64) k_mp_corr(zr_mod M, uint32_t t, uint32_t LC, const uint64_t* __restrict__ Mc,
                                                const uint64_t* __restrict__ v, uint64_t* __restrict__ part) {
  __shared__ uint64_t win[kCorrWin + 64];
  const uint32_t lane = threadIdx.x, d0 = blockIdx.x * 64, c = blockIdx.y;
  const uint32_t r0 = c * LC;
  if (r0 + d0 >= t) return;  // no lane of the block has a term in this chunk (uniform)
  const uint32_t r1 = std::min<uint32_t>(r0 + LC, t - d0);
  const_as<uint64_t> V = (const_as<uint64_t>)v;
  Acc6 acc;
  acc6_zero(acc);
  uint32_t since = 0;
  for (uint32_t rb = r0; rb < r1; rb += kCorrWin) {
    // window: M_s for s = rb + d0 + 1 + k, k < kCorrWin + 64
    for (uint32_t k = lane; k < kCorrWin + 64; k += 64) {
      const uint64_t s = (uint64_t)rb + d0 + 1 + k;
      win[k] = s < t ? Mc[s] : (s == t ? 1 : 0);
    }
    __syncthreads();
    const uint32_t re = std::min<uint32_t>(rb + kCorrWin, r1);
    for (uint32_t r = rb; r < re; ++r) {
      const uint64_t m = win[r - rb + lane];
      const uint64_t x = V[r];  // v_{r+1}
      acc6_mac(acc, (uint32_t)m, (uint32_t)(m >> 32), (uint32_t)(x & 0x3FFFFF), (uint32_t)((x >> 22) & 0x3FFFFF),
               (uint32_t)(x >> 44));
      if (++since == kFold) {
        acc6_fold(acc, M);
        since = 0;
      }
    }
    __syncthreads();
  }
  const uint32_t d = d0 + lane;
  if (d < t) part[(size_t)c * t + d] = acc6_reduce(M, acc);
}

// w_d = sum over the chunks that hold terms of d.
__global__ void k_mp_corr_sum(zr_mod M, uint32_t t, uint32_t LC, const uint64_t* __restrict__ part,
                              uint64_t* __restrict__ w) {
  const uint32_t d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= t) return;
  const uint32_t nc = cdiv(t - d, LC);
  uint64_t s = 0;
  for (uint32_t c = 0; c < nc; ++c) s = zr_add(M, s, part[(size_t)c * t + d]);
  w[d] = s;
}

// Coefficients of M'(z) = sum_r (r+1) M_{r+1} z^r (M_t = 1) and the Shoup
// constants of the monomial values.
__global__ void k_mp_prep(zr_mod M, uint32_t t, const uint64_t* __restrict__ Mc, const uint64_t* __restrict__ mono,
                          uint64_t* __restrict__ dM, uint64_t* __restrict__ mono_p) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= t) return;
  const uint64_t top = r + 1 < t ? Mc[r + 1] : 1;
  dM[r] = zr_mul(M, (r + 1) % M.p, top);
  mono_p[r] = zr_shoup_pre(M, mono[r]);
}

// Chunk values of a polynomial with t coefficients a.Mc at every m_l (the
// chunk-chain body of the solve: baby steps and giant steps, exact block sums).
__global__ void __launch_bounds__(256) k_mp_eval(VsArgs a) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < a.t) vs_chain_body(a, l, blockIdx.y);
}

// P(m) = sum_c m^{lo_c} B_c from the chunk values, by Horner from the top chunk.
__device__ __forceinline__ uint64_t combine_chunks(const zr_mod& M, uint32_t t, uint32_t L, uint32_t S, uint64_t m,
                                                   const uint64_t* __restrict__ B, uint32_t l) {
  uint64_t acc = B[l];
  if (S > 1) {
    const uint64_t mL = zr_pow(M, m, L), mLp = zr_shoup_pre(M, mL);
    const uint64_t mlast = zr_pow(M, m, t - (S - 1) * L);
    for (uint32_t c = 1; c < S; ++c) {
      const uint64_t bc = B[(size_t)c * t + l];
      acc = (c + 1 < S) ? zr_add(M, zr_shoup(M, acc, mL, mLp), bc) : zr_add(M, zr_mul(M, acc, mlast), bc);
    }
  }
  return acc;
}

// a_l = W(m_l) / (m_l M'(m_l)); the block's inverses by one inversion.
__global__ void __launch_bounds__(kDeltaBlock) k_mp_finish(zr_mod M, uint32_t t, uint32_t L, uint32_t S,
                                                          const uint64_t* __restrict__ mono,
                                                          const uint64_t* __restrict__ BW,
                                                          const uint64_t* __restrict__ BD, uint64_t* __restrict__ out,
                                                          int32_t* __restrict__ status) {
  __shared__ uint64_t sh[kDeltaBlock / 64 + 1];
  const uint32_t l = blockIdx.x * kDeltaBlock + threadIdx.x;
  const bool live = l < t;
  uint64_t W = 0, w = 0;
  if (live) {
    const uint64_t m = mono[l];
    W = combine_chunks(M, t, L, S, m, BW, l);
    w = zr_mul(M, m, combine_chunks(M, t, L, S, m, BD, l));
    if (w == 0) atomicCAS(status, 0, -3);  // ZR_ESINGULAR
  }
  const uint64_t wi = block_inverse(M, w, live, sh);
  if (live) out[l] = zr_mul(M, W, wi);
}

// ---- multiword integers (little-endian 64-bit words, kMpWords of them) ----------

constexpr int NW = kMpWords;

__device__ __forceinline__ uint32_t mw_bitlen(const uint64_t (&a)[NW]) {
  uint32_t n = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i)
    if (a[i]) n = 64 * i + 64 - __clzll(a[i]);
  return n;
}

__device__ __forceinline__ bool mw_le(const uint64_t (&a)[NW], const uint64_t (&b)[NW]) {  // a <= b
  bool le = true;  // decided by the most significant differing word
#pragma unroll
  for (int i = 0; i < NW; ++i)
    if (a[i] != b[i]) le = a[i] < b[i];
  return le;
}

__device__ __forceinline__ void mw_sub(uint64_t (&a)[NW], const uint64_t (&b)[NW]) {  // a -= b, a >= b
  uint64_t borrow = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint64_t x = a[i], y = b[i];
    const uint64_t d = x - y - borrow;
    borrow = (x < y) || (x - y < borrow) ? 1 : 0;
    a[i] = d;
  }
}

__device__ __forceinline__ void mw_add(uint64_t (&a)[NW], const uint64_t (&b)[NW]) {  // a += b (no overflow)
  uint64_t carry = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint64_t s = a[i] + b[i];
    const uint64_t c1 = s < a[i] ? 1 : 0;
    const uint64_t s2 = s + carry;
    carry = c1 | (s2 < s ? 1 : 0);
    a[i] = s2;
  }
}

__device__ __forceinline__ void mw_shr1(uint64_t (&a)[NW]) {
#pragma unroll
  for (int i = 0; i < NW; ++i) a[i] = (a[i] >> 1) | (i + 1 < NW ? a[i + 1] << 63 : 0);
}

// out = a << s (the bits shifted out of the top word are zero by the caller's sizes)
__device__ __forceinline__ void mw_shl(const uint64_t (&a)[NW], uint32_t s, uint64_t (&out)[NW]) {
#pragma unroll
  for (int i = 0; i < NW; ++i) out[i] = a[i];
  for (uint32_t k = 0; k < s / 64; ++k) {
#pragma unroll
    for (int i = NW - 1; i >= 0; --i) out[i] = i > 0 ? out[i - 1] : 0;
  }
  const uint32_t b = s % 64;
  if (b) {
#pragma unroll
    for (int i = NW - 1; i >= 0; --i) out[i] = (out[i] << b) | (i > 0 ? out[i - 1] >> (64 - b) : 0);
  }
}

__device__ __forceinline__ bool mw_is_zero(const uint64_t (&a)[NW]) {
  uint64_t o = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) o |= a[i];
  return o == 0;
}

__device__ __forceinline__ bool mw_is_one(const uint64_t (&a)[NW]) {
  uint64_t o = a[0] ^ 1;
#pragma unroll
  for (int i = 1; i < NW; ++i) o |= a[i];
  return o == 0;
}

// gcd(a, b) == 1 by the binary gcd (Stein); a, b copied.
__device__ __forceinline__ bool mw_coprime(uint64_t (&u)[NW], uint64_t (&v)[NW]) {
  if (mw_is_zero(u)) return mw_is_one(v);
  if (mw_is_zero(v)) return mw_is_one(u);
  if (!(u[0] & 1) && !(v[0] & 1)) return false;
  while (!(u[0] & 1)) mw_shr1(u);
  for (;;) {
    while (!(v[0] & 1)) mw_shr1(v);
    if (!mw_le(u, v)) {
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const uint64_t x = u[i];
        u[i] = v[i];
        v[i] = x;
      }
    }
    mw_sub(v, u);
    if (mw_is_zero(v)) break;
  }
  return mw_is_one(u);
}

// Garner's mixed radix, the binary value X < P, then Wang's reconstruction by
// the extended Euclidean algorithm on (P, X) (quotients by binary long
// division, cofactor magnitudes |t_{i+1}| = |t_{i-1}| + q_i |t_i|, signs
// alternating from t_1 = +1) until the remainder drops below 2^e.
__global__ void __launch_bounds__(64) k_mp_crt_rr(MpConsts C, uint32_t t, const uint64_t* __restrict__ res,
                                                  uint64_t* __restrict__ num, uint64_t* __restrict__ den,
                                                  uint32_t* __restrict__ neg, uint32_t* __restrict__ fails) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t) return;
  // mixed-radix digits
  uint64_t dg[NW];
#pragma unroll
  for (int j = 0; j < NW; ++j) dg[j] = 0;
  dg[0] = res[l];
#pragma unroll
  for (int j = 1; j < NW; ++j) {
    if (j < (int)C.J) {
      const zr_mod& Mj = C.mod[j];
      uint64_t x = zr_red2p(Mj, dg[j - 1]);
#pragma unroll
      for (int i = NW - 2; i >= 0; --i)
        if (i <= j - 2) x = zr_add(Mj, zr_mul(Mj, x, C.pmod[j][i]), zr_red2p(Mj, dg[i]));
      const uint64_t rj = res[(size_t)j * t + l];
      dg[j] = zr_mul(Mj, zr_sub(Mj, rj, x), C.cinv[j]);
    }
  }
  // X = d_0 + p_0 (d_1 + p_1 (d_2 + ...))
  uint64_t X[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) X[i] = 0;
#pragma unroll
  for (int j = NW - 1; j >= 0; --j) {
    if (j < (int)C.J) {
      if (j < (int)C.J - 1) {
        // X = X * p_j (X < prod_{i>j} p_i, so the product fits)
        uint64_t carry = 0;
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          const zr_u128 pr = (zr_u128)X[i] * C.mod[j].p + carry;
          X[i] = (uint64_t)pr;
          carry = (uint64_t)(pr >> 64);
        }
      }
      // X += d_j
      uint64_t c = dg[j];
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const uint64_t s = X[i] + c;
        c = s < c ? 1 : 0;
        X[i] = s;
      }
    }
  }
  // extended Euclid on (P, X)
  uint64_t r0[NW], r1[NW], T0[NW], T1[NW], D[NW], E[NW];
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    r0[i] = C.P[i];
    r1[i] = X[i];
    T0[i] = 0;
    T1[i] = i == 0 ? 1 : 0;
  }
  bool negative = false;  // sign of the cofactor of r1
  while (mw_bitlen(r1) > C.e) {
    const uint32_t sh = mw_bitlen(r0) - mw_bitlen(r1);
    mw_shl(r1, sh, D);
    mw_shl(T1, sh, E);
    for (uint32_t s = 0; s <= sh; ++s) {
      if (mw_le(D, r0)) {
        mw_sub(r0, D);
        mw_add(T0, E);
      }
      mw_shr1(D);
      mw_shr1(E);
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      uint64_t x = r0[i];
      r0[i] = r1[i];
      r1[i] = x;
      x = T0[i];
      T0[i] = T1[i];
      T1[i] = x;
    }
    negative = !negative;
  }
  bool ok = mw_bitlen(T1) <= C.e && !mw_is_zero(T1);
  if (ok) {
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      D[i] = r1[i];
      E[i] = T1[i];
    }
    ok = mw_coprime(D, E);
  }
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    if (i < (int)C.nw) {
      num[(size_t)i * t + l] = r1[i];
      den[(size_t)i * t + l] = T1[i];
    }
  }
  neg[l] = negative && !mw_is_zero(r1) ? 1 : 0;
  if (!ok) atomicAdd(fails, 1u);
}

// Count the terms whose fraction num/den does not reduce to res modulo p
// (or whose reconstruction failed, marked by den = 0 modulo p included).
__global__ void k_mp_check(zr_mod M, uint32_t t, uint32_t nw, const uint64_t* __restrict__ num,
                           const uint64_t* __restrict__ den, const uint32_t* __restrict__ neg,
                           const uint64_t* __restrict__ res, uint32_t* __restrict__ mismatches) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t) return;
  uint64_t a = 0, b = 0;
  for (uint32_t i = nw; i-- > 0;) {
    a = zr_mod128(M, a, num[(size_t)i * t + l]);
    b = zr_mod128(M, b, den[(size_t)i * t + l]);
  }
  if (neg[l]) a = zr_neg(M, a);
  if (b == 0 || a != zr_mul(M, res[l], b)) atomicAdd(mismatches, 1u);
}

// ---- host-side launchers ----------------------------------------------------------

MpSolvePlan mp_solve_plan(uint32_t t) {
  MpSolvePlan P{};
  P.t = t;
  // correlation: at most 32 chunks of at least 1024 terms
  P.LC = std::max<uint32_t>(1024, (uint32_t)(((size_t)cdiv(t, 32) + kCorrWin - 1) / kCorrWin * kCorrWin));
  P.C = std::max<uint32_t>(1, cdiv(t, P.LC));
  // evaluation: enough (row block, chunk) blocks to fill the chip, chunks of >= 64 coefficients
  const uint32_t rows = std::max<uint32_t>(1, cdiv(t, 256));
  uint32_t S = std::max<uint32_t>(1, cdiv(4 * device_cus(), rows));
  S = std::min<uint32_t>(S, std::max<uint32_t>(1, t / 64));
  P.L = std::max<uint32_t>(1, cdiv(t, S));
  P.S = std::max<uint32_t>(1, cdiv(t, P.L));
  return P;
}

size_t mp_solve_words(const MpSolvePlan& P) {
  const size_t t = P.t;
  // w | M' | mono_p | corr parts | B_W | B_D
  return 3 * t + (size_t)P.C * t + 2 * (size_t)P.S * t + 64;
}

hipError_t mp_solve(const zr_mod& M, const MpSolvePlan& P, const uint64_t* mono, const uint64_t* Mc,
                    const uint64_t* vals, uint64_t* out, uint64_t* work, int32_t* status, hipStream_t s) {
  const uint32_t t = P.t;
  if (t == 0) return hipSuccess;
  uint64_t* w = work;
  uint64_t* dM = w + t;
  uint64_t* mono_p = dM + t;
  uint64_t* part = mono_p + t;
  uint64_t* BW = part + (size_t)P.C * t;
  uint64_t* BD = BW + (size_t)P.S * t;
  {
    TimedLaunch tl("mp_corr", s);
    hipLaunchKernelGGL(k_mp_corr, dim3(cdiv(t, 64), P.C), dim3(64), 0, s, M, t, P.LC, Mc, vals, part);
    hipLaunchKernelGGL(k_mp_corr_sum, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, P.LC, part, w);
  }
  hipLaunchKernelGGL(k_mp_prep, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, Mc, mono, dM, mono_p);
  VsArgs a{};
  a.M = M;
  a.t = t;
  a.L = P.L;
  a.S = P.S;
  a.mono = mono;
  a.mono_p = mono_p;
  {
    TimedLaunch tl("mp_eval", s);
    a.Mc = w;
    a.Bc = BW;
    hipLaunchKernelGGL(k_mp_eval, dim3(cdiv(t, 256), P.S), dim3(256), 0, s, a);
    a.Mc = dM;
    a.Bc = BD;
    hipLaunchKernelGGL(k_mp_eval, dim3(cdiv(t, 256), P.S), dim3(256), 0, s, a);
  }
  hipLaunchKernelGGL(k_mp_finish, dim3(cdiv(t, kDeltaBlock)), dim3(kDeltaBlock), 0, s, M, t, P.L, P.S, mono, BW, BD,
                     out, status);
  return hipGetLastError();
}

hipError_t mp_crt_rr(const MpConsts& C, uint32_t t, const uint64_t* res, uint64_t* num, uint64_t* den,
                     uint32_t* neg, uint32_t* fails, hipStream_t s) {
  if (t == 0) return hipSuccess;
  TimedLaunch tl("mp_crt_rr", s);
  hipLaunchKernelGGL(k_mp_crt_rr, dim3(cdiv(t, 64)), dim3(64), 0, s, C, t, res, num, den, neg, fails);
  return hipGetLastError();
}

hipError_t mp_check(const zr_mod& M, uint32_t t, uint32_t nw, const uint64_t* num, const uint64_t* den,
                    const uint32_t* neg, const uint64_t* res, uint32_t* mismatches, hipStream_t s) {
  if (t == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mp_check, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, nw, num, den, neg, res, mismatches);
  return hipGetLastError();
}

}  // namespace zr
