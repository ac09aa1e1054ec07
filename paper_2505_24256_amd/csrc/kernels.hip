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

// Right-hand sides per tile: nine accumulator registers each, so that a tile
// of 20 still leaves room for the chain state within 256 VGPRs.
constexpr uint32_t kMaxRT = 20;

static uint32_t dots_waves_per_cu(uint32_t RT);

// Chunking: enough (row block, chunk, tile) waves for about four rounds of the
// device's resident wave slots, so the tail of the launch stays short, with
// chunks of at least 128 steps.
VsolvePlan vsolve_plan(uint32_t t, uint32_t R, uint32_t num_cus) {
  VsolvePlan P;
  P.t = t;
  P.R = R;
  P.ntile = R == 0 ? 1 : cdiv(R, kMaxRT);
  P.RT = R == 0 ? 1 : cdiv(R, P.ntile);
  P.ldv = (3 * P.RT + 2 + 15) & ~15u;  // 32-bit words per packed row: 3 limbs per value + M_r, 64-byte groups
  const uint32_t slots = std::max<uint32_t>(1, num_cus) * dots_waves_per_cu(P.RT);
  const uint32_t row_blocks = std::max<uint32_t>(1, cdiv(t, 64));
  uint32_t S = std::max<uint32_t>(1, cdiv(4ull * slots, (uint64_t)row_blocks * P.ntile));
  S = std::min<uint32_t>(S, std::max<uint32_t>(1, t / 128));
  S = std::min<uint32_t>(S, 256);
  P.L = std::max<uint32_t>(1, cdiv(t, S));
  P.S = std::max<uint32_t>(1, cdiv(t, P.L));
  return P;
}

// workspace layout (64-bit words): VT [ntile][t][ldv/2] | mono_p [t] | Bc [S][t] |
//                   qstart [S][t] | mL [t] | spart [S][R][t] | hpart [S][t] | winv [2t]
size_t vsolve_workspace_words(const VsolvePlan& P) {
  const size_t t = P.t, S = P.S;
  return P.ntile * t * (P.ldv / 2) + t + 2 * S * t + t + S * (size_t)P.R * t + S * t + 2 * t + 64;
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

// Packed row r of tile `tile` (32-bit words): for jj < RT the value
// v = v^(tile*RT + jj)_{r+1} as three limbs v & (2^22-1), (v >> 22) & (2^22-1),
// v >> 44 at words 3jj..3jj+2; M_r at words 3RT, 3RT+1; zero padding.
__global__ void k_pack(uint32_t t, uint32_t R, uint32_t RT, uint32_t ntile, uint32_t ldv,
                       const uint64_t* __restrict__ rhs, size_t ld_rhs, const uint64_t* __restrict__ Mc,
                       uint32_t* __restrict__ VT, const uint64_t* __restrict__ mono, uint64_t* __restrict__ mono_p,
                       zr_mod M) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)ntile * t * ldv;
  if (idx < total) {
    const uint32_t w = (uint32_t)(idx % ldv);
    const size_t rest = idx / ldv;
    const uint32_t r = (uint32_t)(rest % t), tile = (uint32_t)(rest / t);
    uint32_t out = 0;
    if (w < 3 * RT) {
      const uint32_t jj = w / 3, limb = w % 3;
      const uint32_t j = tile * RT + jj;
      const uint64_t v = j < R ? rhs[(size_t)j * ld_rhs + r] : 0;
      out = (uint32_t)((v >> (22 * limb)) & (limb < 2 ? 0x3FFFFFu : 0xFFFFFFFFu));
    } else if (w == 3 * RT) {
      out = (uint32_t)Mc[r];
    } else if (w == 3 * RT + 1) {
      out = (uint32_t)(Mc[r] >> 32);
    }
    VT[idx] = out;
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

// Exact sum of 64x64-bit products in column form.  With q = q0 + q1 2^32 and
// v = v0 + v1 2^32 (32-bit halves),
//     q v = q0 v0 + (q0 v1 + q1 v0) 2^32 + q1 v1 2^64,
// and each column is accumulated in 64 bits by v_mad_u64_u32 (32x32 product
// plus 64-bit addend, carry out); the carries are counted in 32-bit registers.
// The represented value is  A + B 2^32 + (C + KA) 2^64 + KB 2^96 + KC 2^128,
// exact for up to 2^32 terms: 4 multiplies and 4 carry additions per term,
// nine registers per right-hand side, one reduction mod p at the end.
struct ColAcc {
  uint64_t A, B, C;
  uint32_t KA, KB, KC;
};

__device__ __forceinline__ void col_zero(ColAcc& a) {
  a.A = 0;
  a.B = 0;
  a.C = 0;
  a.KA = 0;
  a.KB = 0;
  a.KC = 0;
}

// The four products write distinct carry registers; each carry is consumed
// three instructions after it is produced.  v0, v1 are wave-uniform (SGPR).
__device__ __forceinline__ void col_mac(ColAcc& a, uint32_t q0, uint32_t q1, uint32_t v0, uint32_t v1) {
  uint64_t c0, c1, c2, c3, d;
  asm("v_mad_u64_u32 %[A], %[c0], %[q0], %[v0], %[A]\n\t"
      "v_mad_u64_u32 %[B], %[c1], %[q0], %[v1], %[B]\n\t"
      "v_mad_u64_u32 %[C], %[c3], %[q1], %[v1], %[C]\n\t"
      "v_mad_u64_u32 %[B], %[c2], %[q1], %[v0], %[B]\n\t"
      "v_addc_co_u32_e64 %[KA], %[d], 0, %[KA], %[c0]\n\t"
      "v_addc_co_u32_e64 %[KB], %[d], 0, %[KB], %[c1]\n\t"
      "v_addc_co_u32_e64 %[KC], %[d], 0, %[KC], %[c3]\n\t"
      "v_addc_co_u32_e64 %[KB], %[d], 0, %[KB], %[c2]"
      : [A] "+v"(a.A), [B] "+v"(a.B), [C] "+v"(a.C), [KA] "+v"(a.KA), [KB] "+v"(a.KB), [KC] "+v"(a.KC),
        [c0] "=&s"(c0), [c1] "=&s"(c1), [c2] "=&s"(c2), [c3] "=&s"(c3), [d] "=&s"(d)
      : [q0] "v"(q0), [q1] "v"(q1), [v0] "s"(v0), [v1] "s"(v1));
}

__device__ __forceinline__ uint64_t col_reduce(const zr_mod& M, const ColAcc& a) {
  uint64_t w0 = a.A, w1, w2 = 0;
  const uint64_t bl = a.B << 32, bh = a.B >> 32;
  w0 += bl;
  w1 = bh + (w0 < bl);
  w1 += a.C;
  w2 += w1 < a.C;
  w1 += a.KA;
  w2 += w1 < (uint64_t)a.KA;
  const uint64_t kb = (uint64_t)a.KB << 32;
  w1 += kb;
  w2 += w1 < kb;
  w2 += a.KC;
  uint64_t r = zr_mod128(M, 0, w2);
  r = zr_mod128(M, r, w1);
  return zr_mod128(M, r, w0);
}

// Carry-free exact dot products.  q = q0 + q1 2^32 (32-bit halves, per lane)
// and v = v0 + v1 2^22 + v2 2^44 (22-bit limbs, packed once per system), so
//   q v = q0 v0 + q0 v1 2^22 + q1 v0 2^32 + q0 v2 2^44 + q1 v1 2^54 + q1 v2 2^76,
// six 32x32 products below 2^54, each summed by one v_mad_u64_u32 into its own
// 64-bit column.  A column absorbs 1024 such products; every kFold steps the
// bits above each column's range are moved into the column of matching weight
// (exact shifts and adds), so chunks of any length stay exact.
struct Acc6 {
  uint64_t w0, w22, w32, w44, w54, w76;
};
constexpr uint32_t kFold = 512;

__device__ __forceinline__ void acc6_zero(Acc6& a) {
  a.w0 = a.w22 = a.w32 = a.w44 = a.w54 = a.w76 = 0;
}

__device__ __forceinline__ void acc6_mac(Acc6& a, uint32_t q0, uint32_t q1, uint32_t v0, uint32_t v1, uint32_t v2) {
  a.w0 += (uint64_t)q0 * v0;
  a.w22 += (uint64_t)q0 * v1;
  a.w44 += (uint64_t)q0 * v2;
  a.w32 += (uint64_t)q1 * v0;
  a.w54 += (uint64_t)q1 * v1;
  a.w76 += (uint64_t)q1 * v2;
}

// Move everything above bit 54 of each weight-0..44 column into w54, and
// everything above bit 22 of w54 into w76.
__device__ __forceinline__ void acc6_fold(Acc6& a) {
  a.w54 += (a.w0 >> 54) + (a.w22 >> 32) + (a.w32 >> 22) + (a.w44 >> 10);
  a.w0 &= (1ull << 54) - 1;
  a.w22 &= (1ull << 32) - 1;
  a.w32 &= (1ull << 22) - 1;
  a.w44 &= (1ull << 10) - 1;
  a.w76 += a.w54 >> 22;
  a.w54 &= (1ull << 22) - 1;
}

// add x * 2^s (x < 2^64, s < 128) to the 192-bit (w[0], w[1], w[2])
__device__ __forceinline__ void add_shift192(uint64_t w[3], uint64_t x, uint32_t s) {
  const uint32_t o = s >> 6, b = s & 63;
  const zr_u128 v = ((zr_u128)x) << b;
  const uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
  if (o == 0) {
    zr_u128 t = (zr_u128)w[0] + lo;
    w[0] = (uint64_t)t;
    t = (zr_u128)w[1] + hi + (uint64_t)(t >> 64);
    w[1] = (uint64_t)t;
    w[2] += (uint64_t)(t >> 64);
  } else {
    zr_u128 t = (zr_u128)w[1] + lo;
    w[1] = (uint64_t)t;
    w[2] += hi + (uint64_t)(t >> 64);
  }
}

__device__ __forceinline__ uint64_t acc6_reduce(const zr_mod& M, const Acc6& a) {
  uint64_t w[3] = {0, 0, 0};
  add_shift192(w, a.w0, 0);
  add_shift192(w, a.w22, 22);
  add_shift192(w, a.w32, 32);
  add_shift192(w, a.w44, 44);
  add_shift192(w, a.w54, 54);
  add_shift192(w, a.w76, 76);
  uint64_t r = zr_mod128(M, 0, w[2]);
  r = zr_mod128(M, r, w[1]);
  return zr_mod128(M, r, w[0]);
}

// Pass 2: chain + Horner + RT right-hand-side dot products over one chunk.
// One lane per row.  Packed row r of a tile is identical for all lanes: each
// 64-byte group of it is one scalar load, issued for step r-1 as soon as step
// r has consumed the group, so its latency hides behind the remaining work.
struct alignas(64) VGroup {
  uint32_t w[16];
};

template <int RT>
__global__ void __launch_bounds__(64) k_vs_dots(VsArgs a) {
  constexpr int LDV = (3 * RT + 2 + 15) & ~15;
  constexpr int G = LDV / 16;
  const uint32_t l0 = blockIdx.x * 64 + threadIdx.x;
  const uint32_t c = blockIdx.y;
  const uint32_t tile = blockIdx.z;
  const bool live = l0 < a.t;
  const uint32_t l = live ? l0 : a.t - 1;
  uint32_t lo, hi;
  chunk_range(a.t, a.L, c, lo, hi);
  const zr_mod M = a.M;
  const uint64_t m = a.mono[l], mp = a.mono_p[l];
  uint64_t q = a.qstart ? a.qstart[(size_t)c * a.t + l] : 1 % M.p;
  uint64_t h = 0;
  Acc6 acc[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) acc6_zero(acc[j]);
  const VGroup* __restrict__ rows = (const VGroup*)((const uint32_t*)a.VT + (size_t)tile * a.t * LDV);
  const bool horner = tile == 0;
  uint32_t r = hi - 1;
  uint32_t since = 0;
  VGroup buf[G];
#pragma unroll
  for (int g = 0; g < G; ++g) buf[g] = rows[(size_t)r * G + g];
  for (;;) {
    const uint32_t rn = r > lo ? r - 1 : r;
    const uint32_t q0 = (uint32_t)q, q1 = (uint32_t)(q >> 32);
    uint32_t mlo = 0, mhi = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
      for (int jj = 0; jj < RT; ++jj) {
        if (3 * jj / 16 == g) {
          // the three limbs of value jj may straddle two groups
          const int w0 = 3 * jj, w1 = 3 * jj + 1, w2 = 3 * jj + 2;
          const uint32_t v0 = buf[w0 / 16].w[w0 % 16];
          const uint32_t v1 = buf[w1 / 16].w[w1 % 16];
          const uint32_t v2 = buf[w2 / 16].w[w2 % 16];
          acc6_mac(acc[jj], q0, q1, v0, v1, v2);
        }
      }
      if ((3 * RT) / 16 == g) mlo = buf[g].w[(3 * RT) % 16];
      if ((3 * RT + 1) / 16 == g) mhi = buf[g].w[(3 * RT + 1) % 16];
      // every later read of this step lies in groups > g (a value's limbs
      // only extend forward), so group g can be refilled for step r-1 now
      buf[g] = rows[(size_t)rn * G + g];
    }
    const uint64_t Mr = ((uint64_t)mhi << 32) | mlo;
    if (horner) h = zr_add(M, zr_shoup(M, h, m, mp), q);
    q = zr_add(M, zr_shoup(M, q, m, mp), Mr);
    if (++since == kFold) {
#pragma unroll
      for (int j = 0; j < RT; ++j) acc6_fold(acc[j]);
      since = 0;
    }
    if (r == lo) break;
    r = rn;
  }
  if (!live) return;
  const uint32_t j0 = tile * RT;
#pragma unroll
  for (int j = 0; j < RT; ++j)
    if (j0 + j < a.R) a.spart[((size_t)c * a.R + j0 + j) * a.t + l] = acc6_reduce(M, acc[j]);
  if (horner) a.hpart[(size_t)c * a.t + l] = h;
}

// Combine chunks, part 1 (one lane per row): delta = sum_c m^{lo_c} H_c by
// Horner over the chunk partials, w = m delta, and its inverse (with Shoup
// constant) into winv[2t]; a zero w marks the system singular.
__global__ void k_vs_delta(VsArgs a, const uint64_t* __restrict__ mLv, uint64_t* __restrict__ winv,
                           int32_t* __restrict__ status) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.t) return;
  const zr_mod M = a.M;
  const uint64_t m = a.mono[l];
  uint64_t delta = a.hpart[l];
  if (a.S > 1) {
    const uint64_t mL = mLv[l], mLp = zr_shoup_pre(M, mL);
    const uint32_t len_last = a.t - (a.S - 1) * a.L;
    const uint64_t mlast = zr_pow(M, m, len_last);
    for (uint32_t c = 1; c < a.S; ++c) {
      const uint64_t hc = a.hpart[(size_t)c * a.t + l];
      delta = (c + 1 < a.S) ? zr_add(M, zr_shoup(M, delta, mL, mLp), hc) : zr_add(M, zr_mul(M, delta, mlast), hc);
    }
  }
  const uint64_t w = zr_mul(M, m, delta);
  if (w == 0) {
    atomicExch(status, -3);  // ZR_ESINGULAR
    winv[l] = 0;
    winv[a.t + l] = 0;
    return;
  }
  const uint64_t wi = zr_inv(M, w);
  winv[l] = wi;
  winv[a.t + l] = zr_shoup_pre(M, wi);
}

// Combine chunks, part 2 (one lane per row and right-hand side):
// a^(j)_l = (sum_c s^(j)_{l,c}) / (m_l delta_l).
__global__ void k_vs_scale(VsArgs a, const uint64_t* __restrict__ winv, uint64_t* __restrict__ out, size_t ld_out) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t j = blockIdx.y;
  if (l >= a.t) return;
  const zr_mod M = a.M;
  uint64_t s = 0;
  for (uint32_t c = 0; c < a.S; ++c) s = zr_add(M, s, a.spart[((size_t)c * a.R + j) * a.t + l]);
  out[(size_t)j * ld_out + l] = zr_shoup(M, s, winv[l], winv[a.t + l]);
}

typedef void (*DotsKernel)(VsArgs);
template <int RT>
static DotsKernel dots_ptr() {
  return k_vs_dots<RT>;
}
static DotsKernel dots_kernel(uint32_t RT) {
  static const DotsKernel table[kMaxRT + 1] = {
      nullptr,        dots_ptr<1>(),  dots_ptr<2>(),  dots_ptr<3>(),  dots_ptr<4>(),  dots_ptr<5>(),
      dots_ptr<6>(),  dots_ptr<7>(),  dots_ptr<8>(),  dots_ptr<9>(),  dots_ptr<10>(), dots_ptr<11>(),
      dots_ptr<12>(), dots_ptr<13>(), dots_ptr<14>(), dots_ptr<15>(), dots_ptr<16>(), dots_ptr<17>(),
      dots_ptr<18>(), dots_ptr<19>(), dots_ptr<20>()};
  return RT >= 1 && RT <= kMaxRT ? table[RT] : nullptr;
}

static uint32_t dots_waves_per_cu(uint32_t RT) {
  static int cache[kMaxRT + 1] = {0};
  if (RT < 1 || RT > kMaxRT) return 8;
  if (!cache[RT]) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, dots_kernel(RT), 64, 0) != hipSuccess || nb <= 0) nb = 8;
    cache[RT] = nb;
  }
  return (uint32_t)cache[RT];
}

hipError_t vsolve(const zr_mod& M, const VsolvePlan& P, const uint64_t* mono, const uint64_t* Mc, const uint64_t* rhs,
                  size_t ld_rhs, uint64_t* out, size_t ld_out, uint64_t* work, int32_t* status, hipStream_t s) {
  if (P.t == 0) return hipSuccess;
  const size_t t = P.t, S = P.S;
  uint64_t* VT = work;
  uint64_t* mono_p = VT + P.ntile * t * (P.ldv / 2);
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
    const size_t total = std::max<size_t>(P.ntile * t * P.ldv, t);  // 32-bit words
    TimedLaunch tl("vs_pack", s);
    hipLaunchKernelGGL(k_pack, dim3(cdiv(total, 256)), dim3(256), 0, s, P.t, P.R, P.RT, P.ntile, P.ldv, rhs, ld_rhs,
                       Mc, (uint32_t*)VT, mono, mono_p, M);
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
    uint64_t* winv = hpart + S * t;
    hipLaunchKernelGGL(k_vs_delta, dim3(cdiv(t, 256)), dim3(256), 0, s, a, mL, winv, status);
    hipLaunchKernelGGL(k_vs_scale, dim3(cdiv(t, 256), P.R), dim3(256), 0, s, a, winv, out, ld_out);
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

// Large levels (factors of degree >= 32): a wave owns 64 consecutive output
// coefficients of one product and one chunk [i0, i1) of the convolution index.
// The factor L_i is wave-uniform (scalar load, split into 22-bit limbs); the
// window of R needed by the wave, R_{k-i} for its k and i, is staged once in
// LDS.  Chunk partial sums go to part[ic][g]; k_master_sum adds them and the
// two terms contributed by the leading ones.
constexpr uint32_t kConvIC = 512;

__global__ void __launch_bounds__(64) k_master_conv(zr_mod M, uint32_t t, uint32_t half, uint32_t IC,
                                                    const uint64_t* __restrict__ cur, uint64_t* __restrict__ part) {
  __shared__ uint64_t win[64 + kConvIC];
  const uint32_t g0 = blockIdx.x * 64;
  const uint32_t g = g0 + threadIdx.x;
  const uint32_t ic = blockIdx.y;
  const uint32_t a = (g0 / (2 * half)) * (2 * half);  // one product per wave since 2*half >= 64
  const uint32_t n1 = std::min(half, t - a);
  const uint32_t n2 = std::min(half, t - a - n1);
  const uint32_t k0 = g0 - a;
  const uint32_t k = g - a;
  const uint64_t* __restrict__ Lc = cur + a;
  const uint64_t* __restrict__ Rc = cur + a + n1;
  Acc6 acc;
  acc6_zero(acc);
  uint32_t ilo = ic * IC, ihi = std::min(ilo + IC, n1);
  if (n2 > 0) {
    const uint32_t wlo = k0 + 1 > n2 ? k0 + 1 - n2 : 0;
    const uint32_t whi = std::min(k0 + 64, n1);
    ilo = std::max(ilo, wlo);
    ihi = std::min(ihi, whi);
  } else {
    ihi = ilo;
  }
  if (ilo < ihi) {
    // window: R index j = k - i for k in [k0, k0+63], i in [ilo, ihi): j in [k0 - ihi + 1, k0 + 63 - ilo]
    const int64_t jbase = (int64_t)k0 - (int64_t)ihi + 1;
    const uint32_t wlen = 63 + (ihi - ilo);
    for (uint32_t x = threadIdx.x; x < wlen; x += 64) {
      const int64_t j = jbase + x;
      win[x] = (j >= 0 && j < (int64_t)n2) ? Rc[j] : 0;
    }
    __syncthreads();
    uint32_t since = 0;
    for (uint32_t i = ilo; i < ihi; ++i) {
      const uint64_t Li = Lc[i];
      // lane k reads R_{k-i} at window index k - i - jbase (in range for every lane)
      const uint64_t Rv = win[(int64_t)k - (int64_t)i - jbase];
      acc6_mac(acc, (uint32_t)Rv, (uint32_t)(Rv >> 32), (uint32_t)(Li & 0x3FFFFF), (uint32_t)((Li >> 22) & 0x3FFFFF),
               (uint32_t)(Li >> 44));
      if (++since == kFold) {
        acc6_fold(acc);
        since = 0;
      }
    }
  }
  if (g < t) part[(size_t)ic * t + g] = acc6_reduce(M, acc);
}

__global__ void k_master_sum(zr_mod M, uint32_t t, uint32_t half, uint32_t nic, const uint64_t* __restrict__ cur,
                             const uint64_t* __restrict__ part, uint64_t* __restrict__ nxt) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= t) return;
  const uint32_t a = (g / (2 * half)) * (2 * half);
  const uint32_t n1 = std::min(half, t - a);
  const uint32_t n2 = std::min(half, t - a - n1);
  const uint32_t k = g - a;
  uint64_t s = 0;
  for (uint32_t ic = 0; ic < nic; ++ic) s = zr_add(M, s, part[(size_t)ic * t + g]);
  if (k >= n1) s = zr_add(M, s, cur[a + n1 + (k - n1)]);
  if (k >= n2) s = zr_add(M, s, cur[a + (k - n2)]);
  nxt[g] = s;
}

size_t master_tmp_words(uint32_t t) {
  // t for the ping-pong level array plus chunk partials of the large levels
  uint32_t nic_max = 1;
  for (uint32_t half = 32; half < t; half *= 2) nic_max = std::max(nic_max, cdiv(half, kConvIC));
  return (size_t)t + (size_t)nic_max * t + 64;
}

hipError_t master_poly(const zr_mod& M, uint32_t t, const uint64_t* mono, uint64_t* Mc, uint64_t* tmp,
                       hipStream_t s) {
  if (t == 0) return hipSuccess;
  TimedLaunch tl("master", s);
  // count levels so that the final level lands in Mc
  uint32_t levels = 0;
  for (uint32_t half = 1; half < t; half *= 2) ++levels;
  uint64_t* bufs[2] = {Mc, tmp};
  uint64_t* part = tmp + t;
  uint64_t* cur = bufs[levels % 2];
  hipLaunchKernelGGL(k_master_leaf, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, mono, cur);
  uint32_t lev = 0;
  for (uint32_t half = 1; half < t; half *= 2, ++lev) {
    uint64_t* nxt = bufs[(levels - lev - 1) % 2];
    if (half < 32) {
      hipLaunchKernelGGL(k_master_level, dim3(cdiv(t, 128)), dim3(128), 0, s, M, t, half, cur, nxt);
    } else {
      const uint32_t IC = kConvIC;
      const uint32_t nic = cdiv(half, IC);
      hipLaunchKernelGGL(k_master_conv, dim3(cdiv(t, 64), nic), dim3(64), 0, s, M, t, half, IC, cur, part);
      hipLaunchKernelGGL(k_master_sum, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, half, nic, cur, part, nxt);
    }
    cur = nxt;
  }
  return hipGetLastError();
}

// ============================================================================
// Newton lift (eq. 1).  Interpolating values a_0..a_D at fixed nodes into
// monomial coefficients is linear: g = W a with W the inverse of the
// Vandermonde matrix of the nodes, the same for every term of a stage.  The
// host builds W by running Newton's divided differences and nested expansion
// on unit vectors; here each lane owns one term and DB output coefficients,
// and the products are the carry-free 64x64-bit sums of the solve.
// Wl: [i][d][3] 22-bit limbs of W[d][i].
// ============================================================================

constexpr int kNewtonDB = 8;

__global__ void __launch_bounds__(64) k_newton_mat(zr_mod M, uint32_t t, uint32_t D1,
                                                   const uint64_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ Wl, uint64_t* __restrict__ g) {
  const uint32_t l0 = blockIdx.x * 64 + threadIdx.x;
  const bool live = l0 < t;
  const uint32_t l = live ? l0 : t - 1;
  const uint32_t d0 = blockIdx.y * kNewtonDB;
  Acc6 acc[kNewtonDB];
#pragma unroll
  for (int e = 0; e < kNewtonDB; ++e) acc6_zero(acc[e]);
  for (uint32_t i0 = 0; i0 < D1; i0 += 8) {
    uint64_t vv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) vv[u] = i0 + u < D1 ? vals[(size_t)(i0 + u) * t + l] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t i = i0 + u;
      if (i >= D1) break;
      const uint32_t v0 = (uint32_t)vv[u], v1 = (uint32_t)(vv[u] >> 32);
      const uint32_t* __restrict__ w = Wl + ((size_t)i * D1 + d0) * 3;
#pragma unroll
      for (int e = 0; e < kNewtonDB; ++e)
        if (d0 + e < D1) acc6_mac(acc[e], v0, v1, w[3 * e], w[3 * e + 1], w[3 * e + 2]);
    }
  }
  if (!live) return;
#pragma unroll
  for (int e = 0; e < kNewtonDB; ++e)
    if (d0 + e < D1) g[(size_t)(d0 + e) * t + l] = acc6_reduce(M, acc[e]);
}

__global__ void k_count_nz(uint32_t t, uint32_t D1, const uint64_t* __restrict__ g, uint32_t* __restrict__ cnt) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t) return;
  uint32_t n = 0;
  for (uint32_t d = 0; d < D1; ++d) n += g[(size_t)d * t + l] != 0;
  cnt[l] = n;
}

hipError_t newton_lift(const zr_mod& M, uint32_t t, uint32_t D1, const uint64_t* vals, const uint32_t* Wl,
                       uint64_t* g, uint32_t* cnt, hipStream_t s) {
  if (t == 0) return hipSuccess;
  TimedLaunch tl("newton", s);
  hipLaunchKernelGGL(k_newton_mat, dim3(cdiv(t, 64), cdiv(D1, kNewtonDB)), dim3(64), 0, s, M, t, D1, vals, Wl, g);
  hipLaunchKernelGGL(k_count_nz, dim3(cdiv(t, 256)), dim3(256), 0, s, t, D1, g, cnt);
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
  const uint32_t d = blockIdx.y;
  if (l >= t) return;
  const uint64_t c = g[(size_t)d * t + l];
  if (c == 0) return;
  // rank of (l, d) among the nonzero coefficients of term l
  uint32_t pos = off[l];
  for (uint32_t e = 0; e < d; ++e) pos += g[(size_t)e * t + l] != 0;
  for (uint32_t v = 0; v < nvars; ++v)
    exps_new[(size_t)v * ld_new + pos] = v == kvar ? (uint16_t)d : exps_old[(size_t)v * t + l];
  coef_new[pos] = c;
  mono_new[pos] = zr_shoup(M, mono_old[l], ypow[d], ypowp[d]);
}

hipError_t expand(const zr_mod& M, uint32_t t, uint32_t D1, uint32_t kvar, uint32_t nvars, const uint16_t* exps_old,
                  const uint64_t* mono_old, const uint64_t* g, const uint32_t* off, const uint64_t* ypow,
                  const uint64_t* ypowp, uint16_t* exps_new, uint64_t* coef_new, uint64_t* mono_new, uint32_t ld_new,
                  hipStream_t s) {
  if (t == 0) return hipSuccess;
  TimedLaunch tl("expand", s);
  hipLaunchKernelGGL(k_expand, dim3(cdiv(t, 256), D1), dim3(256), 0, s, M, t, D1, kvar, nvars, exps_old, mono_old, g,
                     off, ypow, ypowp, exps_new, coef_new, mono_new, ld_new);
  return hipGetLastError();
}

// ============================================================================
// Probe: value of the sparse polynomial at one point (power tables per
// variable; partial sums per thread, wave and block reductions mod p).
// ============================================================================

__device__ __forceinline__ uint64_t block_sum_mod(const zr_mod& M, uint64_t v, uint64_t* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = zr_add(M, sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(256) k_poly_eval(zr_mod M, uint32_t t, uint32_t nvars,
                                                   const uint16_t* __restrict__ exps, uint32_t ld,
                                                   const uint64_t* __restrict__ coef,
                                                   const uint64_t* __restrict__ tab, uint32_t ldtab,
                                                   uint64_t* __restrict__ partial) {
  __shared__ uint64_t sh[256];
  uint64_t acc = 0;
  for (uint32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < t; l += gridDim.x * blockDim.x) {
    uint64_t v = coef[l];
    for (uint32_t j = 0; j < nvars; ++j) v = zr_mul(M, v, tab[(size_t)j * ldtab + exps[(size_t)j * ld + l]]);
    acc = zr_add(M, acc, v);
  }
  const uint64_t s = block_sum_mod(M, acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_sum_mod(zr_mod M, uint32_t n, const uint64_t* __restrict__ partial,
                                                 uint64_t* __restrict__ result) {
  __shared__ uint64_t sh[256];
  uint64_t acc = 0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) acc = zr_add(M, acc, partial[i]);
  const uint64_t s = block_sum_mod(M, acc, sh);
  if (threadIdx.x == 0) *result = s;
}

hipError_t poly_eval_point(const zr_mod& M, uint32_t t, uint32_t nvars, const uint16_t* exps, uint32_t ld,
                           const uint64_t* coef, const uint64_t* tab, uint32_t ldtab, uint64_t* result,
                           uint64_t* partial, hipStream_t s) {
  const uint32_t nb = std::max<uint32_t>(1, std::min<uint32_t>(kPolyEvalBlocks, cdiv(t, 256)));
  hipLaunchKernelGGL(k_poly_eval, dim3(nb), dim3(256), 0, s, M, t, nvars, exps, ld, coef, tab, ldtab, partial);
  hipLaunchKernelGGL(k_sum_mod, dim3(1), dim3(256), 0, s, M, nb, partial, result);
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
  std::vector<hipEvent_t> pool;  // recycled events
  std::unordered_map<std::string, std::pair<uint64_t, double>> totals;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void resolve() {
    for (auto& p : pending) {
      (void)hipEventSynchronize(p.e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, p.e0, p.e1);
      auto& e = totals[p.name];
      e.first += 1;
      e.second += ms;
      pool.push_back(p.e0);
      pool.push_back(p.e1);
    }
    pending.clear();
  }
};
static TimingState g_timing;

TimedLaunch::TimedLaunch(const char* n, hipStream_t st) : name(n), s(st), e0(nullptr), e1(nullptr), on(false) {
  if (!g_timing.on) return;
  on = true;
  {
    std::lock_guard<std::mutex> g(g_timing.mu);
    e0 = g_timing.get();
    e1 = g_timing.get();
  }
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
