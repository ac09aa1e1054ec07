// Device bodies of the polynomial-path kernels, shared by the one-system
// launches (kernels.hip) and the batched, work-list launches (batch.hip).
// Each body handles one block's worth of work given its block coordinates, so
// that the same arithmetic runs whether the coordinates come from the launch
// grid or from a work list.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "field.hpp"

namespace zr {

__host__ __device__ static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// ---- transposed Vandermonde solve ----------------------------------------------

// Right-hand sides per tile: a tile of 20 leaves room for the chain state
// within 256 VGPRs.
constexpr uint32_t kMaxRT = 20;

struct VsArgs {
  zr_mod M;
  uint32_t t, L, S, R, ldv;
  uint32_t Sd;  // partial-sum slots per row and right-hand side in spart (chunk c adds into c mod Sd)
  const uint64_t* mono;
  const uint64_t* mono_p;
  const uint64_t* Mc;
  const uint64_t* VT;
  const uint64_t* qstart;
  uint64_t* Bc;
  uint64_t* spart;
  uint64_t* hpart;              // Horner partials per chunk (null: the dot-product pass runs no Horner)
  const uint32_t* CL = nullptr;  // limbs of M_r and r M_r for the chain pass (kChainW words per r)
  uint64_t* dpart = nullptr;      // D_c = sum over chunk c of r M_r m^(r - lo_c), per chunk and row
  // producer/consumer pass: right-hand sides of consumer k's tile; tile k's
  // rows (pc_ldv(tw[k]) words each) follow those of the tiles before it
  uint8_t tw[8] = {};
};

__device__ __forceinline__ void chunk_range(uint32_t t, uint32_t L, uint32_t c, uint32_t& lo, uint32_t& hi) {
  hi = t - c * L;
  lo = hi > L ? hi - L : 0;
}

// Packed right-hand sides, word idx of [ntile][t][ldv] (32-bit words): for
// jj < RT the value v = v^(tile*RT + jj)_{r+1} as three limbs v & (2^22-1),
// (v >> 22) & (2^22-1), v >> 44 at words 3jj..3jj+2; M_r at words 3RT, 3RT+1;
// zero padding.
__device__ __forceinline__ uint32_t pack_word(size_t idx, uint32_t t, uint32_t R, uint32_t RT, uint32_t ldv,
                                              const uint64_t* __restrict__ rhs, size_t ld_rhs,
                                              const uint64_t* __restrict__ Mc) {
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
  return out;
}

// Word w of packed row r of a producer/consumer tile of width tw whose first
// right-hand side is j0: the three 22-bit limbs of v^(j0+jj)_{r+1} at words
// 3jj..3jj+2, zero beyond (and for right-hand sides past R).
__device__ __forceinline__ uint32_t pack_word_pc(uint32_t r, uint32_t w, uint32_t R, uint32_t tw, uint32_t j0,
                                                 const uint64_t* __restrict__ rhs, size_t ld_rhs) {
  if (w >= 3 * tw) return 0;
  const uint32_t j = j0 + w / 3, limb = w % 3;
  const uint64_t v = j < R ? rhs[(size_t)j * ld_rhs + r] : 0;
  return (uint32_t)((v >> (22 * limb)) & (limb < 2 ? 0x3FFFFFu : 0xFFFFFFFFu));
}

// Shoup product x*w mod p in [0, 2p) for any 64-bit x (w < p, wp its Shoup
// quotient floor(w 2^64 / p)), for the producer's chain.  The high half of
// x*wp takes four 32x32->64 multiplies; the middle column is summed as a
// 65-bit value, so its carry travels through add-with-carry instructions
// (a compare and select for it cost three more vector instructions a step).
__device__ __forceinline__ uint64_t shoup_lazy_v(uint64_t x, uint64_t w, uint64_t wp, uint64_t p) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t w0 = (uint32_t)wp, w1 = (uint32_t)(wp >> 32);
  const uint64_t b = (uint64_t)x1 * w0 + __umulhi(x0, w0);                          // < 2^64
  const unsigned __int128 s = (unsigned __int128)((uint64_t)x0 * w1) + b;            // < 2^65
  const uint64_t qh = (uint64_t)x1 * w1 + (uint64_t)(s >> 32);                       // high half of x*wp
  return x * w - qh * p;
}

// r + c reduced into [0, 2p) for r, c in [0, 2p), given cm = c - 2p mod 2^64:
// r + c - 2p lies in [-2p, 2p), and r + cm carries out of bit 64 exactly
// when it is not negative; otherwise 2p is added back.
__device__ __forceinline__ uint64_t add_lazy2p(uint64_t r, uint64_t cm, uint64_t p2) {
  const uint64_t t = r + cm;
  return t + (t < r ? 0 : p2);
}

// Per-row scan over chunks: qstart[0] = 1, qstart[c] = m^L qstart[c-1] + B_{c-1}.
__device__ __forceinline__ void vs_scan_body(const VsArgs& a, uint32_t l, uint64_t* __restrict__ qstart,
                                             uint64_t* __restrict__ mL_out) {
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

// Carry-free exact dot products.  q = q0 + q1 2^32 (32-bit halves, per lane)
// and v = v0 + v1 2^22 + v2 2^44 (22-bit limbs, packed once per system), so
//   q v = q0 v0 + q0 v1 2^22 + q1 v0 2^32 + q0 v2 2^44 + q1 v1 2^54 + q1 v2 2^76,
// six 32x32 products below 2^54, each summed by one v_mad_u64_u32 into its own
// 64-bit column.  Every kFold steps the bits above each column's range are
// moved into the column of matching weight (exact shifts and adds) and the top
// column is reduced mod p, so sums of any length stay exact.
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

// Move everything above bit 54 of each weight-0..44 column into w54,
// everything above bit 22 of w54 into w76, and reduce w76 mod p (its weight
// 2^76 is applied mod p at the end, so only its residue matters).  Between two
// folds each column gains at most kFold products below 2^54, so no column can
// wrap, however long the sum.
__device__ __forceinline__ void acc6_fold(Acc6& a, const zr_mod& M) {
  a.w54 += (a.w0 >> 54) + (a.w22 >> 32) + (a.w32 >> 22) + (a.w44 >> 10);
  a.w0 &= (1ull << 54) - 1;
  a.w22 &= (1ull << 32) - 1;
  a.w32 &= (1ull << 22) - 1;
  a.w44 &= (1ull << 10) - 1;
  a.w76 += a.w54 >> 22;
  a.w54 &= (1ull << 22) - 1;
  a.w76 = zr_mod128(M, 0, a.w76);
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


// Pass 2 for 64 rows (one wave, lane = row): chain + Horner + RT right-hand-side
// dot products over one chunk.  Packed row r of a tile is identical for all
// lanes: each 64-byte group of it is one scalar load, issued for step r-1 as
// soon as step r has consumed the group, so its latency hides behind the
// remaining work.
struct alignas(64) VGroup {
  uint32_t w[16];
};

template <int RT>
__device__ __forceinline__ void vs_dots_body(const VsArgs& a, uint32_t rb, uint32_t c, uint32_t tile) {
  constexpr int LDV = (3 * RT + 2 + 15) & ~15;
  constexpr int G = LDV / 16;
  const uint32_t l0 = rb * 64 + (threadIdx.x & 63);
  const bool live = l0 < a.t;
  const uint32_t l = live ? l0 : a.t - 1;
  uint32_t lo, hi;
  chunk_range(a.t, a.L, c, lo, hi);
  const zr_mod M = a.M;
  const uint64_t p2 = 2 * M.p;  // below 2^64 since p < 2^63
  const uint64_t m = a.mono[l], mp = a.mono_p[l];
  uint64_t q = a.qstart ? a.qstart[(size_t)c * a.t + l] : 1 % M.p;
  uint64_t h = 0;
  Acc6 acc[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) acc6_zero(acc[j]);
  const VGroup* __restrict__ rows = (const VGroup*)((const uint32_t*)a.VT + (size_t)tile * a.t * LDV);
  const bool horner = tile == 0 && a.hpart != nullptr;
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
    // q and h kept in [0, 2p) (the column sums take any q below 2^64)
    if (horner) h = add_lazy2p(shoup_lazy_v(h, m, mp, M.p), q - p2, p2);
    q = add_lazy2p(shoup_lazy_v(q, m, mp, M.p), Mr - p2, p2);
    if (++since == kFold) {
#pragma unroll
      for (int j = 0; j < RT; ++j) acc6_fold(acc[j], M);
      since = 0;
    }
    if (r == lo) break;
    r = rn;
  }
  if (live) {
    const uint32_t j0 = tile * RT;
#pragma unroll
    for (int j = 0; j < RT; ++j)
      if (j0 + j < a.R) a.spart[((size_t)c * a.R + j0 + j) * a.t + l] = acc6_reduce(M, acc[j]);
    if (horner) a.hpart[(size_t)c * a.t + l] = h >= M.p ? h - M.p : h;
  }
}

// Producer/consumer form of pass 2 for systems with several right-hand-side
// tiles: wave 0 of the workgroup runs the chain and Horner once and publishes
// q_{l,r} through LDS in blocks of kQB steps (double buffered); wave 1 + tile
// accumulates that tile's RT dot products.  Compared with one wave per tile,
// the chain is computed once instead of ntile times and the consumer waves
// hold no chain state.
constexpr uint32_t kQB = 16;
constexpr uint32_t kPcMinR = 10;     // more right-hand sides than this: producer/consumer pass
constexpr uint32_t kPcRT = 10;       // right-hand sides per consumer wave (at most)
constexpr uint32_t kPcMaxTiles = 7;  // consumer waves per workgroup (at most)
// Right-hand sides of one producer/consumer pass, at most: seven consumer waves
// of ten values take 140 VGPRs, which leaves one 8-wave workgroup per CU; of
// nine (128 VGPRs) two fit (t = 10^5: 64 values ran at 14.5 TOP/s, 60 at 19.3).
// More right-hand sides are solved in groups (vsolve).
constexpr uint32_t kPcMaxR = 63;
// Widest tile of an uneven split (pc_widths): nine values keep 128 VGPRs and
// two 8-wave workgroups per CU.
constexpr uint32_t kPcUnevenMax = 9;

// Consumer waves per workgroup for R right-hand sides: at least
// cdiv(R, kPcRT), rounded up so that the workgroup's 1 + ntile waves are a
// multiple of the CU's four SIMDs.  Every SIMD then carries the same share of
// the workgroup, and the barriers that pace producer and consumers do not wait
// on one overloaded SIMD (at R = 40, workgroups of 5 and 6 waves measured 1.7x
// and 1.2x slower than 8).  0 when R is above kPcMaxR.
__host__ __device__ inline uint32_t pc_tiles_for(uint32_t R) {
  if (R > kPcMaxR) return 0;
  uint32_t n = cdiv(R, kPcRT);
  while ((1 + n) % 4) ++n;
  return n <= kPcMaxTiles ? n : 0;
}

// Read-only data that every lane of a wave reads at the same address, seen
// through the constant address space: the loads stay scalar even after the
// workgroup barriers (which otherwise count as possible writers).
template <class T>
using const_as = const __attribute__((address_space(4))) T*;

// 16 words of a uniform array at any 4-byte boundary (one scalar load)
typedef uint32_t u32x16a4 __attribute__((ext_vector_type(16))) __attribute__((aligned(4)));

// Pass 1 for row l, chunk c < S-1: B_c = sum_{lo <= r < hi} M_r m^(r-lo), the
// chain over the chunk started from 0, evaluated by baby steps and giant
// steps.  With r - lo = K j + i (0 <= i < K),
//   B_c = sum_j (m^K)^j s_j,   s_j = sum_i M_(lo+Kj+i) m^i:
// the K powers m^i are made once per row and chunk (K Shoup products); each
// s_j is an exact six-column sum of K products of the uniform M_r (22-bit
// limbs, scalar) with the lane's powers, reduced once; the outer sum is Horner
// in m^K.  (The batched solve and the multi-prime evaluation; the one-system
// solve uses vs_chain_cl below.)
constexpr int kChainK = 32;  // K: below kFold, so a block's columns never fold

__device__ __forceinline__ void vs_chain_body(const VsArgs& a, uint32_t l, uint32_t c) {
  uint32_t lo, hi;
  chunk_range(a.t, a.L, c, lo, hi);
  const zr_mod M = a.M;
  const uint64_t m = a.mono[l], mp = a.mono_p[l];
  const_as<uint64_t> Mc = (const_as<uint64_t>)a.Mc;  // uniform: the chunk is the block's
  uint64_t pw[kChainK];
  pw[0] = 1 % M.p;
#pragma unroll
  for (int i = 1; i < kChainK; ++i) pw[i] = zr_shoup(M, pw[i - 1], m, mp);
  const uint64_t mK = zr_shoup(M, pw[kChainK - 1], m, mp), mKp = zr_shoup_pre(M, mK);
  // s_j of the block starting at base: the top block may be partial (guarded
  // loads), every other block is full
  auto block = [&](uint32_t base, bool guard) {
    Acc6 acc;
    acc6_zero(acc);
#pragma unroll
    for (int i = 0; i < kChainK; ++i) {
      const uint64_t Mr = (!guard || base + i < hi) ? Mc[base + i] : 0;
      acc6_mac(acc, (uint32_t)pw[i], (uint32_t)(pw[i] >> 32), (uint32_t)(Mr & 0x3FFFFF),
               (uint32_t)((Mr >> 22) & 0x3FFFFF), (uint32_t)(Mr >> 44));
    }
    return acc6_reduce(M, acc);
  };
  const uint32_t nfull = (hi - lo) / kChainK;
  uint64_t y = 0;
  if (lo + nfull * kChainK < hi) y = block(lo + nfull * kChainK, true);
  for (uint32_t j = nfull; j-- > 0;) y = zr_add(M, zr_shoup(M, y, mK, mKp), block(lo + j * kChainK, false));
  a.Bc[(size_t)c * a.t + l] = y;
}

// Coefficients of the one-system chain pass, split once into 22-bit limbs:
// per r < t the limbs of M_r and of r M_r (six 32-bit words).
constexpr uint32_t kChainW = 6;

// Sum of a block's six columns mod p when every column is below 2^60 (at most
// 64 products since the last fold): the value is below 2^137, three words
// with the top one below 2^9.  No branch, so the products of a block and its
// reduction stay in one basic block.
__device__ __forceinline__ uint64_t acc6_reduce_block(const zr_mod& M, const Acc6& a) {
  const zr_u128 low = (zr_u128)a.w0 + ((zr_u128)a.w22 << 22) + ((zr_u128)a.w32 << 32) + ((zr_u128)a.w44 << 44) +
                      ((zr_u128)a.w54 << 54);  // below 2^115
  const zr_u128 mid = (low >> 64) + ((zr_u128)a.w76 << 12);  // bits 64.. of the value, below 2^73
  const uint64_t w0 = (uint64_t)low, w1 = (uint64_t)mid, w2 = (uint64_t)(mid >> 64);
  uint64_t r = zr_mod128(M, 0, w2);
  r = zr_mod128(M, r, w1);
  return zr_mod128(M, r, w0);
}

// Pass 1 of the one-system solve for row l and chunk c: B_c as above (WB,
// chunks c < S-1) and, when delta comes from this pass (WD), also
// D_c = sum_{lo <= r < hi} r M_r m^(r-lo), the chunk's share of
// m M'(m) = sum_r r M_r m^r, from the same powers of m.  The coefficients come
// from the limb array CL: eight steps of both streams (48 words) arrive by
// three 16-word scalar loads at a time.
template <bool WB, bool WD>
__device__ __forceinline__ void vs_chain_cl(const VsArgs& a, uint32_t l, uint32_t c) {
  // baby steps per block: with both streams 48 (against 32) cuts the
  // reductions per step and still leaves two waves per SIMD; one stream keeps
  // 32 and three waves.  A block's columns stay below 2^60, as
  // acc6_reduce_block needs.
  constexpr int KC = WB && WD ? 48 : kChainK;
  uint32_t lo, hi;
  chunk_range(a.t, a.L, c, lo, hi);
  const zr_mod M = a.M;
  const uint64_t m = a.mono[l], mp = a.mono_p[l];
  const_as<uint32_t> CL = (const_as<uint32_t>)a.CL;  // uniform: the chunk is the block's
  uint64_t pw[KC];
  pw[0] = 1 % M.p;
#pragma unroll
  for (int i = 1; i < KC; ++i) pw[i] = zr_shoup(M, pw[i - 1], m, mp);
  const uint64_t mK = zr_shoup(M, pw[KC - 1], m, mp), mKp = zr_shoup_pre(M, mK);
  uint64_t y = 0, z = 0;
  Acc6 ab, ad;
  auto fold_in = [&]() {
    if (WB) y = zr_add(M, zr_shoup(M, y, mK, mKp), acc6_reduce_block(M, ab));
    if (WD) z = zr_add(M, zr_shoup(M, z, mK, mKp), acc6_reduce_block(M, ad));
  };
  auto step = [&](int i, uint32_t b0, uint32_t b1, uint32_t b2, uint32_t d0, uint32_t d1, uint32_t d2) {
    const uint32_t p0 = (uint32_t)pw[i], p1 = (uint32_t)(pw[i] >> 32);
    if (WB) acc6_mac(ab, p0, p1, b0, b1, b2);
    if (WD) acc6_mac(ad, p0, p1, d0, d1, d2);
  };
  // the top block, r in [base, hi), may be partial
  const uint32_t nfull = (hi - lo) / KC;
  const uint32_t base_top = lo + nfull * KC;
  if (base_top < hi) {
    acc6_zero(ab);
    acc6_zero(ad);
    const uint32_t n = hi - base_top;
#pragma unroll
    for (int i = 0; i < KC; ++i)
      if ((uint32_t)i < n) {
        const_as<uint32_t> w = CL + (size_t)(base_top + i) * kChainW;
        step(i, w[0], w[1], w[2], w[3], w[4], w[5]);
      }
    fold_in();
  }
  for (uint32_t j = nfull; j-- > 0;) {
    acc6_zero(ab);
    acc6_zero(ad);
#pragma unroll
    for (int g = 0; g < KC / 8; ++g) {
      // the group's address passes through an empty asm so that its loads
      // cannot be hoisted above the previous group's products
      const_as<u32x16a4> src = (const_as<u32x16a4>)(CL + (size_t)(lo + j * KC + 8 * g) * kChainW);
      asm volatile("" : "+s"(src));
      const u32x16a4 c0 = src[0], c1 = src[1], c2 = src[2];
      uint32_t w[48];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        w[k] = c0[k];
        w[16 + k] = c1[k];
        w[32 + k] = c2[k];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
        step(8 * g + i, w[6 * i], w[6 * i + 1], w[6 * i + 2], w[6 * i + 3], w[6 * i + 4], w[6 * i + 5]);
      // one group's 48 words live at a time: the next group's loads are not
      // hoisted above this group's products
      __builtin_amdgcn_sched_barrier(0);
    }
    fold_in();
  }
  if (WB) a.Bc[(size_t)c * a.t + l] = y;
  if (WD) a.dpart[(size_t)c * a.t + l] = z;
}

// Packed row of the producer/consumer pass: the 3 RT limbs of the tile's
// values at one step, without M_r (the producer reads M_r itself).  It is
// loaded through the scalar cache as one 16-word group and a tail of K words,
// K a power of two up to 16 (none for RT <= 5), so a row of six values is 18
// words (72 bytes) rather than two 64-byte groups: a chunk's rows take less
// of the L2 that the workgroups on one XCD share.  Rows start at any 4-byte
// boundary, which scalar loads accept.
__host__ __device__ constexpr uint32_t pc_tail(uint32_t RT) {
  return 3 * RT <= 16 ? 0 : 3 * RT - 16 <= 2 ? 2 : 3 * RT - 16 <= 4 ? 4 : 3 * RT - 16 <= 8 ? 8 : 16;
}
__host__ __device__ constexpr uint32_t pc_ldv(uint32_t RT) { return 16 + pc_tail(RT); }

template <int K>
struct PcTail {
  typedef uint32_t type __attribute__((ext_vector_type(K))) __attribute__((aligned(4)));
};
template <int K>
struct PcRow {
  u32x16a4 a;
  typename PcTail<K>::type b;
};
template <>
struct PcRow<0> {
  u32x16a4 a;
};
template <int K>
__device__ __forceinline__ uint32_t pc_word(const PcRow<K>& row, int w) {
  if constexpr (K == 0)
    return row.a[w];
  else
    return w < 16 ? row.a[w] : row.b[w - 16];
}
template <int K>
__device__ __forceinline__ void pc_load(PcRow<K>& row, const_as<uint32_t> base) {
  row.a = *(const_as<u32x16a4>)base;
  if constexpr (K != 0) row.b = *(const_as<typename PcTail<K>::type>)(base + 16);
}
// Every word of the row stays live up to the end of its step, unused words
// included: a value of the step (such as the dead carry-out of a multiply) is
// then never given a register that a still pending row load writes, which
// would force a wait for that load.
template <int K>
__device__ __forceinline__ void pc_keep(const PcRow<K>& row) {
  asm volatile("" ::"s"(row.a));
  if constexpr (K != 0) asm volatile("" ::"s"(row.b));
}

// One consumer step: q (already in registers) times row r held in cur.  Row
// rn and the next step's q are requested into nxt and qn right after the
// first product of the step: the wait that the compiler places before that
// first use of cur and q then covers only requests a whole step old, and the
// sched barriers keep the scheduler from moving the requests down to their
// own uses.
template <int RT, int K>
__device__ __forceinline__ void vs_pc_step(const zr_mod& M, Acc6 (&acc)[RT], const PcRow<K>& cur,
                                           PcRow<K>& nxt, uint64_t& q, const uint64_t* qnext,
                                           const_as<uint32_t> rows, uint32_t rn, uint32_t& since) {
  constexpr uint32_t LDV = pc_ldv(RT);
  const uint32_t q0 = (uint32_t)q, q1 = (uint32_t)(q >> 32);
  acc6_mac(acc[0], q0, q1, pc_word(cur, 0), pc_word(cur, 1), pc_word(cur, 2));
  __builtin_amdgcn_sched_barrier(0);
  pc_load(nxt, rows + (size_t)rn * LDV);
  const uint64_t qn = *qnext;
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int jj = 1; jj < RT; ++jj)
    acc6_mac(acc[jj], q0, q1, pc_word(cur, 3 * jj), pc_word(cur, 3 * jj + 1), pc_word(cur, 3 * jj + 2));
  pc_keep(cur);
  if (++since == kFold) {
#pragma unroll
    for (int j = 0; j < RT; ++j) acc6_fold(acc[j], M);
    since = 0;
  }
  q = qn;
}

// Consumer of a tile of RT right-hand sides, j0 the first of them, whose
// packed rows (pc_ldv(RT) words each) start at rows.
template <int RT>
__device__ __forceinline__ void vs_pc_consume(const VsArgs& a, uint32_t c, uint32_t lo, uint32_t hi, uint32_t nb,
                                              bool live, uint32_t l, uint32_t lane, uint32_t j0,
                                              const_as<uint32_t> rows, uint64_t (*qbuf)[kQB][64], const zr_mod& M) {
  constexpr uint32_t LDV = pc_ldv(RT);
  constexpr int K = (int)pc_tail(RT);
  Acc6 acc[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) acc6_zero(acc[j]);
  // two row buffers: while one feeds the products of step r the other receives
  // row r-1, so each row's scalar loads have a whole step to arrive.  Blocks
  // hold an even number of steps except the last, so steps go in pairs (no
  // branch between a request and its use) and a last odd step, if any, runs
  // alone.
  uint32_t r = hi - 1;
  uint32_t since = 0;
  PcRow<K> b0, b1;
  pc_load(b0, rows + (size_t)r * LDV);
  for (uint32_t it = 0; it <= nb; ++it) {
    if (it >= 1) {
      const uint32_t b = it - 1;
      const uint32_t s_end = min(kQB, hi - lo - b * kQB);
      const uint64_t* qb = &qbuf[b & 1][0][lane];
      uint64_t q = qb[0];
      uint32_t s = 0;
      for (; s + 2 <= s_end; s += 2) {
        // the q of step s_end (past the block) is read from the last slot and not used
        vs_pc_step<RT, K>(M, acc, b0, b1, q, qb + 64 * (s + 1), rows, r > lo ? r - 1 : r, since);
        r = r > lo ? r - 1 : r;
        vs_pc_step<RT, K>(M, acc, b1, b0, q, qb + 64 * min(s + 2, kQB - 1), rows, r > lo ? r - 1 : r, since);
        r = r > lo ? r - 1 : r;
      }
      if (s < s_end) {
        vs_pc_step<RT, K>(M, acc, b0, b1, q, qb, rows, r > lo ? r - 1 : r, since);
        r = r > lo ? r - 1 : r;
        b0 = b1;
      }
    }
    __syncthreads();
  }
  if (live) {
    // chunk c adds into partial-sum slot c mod Sd: the chunks of one launch
    // take distinct slots, and chunks c >= Sd (later launches) add to what
    // the earlier chunk of their slot left there
    const uint32_t slot = c % a.Sd;
#pragma unroll
    for (int j = 0; j < RT; ++j)
      if (j0 + j < a.R) {
        uint64_t* dst = a.spart + ((size_t)slot * a.R + j0 + j) * a.t + l;
        const uint64_t v = acc6_reduce(M, acc[j]);
        *dst = c >= a.Sd ? zr_add(M, v, *dst) : v;
      }
  }
}


// HORNER: the producer also sums h = q(m) over the chunk into hpart (the
// batched solve); without it delta comes from the chain pass's D_c.  UNEVEN:
// tiles may be one value narrower or wider than RT (the bodies for those
// widths are compiled in, which costs registers; off, every tile is RT wide).
template <int RT, bool HORNER, bool UNEVEN = false>
__device__ __forceinline__ void vs_dots_pc_body(const VsArgs& a, uint32_t rb, uint32_t c, uint32_t ntile,
                                                uint64_t (*qbuf)[kQB][64]) {
  // the wave index is uniform within a wave: say so, so that each role's code
  // is compiled as uniform control flow (scalar loads, scalar loop counters)
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const uint32_t l0 = rb * 64 + lane;
  const bool live = l0 < a.t;
  const uint32_t l = live ? l0 : a.t - 1;
  uint32_t lo, hi;
  chunk_range(a.t, a.L, c, lo, hi);
  const uint32_t nb = (hi - lo + kQB - 1) / kQB;
  const zr_mod M = a.M;
  if (wave == 0) {
    // producer: q and Horner; M_r read eight at a time, the next eight in flight
    const uint64_t m = a.mono[l], mp = a.mono_p[l];
    uint64_t q = a.qstart ? a.qstart[(size_t)c * a.t + l] : 1 % M.p;
    uint64_t h = 0;
    const_as<uint64_t> Mc = (const_as<uint64_t>)a.Mc;
    const uint64_t p2 = 2 * M.p;  // below 2^64 since p < 2^63
    // a copy of 2p kept in vector registers: the select that adds it back
    // would otherwise move it from scalar registers at every step (one scalar
    // operand per vector instruction besides the lane mask)
    uint64_t p2v = p2;
    asm volatile("" : "+v"(p2v));
    uint32_t r = hi;  // the next step is r - 1
    uint64_t cur[8], nxt[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) cur[u] = r >= (uint32_t)u + 1 + lo ? Mc[r - 1 - u] : 0;
    for (uint32_t it = 0; it <= nb; ++it) {
      if (it < nb) {
#pragma unroll
        for (uint32_t g8 = 0; g8 < kQB / 8; ++g8) {
          const uint32_t rn = r > lo + 8 ? r - 8 : lo;
#pragma unroll
          for (int u = 0; u < 8; ++u) nxt[u] = rn >= (uint32_t)u + 1 + lo ? Mc[rn - 1 - u] : 0;
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (r > lo + (uint32_t)u) {
              // q and h kept in [0, 2p); the consumers' column sums take any
              // q below 2^64.  cur[u] - 2p is uniform (scalar unit).
              qbuf[it & 1][g8 * 8 + u][lane] = q;
              if (HORNER) h = add_lazy2p(shoup_lazy_v(h, m, mp, M.p), q - p2, p2v);
              q = add_lazy2p(shoup_lazy_v(q, m, mp, M.p), cur[u] - p2, p2v);
            }
          }
          r = rn;
#pragma unroll
          for (int u = 0; u < 8; ++u) cur[u] = nxt[u];
        }
      }
      __syncthreads();
    }
    if (HORNER && live) a.hpart[(size_t)c * a.t + l] = h >= M.p ? h - M.p : h;
    return;
  }
  // consumer of tile wave - 1, of width a.tw[tile]: RT, or (uneven tiles,
  // pc_widths) one less or one more
  const uint32_t tile = wave - 1;
  if (tile >= ntile) {
    for (uint32_t it = 0; it <= nb; ++it) __syncthreads();
    return;
  }
  // the tile's first right-hand side, row offset and width (unrolled, so that
  // tw is only read at fixed indices: a copy of the arguments indexed at run
  // time would go to scratch memory)
  uint32_t j0 = 0, off = 0, w = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPcMaxTiles; ++k) {
    if (k < tile) {
      j0 += a.tw[k];
      off += pc_ldv(a.tw[k]);
    }
    if (k == tile) w = a.tw[k];
  }
  const_as<uint32_t> rows = (const_as<uint32_t>)((const uint32_t*)a.VT + (size_t)off * a.t);
  if constexpr (UNEVEN && RT > 1) {
    if (w == RT - 1) {
      vs_pc_consume<RT - 1>(a, c, lo, hi, nb, live, l, lane, j0, rows, qbuf, M);
      return;
    }
  }
  if constexpr (UNEVEN && RT + 1 <= kPcUnevenMax) {
    if (w == RT + 1) {
      vs_pc_consume<RT + 1>(a, c, lo, hi, nb, live, l, lane, j0, rows, qbuf, M);
      return;
    }
  }
  vs_pc_consume<RT>(a, c, lo, hi, nb, live, l, lane, j0, rows, qbuf, M);
}

// Inverses of the values w of a block's kDeltaBlock threads by Montgomery's
// simultaneous inversion: with P<_i and P>_i the products of the w of the
// threads before and after thread i, 1/w_i = P<_i P>_i / (product of all), so
// the block pays one inversion and a few products per thread instead of one
// inversion per thread.  The products within a wave are shuffle scans; the
// four wave totals meet in LDS.  Threads with use = false or w = 0 enter the
// products as 1 and get 0.  Every thread of the block must call it.
constexpr uint32_t kDeltaBlock = 256;

__device__ __forceinline__ uint64_t block_inverse(const zr_mod& M, uint64_t w, bool use, uint64_t* sh) {
  constexpr uint32_t NW = kDeltaBlock / 64;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t one = 1 % M.p;
  const bool part = use && w != 0;
  uint64_t pre = part ? w : one, suf = pre;  // inclusive prefix / suffix products within the wave
#pragma unroll
  for (uint32_t d = 1; d < 64; d <<= 1) {
    const uint64_t a = __shfl_up(pre, d), b = __shfl_down(suf, d);
    if (lane >= d) pre = zr_mul(M, pre, a);
    if (lane + d < 64) suf = zr_mul(M, suf, b);
  }
  uint64_t epre = __shfl_up(pre, 1), esuf = __shfl_down(suf, 1);
  if (lane == 0) epre = one;
  if (lane == 63) esuf = one;
  if (lane == 63) sh[wave] = pre;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t all = one;
    for (uint32_t q = 0; q < NW; ++q) all = zr_mul(M, all, sh[q]);
    sh[NW] = zr_inv(M, all);
  }
  __syncthreads();
  uint64_t other = sh[NW];
  for (uint32_t q = 0; q < NW; ++q)
    if (q != wave) other = zr_mul(M, other, sh[q]);
  return part ? zr_mul(M, zr_mul(M, epre, esuf), other) : 0;
}

// Combine chunks, part 1 for the rows of one block (l = row of this thread,
// live when l < t): w = m_l delta_l = m_l M'(m_l), either as
// t m^t + sum_c m^{lo_c} D_c from the chain pass's D_c, or as m times
// sum_c m^{lo_c} H_c from the Horner partials H_c of the dot-product pass,
// both by Horner over the chunks; then the inverses of the block's w (one
// inversion per block) with their Shoup constants into winv[2t].  A zero w
// marks the system singular.  Every thread of the block must call it (it
// holds barriers).
__device__ __forceinline__ void vs_delta_block(const VsArgs& a, uint32_t l, const uint64_t* __restrict__ mLv,
                                               uint64_t* __restrict__ winv, int32_t* __restrict__ status,
                                               uint64_t* sh) {
  const zr_mod M = a.M;
  const bool live = l < a.t;
  uint64_t w = 0;
  if (live) {
    const uint64_t m = a.mono[l];
    // chunk partials from the top chunk (c = 0) down, Horner in m^L (m^len
    // for the last, shorter chunk)
    const uint64_t* part = a.dpart ? a.dpart : a.hpart;
    uint64_t acc = part[l];
    uint64_t mL = 0, mLp = 0;
    if (a.S > 1) {
      mL = mLv[l];
      mLp = zr_shoup_pre(M, mL);
      const uint32_t len_last = a.t - (a.S - 1) * a.L;
      const uint64_t mlast = zr_pow(M, m, len_last);
      // with D_c, the leading term t m^t = m^(lo_0) t m^L enters first
      if (a.dpart) acc = zr_add(M, zr_mul(M, a.t % M.p, mL), acc);
      for (uint32_t c = 1; c < a.S; ++c) {
        const uint64_t pc = part[(size_t)c * a.t + l];
        acc = (c + 1 < a.S) ? zr_add(M, zr_shoup(M, acc, mL, mLp), pc) : zr_add(M, zr_mul(M, acc, mlast), pc);
      }
    } else if (a.dpart) {
      acc = zr_add(M, zr_mul(M, a.t % M.p, zr_pow(M, m, a.t)), acc);
    }
    // with D_c the sum is m M'(m) itself; the Horner partials give M'(m)
    w = a.dpart ? acc : zr_mul(M, m, acc);
    if (w == 0) atomicCAS(status, 0, -3);  // ZR_ESINGULAR, unless an earlier step already failed
  }
  const uint64_t wi = block_inverse(M, w, live, sh);
  if (live) {
    winv[l] = wi;
    winv[a.t + l] = wi ? zr_shoup_pre(M, wi) : 0;
  }
}

// Combine chunks, part 2 for row l and right-hand side j:
// a^(j)_l = (sum_c s^(j)_{l,c}) / (m_l delta_l).
__device__ __forceinline__ void vs_scale_body(const VsArgs& a, uint32_t l, uint32_t j, const uint64_t* __restrict__ winv,
                                              uint64_t* __restrict__ out, size_t ld_out) {
  const zr_mod M = a.M;
  uint64_t s = 0;
  for (uint32_t c = 0; c < a.Sd; ++c) s = zr_add(M, s, a.spart[((size_t)c * a.R + j) * a.t + l]);
  out[(size_t)j * ld_out + l] = zr_shoup(M, s, winv[l], winv[a.t + l]);
}

// ---- master polynomial (product tree) -------------------------------------------

__device__ __forceinline__ uint4 limbs22(uint64_t v) {
  return make_uint4((uint32_t)(v & 0x3FFFFF), (uint32_t)((v >> 22) & 0x3FFFFF), (uint32_t)(v >> 44), 0u);
}

// Bottom levels (factors of degree < 64) in LDS for leaves [b, b+64) of a
// system of t leaves: pairwise products level by level; node boundaries
// (multiples of 2h) coincide with those of the whole tree, including the
// ragged end.  Writes the non-leading coefficients and their limbs.
// buf: 2 x 64 words of LDS.
__device__ __forceinline__ void master_small_body(const zr_mod& M, uint32_t t, uint32_t b,
                                                  const uint64_t* __restrict__ mono, uint64_t* __restrict__ out,
                                                  uint4* __restrict__ limbs, uint64_t* buf) {
  const uint32_t k = threadIdx.x & 63;
  const uint32_t n = std::min<uint32_t>(64, t - b);
  uint64_t* cur = buf;
  uint64_t* nxt = buf + 64;
  if (k < n) cur[k] = zr_neg(M, mono[b + k] % M.p);
  __syncthreads();
  for (uint32_t half = 1; half < 64 && half < t; half *= 2) {
    if (k < n) {
      const uint32_t a = (k / (2 * half)) * (2 * half);
      const uint32_t n1 = std::min(half, n - a);
      const uint32_t n2 = std::min(half, n - a - n1);
      const uint32_t kk = k - a;
      const uint64_t* Lc = cur + a;
      const uint64_t* Rc = cur + a + n1;
      zr_acc192 acc;
      zr_acc_zero(acc);
      if (n2 > 0) {
        const uint32_t ilo = kk + 1 > n2 ? kk + 1 - n2 : 0;
        const uint32_t ihi = std::min(kk, n1 - 1);
        for (uint32_t i = ilo; i <= ihi; ++i) zr_acc_mac(acc, Lc[i], Rc[kk - i]);
      }
      if (kk >= n1) zr_acc_mac(acc, 1, Rc[kk - n1]);
      if (kk >= n2) zr_acc_mac(acc, 1, Lc[kk - n2]);
      nxt[k] = zr_acc_reduce(M, acc);
    }
    __syncthreads();
    uint64_t* tswap = cur;
    cur = nxt;
    nxt = tswap;
  }
  if (k < n) {
    out[b + k] = cur[k];
    limbs[b + k] = limbs22(cur[k]);
  }
}

// Large levels (factors of degree >= 64): a wave owns 64 consecutive output
// coefficients g0.. of one product and one chunk ic of the convolution index.
// The factor L_i is wave-uniform: the level's coefficients carry their 22-bit
// limbs (four 32-bit words per value) so that eight of them arrive with two
// 64-byte scalar loads.  The window of R needed by the wave, R_{k-i} for its k
// and i, is staged once in LDS (win: 64 + IC + 8 words).  With one chunk
// per product the wave finishes the coefficient (adding the terms of the
// leading ones) and writes it with its limbs; otherwise chunk partial sums go
// to part[ic][g] and master_sum_body finishes them.
// Chunk length IC of the convolution index for a level with factors of degree
// `half` and `blocks` row blocks in total: short enough that the level has
// about 2048 waves, so that the small levels are not bound by one wave's serial
// sum, long enough to keep the partial sums few (64 chunks per product, up to
// IC = 4096, whose LDS window is 33 KB).
__host__ __device__ inline uint32_t conv_ic(uint32_t half, uint64_t blocks) {
  uint32_t ic = 512;
  while (ic > 64 && blocks * ((half + ic - 1) / ic) < 2048) ic /= 2;
  while ((half + ic - 1) / ic > 64 && ic < 4096) ic *= 2;
  return ic;
}

struct alignas(16) L8 {
  uint4 v[8];
};

__device__ __forceinline__ uint64_t master_linear_terms(const zr_mod& M, uint64_t s, const uint64_t* cur, uint32_t a,
                                                        uint32_t n1, uint32_t n2, uint32_t k) {
  if (k >= n1) s = zr_add(M, s, cur[a + n1 + (k - n1)]);
  if (k >= n2) s = zr_add(M, s, cur[a + (k - n2)]);
  return s;
}

// NW waves of one workgroup take 64 NW consecutive coefficients of one
// product (64 NW <= 2 half) and share one LDS window, so a window of
// 64 NW + IC words serves NW waves.
template <int NW = 1>
__device__ __forceinline__ void master_conv_body(const zr_mod& M, uint32_t t, uint32_t half, uint32_t IC, uint32_t nic,
                                                 uint32_t g0, uint32_t ic, const uint64_t* __restrict__ cur,
                                                 const uint4* __restrict__ limbs, uint64_t* __restrict__ part,
                                                 size_t ld_part, uint64_t* __restrict__ nxt,
                                                 uint4* __restrict__ limbs_nxt, uint64_t* win) {
  constexpr uint32_t W = 64 * NW;  // coefficients of the workgroup, from g0
  const uint32_t g = g0 + (threadIdx.x & (W - 1));
  const uint32_t a = (g0 / (2 * half)) * (2 * half);  // one product per workgroup since 2*half >= W
  const uint32_t n1 = std::min(half, t - a);
  const uint32_t n2 = std::min(half, t - a - n1);
  const uint32_t k0 = g0 - a;
  const uint32_t k = g - a;
  const uint64_t* __restrict__ Rc = cur + a + n1;
  Acc6 acc;
  acc6_zero(acc);
  uint32_t ilo = ic * IC, ihi = std::min(ilo + IC, n1);
  if (n2 > 0) {
    const uint32_t wlo = k0 + 1 > n2 ? k0 + 1 - n2 : 0;
    const uint32_t whi = std::min(k0 + W, n1);
    ilo = std::max(ilo, wlo);
    ihi = std::min(ihi, whi);
  } else {
    ihi = ilo;
  }
  if (ilo < ihi) {
    // round the i range up to whole groups of 8; the extra i are masked
    const uint32_t ihi8 = ilo + ((ihi - ilo + 7) & ~7u);
    // window: R index j = k - i for k in [k0, k0+W-1], i in [ilo, ihi8):
    // j in [k0 - ihi8 + 1, k0 + W - 1 - ilo]; terms with j outside [0, n2)
    // read zeros
    const int64_t jbase = (int64_t)k0 - (int64_t)ihi8 + 1;
    const uint32_t wlen = W - 1 + (ihi8 - ilo);
    for (uint32_t x = threadIdx.x & (W - 1); x < wlen; x += W) {
      const int64_t j = jbase + x;
      win[x] = (j >= 0 && j < (int64_t)n2) ? Rc[j] : 0;
    }
    __syncthreads();
    const uint4* __restrict__ Lg = limbs + a;
    const uint64_t* __restrict__ wk = win + ((int64_t)k - jbase);
    L8 L = *(const L8*)(Lg + ilo);
    uint32_t since = 0;
    for (uint32_t i = ilo; i < ihi8; i += 8) {
      // fetch the next group of eight coefficients while this one is used
      const uint32_t in8 = i + 8 < ihi8 ? i + 8 : i;
      const L8 Ln = *(const L8*)(Lg + in8);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const uint64_t Rv = wk[-(int64_t)(i + u)];
        const bool in = i + u < ihi;
        acc6_mac(acc, (uint32_t)Rv, (uint32_t)(Rv >> 32), in ? L.v[u].x : 0u, in ? L.v[u].y : 0u, in ? L.v[u].z : 0u);
      }
      L = Ln;
      since += 8;
      if (since == kFold) {  // chunks longer than kFold products
        acc6_fold(acc, M);
        since = 0;
      }
    }
  }
  if (g >= t) return;
  const uint64_t s = acc6_reduce(M, acc);
  if (nic == 1) {
    const uint64_t v = master_linear_terms(M, s, cur, a, n1, n2, k);
    nxt[g] = v;
    limbs_nxt[g] = limbs22(v);
  } else {
    part[(size_t)ic * ld_part + g] = s;
  }
}

__device__ __forceinline__ void master_sum_body(const zr_mod& M, uint32_t t, uint32_t half, uint32_t nic, uint32_t g,
                                                const uint64_t* __restrict__ cur, const uint64_t* __restrict__ part,
                                                size_t ld_part, uint64_t* __restrict__ nxt,
                                                uint4* __restrict__ limbs_nxt) {
  const uint32_t a = (g / (2 * half)) * (2 * half);
  const uint32_t n1 = std::min(half, t - a);
  const uint32_t n2 = std::min(half, t - a - n1);
  uint64_t s = 0;
  for (uint32_t ic = 0; ic < nic; ++ic) s = zr_add(M, s, part[(size_t)ic * ld_part + g]);
  const uint64_t v = master_linear_terms(M, s, cur, a, n1, n2, g - a);
  nxt[g] = v;
  limbs_nxt[g] = limbs22(v);
}

// ---- Newton lift (eq. 1) ----------------------------------------------------------
// g[d][l] = sum_i W[d][i] vals[i][l] for the 64 terms of row block rb and the
// kNewtonDB coefficients d0..; Wl holds W as limbs [i][d][3].
constexpr int kNewtonDB = 2;  // two coefficients per lane: enough waves to fill the device at t = 10^4

__device__ __forceinline__ void newton_body(const zr_mod& M, uint32_t t, uint32_t D1, uint32_t rb, uint32_t d0,
                                            const uint64_t* __restrict__ vals, const uint32_t* __restrict__ Wl,
                                            uint64_t* __restrict__ g) {
  const uint32_t l0 = rb * 64 + (threadIdx.x & 63);
  const bool live = l0 < t;
  const uint32_t l = live ? l0 : t - 1;
  Acc6 acc[kNewtonDB];
#pragma unroll
  for (int e = 0; e < kNewtonDB; ++e) acc6_zero(acc[e]);
  // the kNewtonDB x 3 limbs of W[d0..][i] for the next i are fetched ahead
  uint32_t wc[3 * kNewtonDB], wn[3 * kNewtonDB];
#pragma unroll
  for (int e = 0; e < 3 * kNewtonDB; ++e) wc[e] = Wl[(size_t)d0 * 3 + e];
  for (uint32_t i0 = 0; i0 < D1; i0 += 8) {
    uint64_t vv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) vv[u] = i0 + u < D1 ? vals[(size_t)(i0 + u) * t + l] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t i = i0 + u;
      if (i >= D1) break;
      const uint32_t inext = i + 1 < D1 ? i + 1 : i;
#pragma unroll
      for (int e = 0; e < 3 * kNewtonDB; ++e) wn[e] = Wl[((size_t)inext * D1 + d0) * 3 + e];
      const uint32_t v0 = (uint32_t)vv[u], v1 = (uint32_t)(vv[u] >> 32);
#pragma unroll
      for (int e = 0; e < kNewtonDB; ++e)
        if (d0 + e < D1) acc6_mac(acc[e], v0, v1, wc[3 * e], wc[3 * e + 1], wc[3 * e + 2]);
#pragma unroll
      for (int e = 0; e < 3 * kNewtonDB; ++e) wc[e] = wn[e];
    }
  }
  if (!live) return;
#pragma unroll
  for (int e = 0; e < kNewtonDB; ++e)
    if (d0 + e < D1) g[(size_t)(d0 + e) * t + l] = acc6_reduce(M, acc[e]);
}

__device__ __forceinline__ uint32_t count_nz(uint32_t t, uint32_t D1, const uint64_t* __restrict__ g, uint32_t l) {
  uint32_t n = 0;
  for (uint32_t d = 0; d < D1; ++d) n += g[(size_t)d * t + l] != 0;
  return n;
}

// ---- skeleton expansion ------------------------------------------------------------
// Term (e_l, d) of a nonzero g[d][l] goes to position off[l] + (rank of d among
// the nonzero coefficients of term l): lexicographic order is kept.
__device__ __forceinline__ void expand_body(const zr_mod& M, uint32_t t, uint32_t kvar, uint32_t nvars, uint32_t l,
                                            uint32_t d, const uint16_t* __restrict__ exps_old, size_t ld_old,
                                            const uint64_t* __restrict__ mono_old, const uint64_t* __restrict__ g,
                                            uint32_t off_l, const uint64_t* __restrict__ ypow,
                                            const uint64_t* __restrict__ ypowp, uint16_t* __restrict__ exps_new,
                                            uint64_t* __restrict__ coef_new, uint64_t* __restrict__ mono_new,
                                            size_t ld_new) {
  const uint64_t c = g[(size_t)d * t + l];
  if (c == 0) return;
  uint32_t pos = off_l;
  for (uint32_t e = 0; e < d; ++e) pos += g[(size_t)e * t + l] != 0;
  for (uint32_t v = 0; v < nvars; ++v)
    exps_new[(size_t)v * ld_new + pos] = v == kvar ? (uint16_t)d : exps_old[(size_t)v * ld_old + l];
  coef_new[pos] = c;
  mono_new[pos] = zr_shoup(M, mono_old[l], ypow[d], ypowp[d]);
}

}  // namespace zr

namespace zr {

// Host launcher of the product-tree convolution, compiled with the
// latency-aware scheduler (kernels_ilp.hip).
void launch_master_conv(hipStream_t s, const zr_mod& M, uint32_t t, uint32_t half, uint32_t IC, uint32_t nic,
                        const uint64_t* cur, const uint4* limbs, uint64_t* part, uint64_t* nxt, uint4* limbs_nxt);

}  // namespace zr
