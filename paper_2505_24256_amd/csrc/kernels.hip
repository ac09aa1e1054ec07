// gfx950 kernels of the polynomial Zippel path: master polynomial, the fused
// transposed Vandermonde solve, Newton lift, skeleton expansion, probes.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/zippel.h"
#include "field.hpp"
#include "kernels.hpp"
#include "kernels_dev.hpp"

namespace zr {

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

static uint32_t dots_waves_per_cu(uint32_t RT);
static uint32_t dots_pc_blocks_per_cu(uint32_t RT, uint32_t ntile, bool uneven);

// Variant of the dot-product pass: one wave per tile (0) or the
// producer/consumer form (1, the default; systems of at most kPcMinR
// right-hand sides still take one wave per tile); see zr_solve_variant.
constexpr int kDefaultDotsVariant = 1;
static std::atomic<int> g_dots_variant{kDefaultDotsVariant};
static bool dots_pc_enabled() { return g_dots_variant.load() == 1; }
bool vsolve_uses_pc() { return dots_pc_enabled(); }

// Widest tile of the one-wave-per-tile pass: 16 right-hand sides keep two
// waves per SIMD (20 would drop to one).
constexpr uint32_t kPlanRT = 16;

// Packed rows of one chunk of the producer/consumer pass, at most (bytes):
// under half of an XCD's 4 MiB L2.
constexpr uint64_t kChunkRowBytes = 7ull << 18;
// Partial dot-product sums of one solve (Sd R t words), at most (bytes): more
// chunks than fit take the slots in turn over several launches.
constexpr uint64_t kSpartBytes = 4ull << 30;
// Per-chunk state of one solve (chain values, start values and partials of
// delta, 3 S t words), at most (bytes); beyond it chunks grow longer, which
// changes only the speed.  At R = 40 the chunks keep their L2 size up to
// t = 2*10^6 or so (17 GB of state there); with a 4 GiB bound, t = 2*10^6 ran
// in 89 chunks of 11 MB of rows at 17.4 TOP/s against 19.5 at t = 10^6.
constexpr uint64_t kChunkStateBytes = 16ull << 30;

// Tile widths of the producer/consumer pass.  Waves 1..7 of a workgroup take
// tiles 0..6 and sit on SIMD (1 + k) mod 4, and the CU's two workgroups are
// placed alike: tile 3 shares SIMD 0 with the producer, tiles (0, 4), (1, 5)
// and (2, 6) share SIMDs 1, 2 and 3, and the busiest SIMD paces the barriers.
// With seven consumers the widths may differ from RT by one (at most
// kPcUnevenMax) so that the loads, counted in consumer values per step (the
// producer's step, about 22 vector instructions, is worth about 3.6 values,
// 7.1 with its Horner sum), are as even as the sum allows; R = 40: 7 for
// tile 3 and 6 + 5 on each other SIMD against 6 everywhere (t = 10^5: 90.0 ->
// 87.9 ms, 5*10^5: 4% faster).  With the producer's step counted as 4.4 and
// 8.7 values (its cost before its Shoup product lost five instructions), R = 37
// took 6, 6, 5, 5, 5, 5, 5 and ran 1.7% slower than with 5, 5, 5, 7, 5, 5, 5.
static void pc_widths_search(uint32_t R, uint32_t RT, bool dchain, uint32_t tw[7]) {
  const double prod = dchain ? 3.6 : 7.1;
  auto cost = [&](const uint32_t* w) {
    double c = prod + w[3];
    for (uint32_t k = 0; k < 3; ++k) c = std::max(c, (double)(w[k] + w[k + 4]));
    return c;
  };
  uint32_t best[7], w[7];
  for (uint32_t k = 0; k < 7; ++k) best[k] = RT;
  double bc = cost(best);
  uint32_t bsum = 7 * RT;
  for (uint32_t code = 0; code < 2187; ++code) {  // 3^7 choices of RT - 1, RT, RT + 1
    uint32_t x = code, sum = 0;
    for (uint32_t k = 0; k < 7; ++k, x /= 3) sum += (w[k] = RT - 1 + x % 3);
    if (sum < R) continue;
    const double c = cost(w);
    if (c < bc - 1e-9 || (c < bc + 1e-9 && sum < bsum)) {
      bc = c;
      bsum = sum;
      for (uint32_t k = 0; k < 7; ++k) best[k] = w[k];
    }
  }
  for (uint32_t k = 0; k < 7; ++k) tw[k] = best[k];
}

static void pc_widths(uint32_t R, uint32_t ntile, uint32_t RT, bool dchain, uint32_t tw[8]) {
  for (uint32_t k = 0; k < 8; ++k) tw[k] = k < ntile ? RT : 0;
  if (ntile != kPcMaxTiles || RT < 2 || RT + 1 > kPcUnevenMax || R > kPcMaxR) return;
  // the search once per (R, dchain), at the first plan (static initialisation
  // is thread-safe)
  struct Table {
    uint8_t w[kPcMaxR + 1][2][7];
  };
  static const Table T = [] {
    Table t{};
    for (uint32_t r = 1; r <= kPcMaxR; ++r)
      for (uint32_t d = 0; d < 2; ++d) {
        const uint32_t rt = cdiv(r, kPcMaxTiles);
        uint32_t x[7];
        for (uint32_t k = 0; k < 7; ++k) x[k] = rt;
        if (rt >= 2 && rt + 1 <= kPcUnevenMax) pc_widths_search(r, rt, d != 0, x);
        for (uint32_t k = 0; k < 7; ++k) t.w[r][d][k] = (uint8_t)x[k];
      }
    return t;
  }();
  if (cdiv(R, kPcMaxTiles) != RT) return;
  for (uint32_t k = 0; k < 7; ++k) tw[k] = T.w[R][dchain ? 1 : 0][k];
}

// true when the plan's producer/consumer tiles are not all RT wide
static bool plan_uneven(const VsolvePlan& P) {
  bool u = false;
  for (uint32_t k = 0; k < P.ntile && k < 8; ++k) u |= P.tw[k] != P.RT;
  return u;
}

VsolvePlan vsolve_plan(uint32_t t, uint32_t R, uint32_t num_cus) {
  VsolvePlan P;
  P.t = t;
  P.R = R;
  const uint32_t row_blocks = std::max<uint32_t>(1, cdiv(t, 64));
  // Above kPcMinR right-hand sides the chain runs once per row block in a
  // producer wave (k_vs_dots_pc) and consumer waves take tiles of at most
  // kPcRT; the unit of the launch is then a workgroup of 1 + ntile waves, a
  // multiple of four (pc_tiles_for).
  // More than kPcMaxR right-hand sides go through the pass in ng groups of
  // nearly equal size, which share the chain values, start values and
  // inverses of the solve.
  P.ng = 1;
  P.Rg = R;
  if (R > kPcMaxR && dots_pc_enabled()) {
    P.ng = cdiv(R, kPcMaxR);
    P.Rg = cdiv(R, P.ng);
  }
  P.pc = (P.Rg > kPcMinR && pc_tiles_for(P.Rg) && dots_pc_enabled()) ? 1 : 0;
  if (P.pc) {
    P.ntile = pc_tiles_for(P.Rg);
    P.RT = cdiv(P.Rg, P.ntile);
  } else {
    P.ng = 1;
    P.Rg = R;
    P.ntile = R == 0 ? 1 : cdiv(R, kPlanRT);
    P.RT = R == 0 ? 1 : cdiv(R, P.ntile);
  }
  // 32-bit words per packed row: the producer/consumer pass reads only the
  // limbs (pc_ldv); the one-wave-per-tile pass also reads M_r, in 64-byte groups
  P.ldv = P.pc ? pc_ldv(P.RT) : (3 * P.RT + 2 + 15) & ~15u;
  // delta from the chain pass instead of a Horner sum in the producer where the
  // producer's SIMD sets the pace: seven consumers of at most seven values.
  // At R = 40 (seven of six) the pass ran 12% faster without the producer's
  // Horner (t = 5*10^5: 2.46 -> 2.15 s, for 0.26 s more chain pass); at R = 30
  // (three of ten) and R = 56 (seven of eight) 1-2%, less than the chain pass
  // adds.
  P.dchain = P.pc && P.ntile == kPcMaxTiles && P.RT <= 7 ? 1 : 0;
  pc_widths(P.Rg, P.ntile, P.RT, P.dchain, P.tw);
  if (P.pc) {
    // the uneven kernel carries the bodies of the neighbouring widths; where
    // their registers cost a resident workgroup per CU, keep even tiles
    // (R = 31 and 33, RT = 5: three workgroups per CU against two, and the
    // uneven split ran 8-13% slower)
    if (plan_uneven(P) && dots_pc_blocks_per_cu(P.RT, P.ntile, true) < dots_pc_blocks_per_cu(P.RT, P.ntile, false))
      for (uint32_t k = 0; k < P.ntile; ++k) P.tw[k] = P.RT;
  }
  uint32_t row_words = 0;  // one step's packed rows over all tiles
  if (P.pc)
    for (uint32_t k = 0; k < P.ntile; ++k) row_words += pc_ldv(P.tw[k]);
  else
    row_words = P.ntile * P.ldv;
  P.vt32 = (size_t)row_words * t;
  uint32_t S;
  if (P.pc) {
    const uint32_t slots = std::max<uint32_t>(1, num_cus) * dots_pc_blocks_per_cu(P.RT, P.ntile, plan_uneven(P));
    const uint32_t S0 = std::max<uint32_t>(1, cdiv(4ull * slots, (uint64_t)row_blocks));
    // chunk state (chain values, start values, partials of delta: 3 S t words)
    // within kChunkStateBytes; partial sums (Sd R t words) within kSpartBytes,
    // the chunks taking Sd slots in turn, one launch per Sd chunks
    const uint32_t s_cap = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(4096, kChunkStateBytes / (24ull * t)));
    const uint32_t sd_max = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(4096, kSpartBytes / (8ull * std::max<uint32_t>(P.Rg, 1) * t)));
    auto slots_for = [&](uint32_t s) { return cdiv(s, cdiv(s, sd_max)); };
    // The workgroups resident on one XCD work through the same chunk and share
    // its packed rows in that XCD's L2 while the chunk's rows fit in it with
    // room to spare, so chunks hold at most kChunkRowBytes of rows.  At R = 40,
    // t = 5*10^5 the pass took 2.70 s with 26 chunks (19 231 steps, 9.7 MB of
    // rows), 2.58 s with 64, and 2.43 s from 128 chunks (3 906 steps, 2.0 MB)
    // up; 32-word rows (3.5 MB a chunk at 128 chunks) took 2.51 s.  From
    // there, among chunk counts up to a quarter more (at least 32), take the
    // one whose launches waste the least in their last round of `slots` equal
    // workgroups, counting that every chunk but the last also costs a chain
    // pass of about 1/64 of its dot-product pass.
    const uint64_t row_bytes = 4ull * row_words;
    const uint32_t l2_steps = (uint32_t)std::max<uint64_t>(64, kChunkRowBytes / row_bytes);
    const uint32_t s_lo = std::min(s_cap, std::max<uint32_t>(S0 - S0 / 4, cdiv(t, l2_steps)));
    const uint32_t s_hi = std::max<uint32_t>({32u, S0 + S0 / 4, s_lo + s_lo / 4});
    S = std::max<uint32_t>(1, s_lo);
    double best = 1e30;
    for (uint32_t s = std::max<uint32_t>(1, s_lo); s <= s_hi && s <= s_cap; ++s) {
      const uint32_t sd = slots_for(s);
      uint64_t rounds = 0;
      for (uint32_t c0 = 0; c0 < s; c0 += sd)
        rounds += ((uint64_t)row_blocks * std::min(sd, s - c0) + slots - 1) / slots;
      const double cost =
          (double)(rounds * slots) / ((double)row_blocks * s) * (1.0 + (s - 1.0) / s / 64.0);
      if (cost < best) {
        best = cost;
        S = s;
      }
    }
  } else {
    const uint32_t slots = std::max<uint32_t>(1, num_cus) * dots_waves_per_cu(P.RT);
    S = std::max<uint32_t>(1, cdiv(4ull * slots, (uint64_t)row_blocks * P.ntile));
  }
  S = std::min<uint32_t>(S, std::max<uint32_t>(1, t / 128));
  if (!P.pc) S = std::min<uint32_t>(S, 256);
  P.L = std::max<uint32_t>(1, cdiv(t, S));
  P.S = std::max<uint32_t>(1, cdiv(t, P.L));
  P.Sd = P.S;
  if (P.pc) {
    const uint32_t sd_max =
        (uint32_t)std::max<uint64_t>(1, kSpartBytes / (8ull * std::max<uint32_t>(P.Rg, 1) * std::max<uint32_t>(t, 1)));
    P.Sd = cdiv(P.S, cdiv(P.S, sd_max));
  }
  return P;
}

// workspace layout (64-bit words): right-hand sides VT (vt32 32-bit words: per tile [t][row]) |
//                   mono_p [t] | Bc [S][t] | qstart [S][t] | mL [t] |
//                   spart [Sd][Rg][t] | dpart [S][t] | winv [2t] | CL [t][6] (32-bit)
static size_t vsolve_rhs_words(const VsolvePlan& P) { return (P.vt32 + 1) / 2; }

size_t vsolve_workspace_words(const VsolvePlan& P) {
  const size_t t = P.t, S = P.S;
  return vsolve_rhs_words(P) + t + 2 * S * t + t + P.Sd * (size_t)P.Rg * t + S * t + 2 * t + 3 * t + 64;
}

// Packed right-hand sides [ntile][t][ldv], Shoup constants of the monomials
// and the coefficients r M_r of m M'(m).
__global__ void k_pack(uint32_t t, uint32_t R, uint32_t RT, uint32_t ntile, uint32_t ldv,
                       const uint64_t* __restrict__ rhs, size_t ld_rhs, const uint64_t* __restrict__ Mc,
                       uint32_t* __restrict__ VT, const uint64_t* __restrict__ mono, uint64_t* __restrict__ mono_p,
                       uint32_t* __restrict__ CL, zr_mod M) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)ntile * t * ldv;
  if (idx < total) VT[idx] = pack_word(idx, t, R, RT, ldv, rhs, ld_rhs, Mc);
  if (idx < t) {
    mono_p[idx] = zr_shoup_pre(M, mono[idx]);
    const uint64_t v = Mc[idx], d = zr_mul(M, idx % M.p, v);
    uint32_t* w = CL + idx * kChainW;
    w[0] = (uint32_t)(v & 0x3FFFFF);
    w[1] = (uint32_t)((v >> 22) & 0x3FFFFF);
    w[2] = (uint32_t)(v >> 44);
    w[3] = (uint32_t)(d & 0x3FFFFF);
    w[4] = (uint32_t)((d >> 22) & 0x3FFFFF);
    w[5] = (uint32_t)(d >> 44);
  }
}

// Packed rows of the producer/consumer tiles (blockIdx.y = tile), widths tw.
__global__ void k_pack_pc(VsArgs a, const uint64_t* __restrict__ rhs, size_t ld_rhs, uint32_t* __restrict__ VT) {
  const uint32_t tile = blockIdx.y;
  uint32_t j0 = 0, off = 0, w = 0;
#pragma unroll
  for (uint32_t k = 0; k < kPcMaxTiles; ++k) {
    if (k < tile) {
      j0 += a.tw[k];
      off += pc_ldv(a.tw[k]);
    }
    if (k == tile) w = a.tw[k];
  }
  const uint32_t ldv = pc_ldv(w);
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (size_t)a.t * ldv)
    VT[(size_t)off * a.t + idx] =
        pack_word_pc((uint32_t)(idx / ldv), (uint32_t)(idx % ldv), a.R, w, j0, rhs, ld_rhs);
}

// Chain values B_c (WB, the chunks c < S-1) and partials D_c of m M'(m) (WD):
// B and D for the chunks c < S-1 and D alone for the last one when delta
// comes from this pass, else B alone.  One kernel per stream set, so that each
// is compiled for its own registers.
template <bool WB, bool WD>
__global__ void __launch_bounds__(256) k_vs_chain(VsArgs a) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < a.t) vs_chain_cl<WB, WD>(a, l, WB ? blockIdx.y : a.S - 1);
}

__global__ void k_vs_scan(VsArgs a, uint64_t* __restrict__ qstart, uint64_t* __restrict__ mL_out) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < a.t) vs_scan_body(a, l, qstart, mL_out);
}

template <int RT>
__global__ void __launch_bounds__(64) k_vs_dots(VsArgs a) {
  vs_dots_body<RT>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// producer + one consumer wave per tile (64 * (1 + ntile) threads)
template <int RT, bool HORNER, bool UNEVEN>
__global__ void __launch_bounds__(64 * (1 + kPcMaxTiles)) k_vs_dots_pc(VsArgs a, uint32_t ntile, uint32_t c0) {
  __shared__ uint64_t qbuf[2][kQB][64];
  vs_dots_pc_body<RT, HORNER, UNEVEN>(a, blockIdx.x, c0 + blockIdx.y, ntile, qbuf);
}

__global__ void __launch_bounds__(kDeltaBlock) k_vs_delta(VsArgs a, const uint64_t* __restrict__ mLv,
                                                           uint64_t* __restrict__ winv, int32_t* __restrict__ status) {
  __shared__ uint64_t sh[kDeltaBlock / 64 + 1];
  vs_delta_block(a, blockIdx.x * kDeltaBlock + threadIdx.x, mLv, winv, status, sh);
}

__global__ void k_vs_scale(VsArgs a, const uint64_t* __restrict__ winv, uint64_t* __restrict__ out, size_t ld_out) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < a.t) vs_scale_body(a, l, blockIdx.y, winv, out, ld_out);
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

typedef void (*DotsPcKernel)(VsArgs, uint32_t, uint32_t);
template <int RT, bool H, bool U>
static DotsPcKernel dots_pc_ptr() {
  return k_vs_dots_pc<RT, H, U>;
}
template <bool H, bool U>
static DotsPcKernel dots_pc_pick(uint32_t RT) {
  static const DotsPcKernel table[kPcRT + 1] = {
      nullptr,                  dots_pc_ptr<1, H, U>(), dots_pc_ptr<2, H, U>(), dots_pc_ptr<3, H, U>(),
      dots_pc_ptr<4, H, U>(),   dots_pc_ptr<5, H, U>(), dots_pc_ptr<6, H, U>(), dots_pc_ptr<7, H, U>(),
      dots_pc_ptr<8, H, U>(),   dots_pc_ptr<9, H, U>(), dots_pc_ptr<10, H, U>()};
  return RT >= 1 && RT <= kPcRT ? table[RT] : nullptr;
}
// the producer/consumer pass for RT values per consumer, with the producer's
// Horner sum (horner) or without it (delta from the chain pass), with tiles of
// RT - 1 to RT + 1 values (uneven) or all of RT
static DotsPcKernel dots_pc_kernel(uint32_t RT, bool horner = true, bool uneven = false) {
  return horner ? (uneven ? dots_pc_pick<true, true>(RT) : dots_pc_pick<true, false>(RT))
                : (uneven ? dots_pc_pick<false, true>(RT) : dots_pc_pick<false, false>(RT));
}

// Workgroups of the producer/consumer pass resident per CU for ntile tiles
// (uneven: the kernel with the bodies of the neighbouring widths).
static uint32_t dots_pc_blocks_per_cu(uint32_t RT, uint32_t ntile, bool uneven) {
  static int cache[2][kPcRT + 1][kPcMaxTiles + 1] = {{{0}}};
  if (RT < 1 || RT > kPcRT || ntile < 1 || ntile > kPcMaxTiles) return 2;
  int& c = cache[uneven ? 1 : 0][RT][ntile];
  if (!c) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, dots_pc_kernel(RT, true, uneven), 64 * (1 + ntile), 0) !=
            hipSuccess ||
        nb <= 0)
      nb = 2;
    c = nb;
  }
  return (uint32_t)c;
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
  uint64_t* mono_p = VT + vsolve_rhs_words(P);
  uint64_t* Bc = mono_p + t;
  uint64_t* qstart = Bc + S * t;
  uint64_t* mL = qstart + S * t;
  uint64_t* spart = mL + t;
  uint64_t* dpart = spart + P.Sd * (size_t)P.Rg * t;
  uint64_t* winv = dpart + S * t;
  uint32_t* CL = (uint32_t*)(winv + 2 * t);
  VsArgs a;
  a.M = M;
  a.t = P.t;
  a.L = P.L;
  a.S = P.S;
  a.Sd = P.Sd;
  a.R = P.R;
  a.ldv = P.ldv;
  for (uint32_t k = 0; k < 8; ++k) a.tw[k] = (uint8_t)P.tw[k];
  a.mono = mono;
  a.mono_p = mono_p;
  a.Mc = Mc;
  a.VT = VT;
  a.qstart = S > 1 ? qstart : nullptr;
  a.Bc = Bc;
  a.spart = spart;
  a.CL = CL;
  // per-chunk partials of delta: D_c from the chain pass, or the Horner sums
  // of the dot-product pass
  a.hpart = P.dchain ? nullptr : dpart;
  a.dpart = P.dchain ? dpart : nullptr;
  // right-hand-side groups in turn; the chain values and start values (before
  // the first group's dot products) and the inverses (after them, from the
  // Horner partials) are the same for all and made once
  for (uint32_t g = 0, r0 = 0; g < P.ng; ++g) {
    const uint32_t Rg = P.R / P.ng + (g < P.R % P.ng ? 1 : 0);
    a.R = Rg;
    {
      TimedLaunch tl("vs_pack", s);
      if (P.pc) {
        uint32_t wmax = 0;
        for (uint32_t k = 0; k < P.ntile; ++k) wmax = std::max(wmax, P.tw[k]);
        hipLaunchKernelGGL(k_pack_pc, dim3(cdiv((size_t)t * pc_ldv(wmax), 256), P.ntile), dim3(256), 0, s, a,
                           rhs + (size_t)r0 * ld_rhs, ld_rhs, (uint32_t*)VT);
      }
      // the one-wave-per-tile rows (ldv words with M_r), Shoup constants and chain limbs
      const size_t total = std::max<size_t>(P.pc ? 0 : P.ntile * t * P.ldv, t);  // 32-bit words
      hipLaunchKernelGGL(k_pack, dim3(cdiv(total, 256)), dim3(256), 0, s, P.t, Rg, P.RT, P.pc ? 0 : P.ntile, P.ldv,
                         rhs + (size_t)r0 * ld_rhs, ld_rhs, Mc, (uint32_t*)VT, mono, mono_p, CL, M);
    }
    if (g == 0) {
      {
        TimedLaunch tl("vs_chain", s);
        if (P.dchain) {
          if (S > 1) hipLaunchKernelGGL((k_vs_chain<true, true>), dim3(cdiv(t, 256), P.S - 1), dim3(256), 0, s, a);
          hipLaunchKernelGGL((k_vs_chain<false, true>), dim3(cdiv(t, 256)), dim3(256), 0, s, a);
        } else if (S > 1) {
          hipLaunchKernelGGL((k_vs_chain<true, false>), dim3(cdiv(t, 256), P.S - 1), dim3(256), 0, s, a);
        }
      }
      if (S > 1) {
        TimedLaunch tl("vs_scan", s);
        hipLaunchKernelGGL(k_vs_scan, dim3(cdiv(t, 256)), dim3(256), 0, s, a, qstart, mL);
      }
    }
    if (P.pc) {
      DotsPcKernel kp = dots_pc_kernel(P.RT, !P.dchain, plan_uneven(P));
      if (!kp) return hipErrorInvalidValue;
      // chunks in launches of Sd (one partial-sum slot each), in order
      for (uint32_t c0 = 0; c0 < P.S; c0 += P.Sd) {
        TimedLaunch tl("vs_dots", s);
        hipLaunchKernelGGL(kp, dim3(cdiv(t, 64), std::min<uint32_t>(P.Sd, P.S - c0)), dim3(64 * (1 + P.ntile)), 0,
                           s, a, P.ntile, c0);
      }
    } else {
      DotsKernel kd = dots_kernel(P.RT);
      if (!kd) return hipErrorInvalidValue;
      TimedLaunch tl("vs_dots", s);
      hipLaunchKernelGGL(kd, dim3(cdiv(t, 64), P.S, P.ntile), dim3(64), 0, s, a);
    }
    {
      TimedLaunch tl("vs_finish", s);
      if (g == 0)
        hipLaunchKernelGGL(k_vs_delta, dim3(cdiv(t, kDeltaBlock)), dim3(kDeltaBlock), 0, s, a, mL, winv, status);
      hipLaunchKernelGGL(k_vs_scale, dim3(cdiv(t, 256), Rg), dim3(256), 0, s, a, winv, out + (size_t)r0 * ld_out,
                         ld_out);
    }
    r0 += Rg;
  }
  return hipGetLastError();
}

// ============================================================================
// Master polynomial by a product tree.  Level s multiplies pairs of monic
// factors of degree <= 2^s; every level stores the non-leading coefficients
// of all its factors in one array of length t (factor [a, b) at [a, b)).
// ============================================================================

__global__ void __launch_bounds__(64) k_master_small(zr_mod M, uint32_t t, const uint64_t* __restrict__ mono,
                                                     uint64_t* __restrict__ out, uint4* __restrict__ limbs) {
  __shared__ uint64_t buf[128];
  master_small_body(M, t, blockIdx.x * 64, mono, out, limbs, buf);
}

__global__ void k_master_sum(zr_mod M, uint32_t t, uint32_t half, uint32_t nic, const uint64_t* __restrict__ cur,
                             const uint64_t* __restrict__ part, uint64_t* __restrict__ nxt,
                             uint4* __restrict__ limbs_nxt) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < t) master_sum_body(M, t, half, nic, g, cur, part, t, nxt, limbs_nxt);
}

size_t master_tmp_words(uint32_t t) {
  // t for the ping-pong level array, two limb arrays of t + 16 entries (two
  // words each) and the chunk partials of the largest levels
  uint32_t nic_max = 1;
  for (uint32_t half = 64; half < t; half *= 2) nic_max = std::max(nic_max, cdiv(half, conv_ic(half, cdiv(t, 64))));
  return (size_t)t + 1 + 4 * ((size_t)t + 16) + (nic_max > 1 ? (size_t)nic_max * t : 0) + 64;
}

hipError_t master_poly(const zr_mod& M, uint32_t t, const uint64_t* mono, uint64_t* Mc, uint64_t* tmp,
                       hipStream_t s) {
  if (t == 0) return hipSuccess;
  TimedLaunch tl("master", s);
  uint32_t big = 0;  // levels with half >= 64
  for (uint32_t half = 64; half < t; half *= 2) ++big;
  const size_t t2 = ((size_t)t + 1) & ~(size_t)1;  // keep the limb arrays 16-byte aligned
  uint4* limbs[2] = {(uint4*)(tmp + t2), (uint4*)(tmp + t2 + 2 * ((size_t)t + 16))};
  uint64_t* part = tmp + t2 + 4 * ((size_t)t + 16);
  uint64_t* bufs[2] = {Mc, tmp};
  // the level written last must be Mc: the small kernel writes bufs[big % 2]
  uint32_t w = big % 2;
  hipLaunchKernelGGL(k_master_small, dim3(cdiv(t, 64)), dim3(64), 0, s, M, t, mono, bufs[w], limbs[w]);
  for (uint32_t half = 64; half < t; half *= 2) {
    const uint32_t r = w;
    w ^= 1;
    const uint32_t IC = conv_ic(half, cdiv(t, 64));
    const uint32_t nic = cdiv(half, IC);
    launch_master_conv(s, M, t, half, IC, nic, bufs[r], limbs[r], part, bufs[w], limbs[w]);
    if (nic > 1)
      hipLaunchKernelGGL(k_master_sum, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, half, nic, bufs[r], part, bufs[w],
                         limbs[w]);
  }
  return hipGetLastError();
}

// ============================================================================
// Newton lift (eq. 1).  Interpolating values a_0..a_D at fixed nodes into
// monomial coefficients is linear: g = W a with W the inverse of the
// Vandermonde matrix of the nodes, the same for every term of a stage (built
// from the Lagrange basis polynomials of the nodes); here each lane owns one
// term and kNewtonDB output coefficients, and the products are the carry-free
// 64x64-bit sums of the solve.
// Wl: [i][d][3] 22-bit limbs of W[d][i].
// ============================================================================

__global__ void __launch_bounds__(64) k_newton_mat(zr_mod M, uint32_t t, uint32_t D1,
                                                   const uint64_t* __restrict__ vals,
                                                   const uint32_t* __restrict__ Wl, uint64_t* __restrict__ g) {
  newton_body(M, t, D1, blockIdx.x, blockIdx.y * kNewtonDB, vals, Wl, g);
}

__global__ void k_count_nz(uint32_t t, uint32_t D1, const uint64_t* __restrict__ g, uint32_t* __restrict__ cnt) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < t) cnt[l] = count_nz(t, D1, g, l);
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
  if (l < t)
    expand_body(M, t, kvar, nvars, l, blockIdx.y, exps_old, t, mono_old, g, off[l], ypow, ypowp, exps_new, coef_new,
                mono_new, ld_new);
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
// Monomial values of a skeleton from per-variable power tables.
// ============================================================================

__global__ void k_mono(zr_mod M, uint32_t t, uint32_t nv, const uint16_t* __restrict__ exps, uint32_t ld,
                       const uint64_t* __restrict__ tabs, MonoTables T, uint64_t* __restrict__ mono) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= t) return;
  uint64_t m = 1 % M.p;
  for (uint32_t v = 0; v < nv; ++v) m = zr_mul(M, m, tabs[T.off[v] + exps[(size_t)v * ld + l]]);
  mono[l] = m;
}

hipError_t mono_values(const zr_mod& M, uint32_t t, uint32_t nv, const uint16_t* exps, uint32_t ld,
                       const uint64_t* tabs, const MonoTables& T, uint64_t* mono, hipStream_t s) {
  if (t == 0) return hipSuccess;
  if (nv > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mono, dim3(cdiv(t, 256)), dim3(256), 0, s, M, t, nv, exps, ld, tabs, T, mono);
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
  int on = 0;  // 0 off, 1 every named launch, 2 only the solve's dot-product pass ("vs_dots")
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
  if (!g_timing.on || (g_timing.on == 2 && strcmp(n, "vs_dots") != 0)) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;  // not in graphs
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
zr_status zr_solve_variant(int variant) {
  if (variant != 0 && variant != 1) return ZR_EINVAL;
  zr::g_dots_variant.store(variant);
  return ZR_OK;
}

void zr_timing_enable(int on) {
  std::lock_guard<std::mutex> g(zr::g_timing.mu);
  zr::g_timing.on = on == 2 ? 2 : (on != 0 ? 1 : 0);
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
