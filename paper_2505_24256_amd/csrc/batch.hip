// Batched forms of the polynomial-path kernels (§1, §2.2): the same device
// bodies as the one-system launches, with the block index mapped to
// (system, local block) by a binary search over a prefix array of per-system
// block counts, and the dominant solve pass as a persistent kernel over a
// work queue.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>
#include <vector>

#include "batch.hpp"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"
#include "kernels_dev.hpp"

namespace zr {

// largest s < n with prefix[s] <= b (prefix[0] = 0, prefix[n] > b); b is
// wave-uniform, so the search runs on scalar loads
__device__ __forceinline__ uint32_t seg_find(const uint32_t* __restrict__ prefix, uint32_t n, uint32_t b) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- solve ---------------------------------------------------------------------------

struct BSolve {
  VsArgs a;
  uint64_t* qstart;
  uint64_t* mL;
  uint64_t* winv;
  const uint64_t* rhs;  // [R][t]
  uint64_t* out;        // [R][t]
  int32_t* status;
  uint32_t RT, ntile;
  // offsets of VT, spart and hpart in the batch's shared packed-row and
  // partial-sum allocations (the persistent pass addresses them from the two
  // base pointers, so its packed-row loads provably never alias its stores)
  uint64_t vt_off, sp_off, hp_off;
};

__global__ void k_b_pack(uint32_t n, const uint32_t* __restrict__ prefix, const BSolve* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BSolve& b = sys[s];
  const size_t idx = (size_t)(blockIdx.x - prefix[s]) * blockDim.x + threadIdx.x;
  const uint32_t t = b.a.t;
  if (idx < (size_t)b.ntile * t * b.a.ldv)
    ((uint32_t*)b.a.VT)[idx] = pack_word(idx, t, b.a.R, b.RT, b.a.ldv, b.rhs, t, b.a.Mc);
  if (idx < t) ((uint64_t*)b.a.mono_p)[idx] = zr_shoup_pre(b.a.M, b.a.mono[idx]);
}

__global__ void __launch_bounds__(256) k_b_chain(uint32_t n, const uint32_t* __restrict__ prefix,
                                                 const BSolve* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const VsArgs& a = sys[s].a;
  const uint32_t lb = blockIdx.x - prefix[s], nrb = cdiv(a.t, 256);
  const uint32_t l = (lb % nrb) * 256 + threadIdx.x;
  if (l < a.t) vs_chain_body(a, l, lb / nrb);
}

__global__ void k_b_scan(uint32_t n, const uint32_t* __restrict__ prefix, const BSolve* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BSolve& b = sys[s];
  const uint32_t l = (blockIdx.x - prefix[s]) * blockDim.x + threadIdx.x;
  if (l < b.a.t) vs_scan_body(b.a, l, b.qstart, b.mL);
}

// Persistent pass 2: each wave pops (system, row block, chunk, tile) items
// until the queue is empty.  head must be zero at launch.
template <int RT>
__global__ void __launch_bounds__(64) k_b_dots(const BSolve* __restrict__ sys, const uint4* __restrict__ items,
                                               uint32_t nitems, uint32_t* __restrict__ head,
                                               const uint64_t* __restrict__ vt_base, uint64_t* __restrict__ part_base) {
  for (;;) {
    uint32_t it = 0;
    if (threadIdx.x == 0) it = atomicAdd(head, 1u);
    it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
    if (it >= nitems) break;
    const uint4 w = items[it];
    const BSolve& b = sys[w.x];
    VsArgs a = b.a;
    a.VT = vt_base + b.vt_off;
    a.spart = part_base + b.sp_off;
    a.hpart = part_base + b.hp_off;
    vs_dots_body<RT>(a, w.y, w.z, w.w);
  }
}

// Persistent producer/consumer pass: each workgroup (a producer wave and one
// consumer wave per tile, as many as the class's widest system needs) pops
// (system, row block, chunk) items until the queue is empty; every wave of the
// workgroup takes the same item, so all of them reach the same barriers and
// the same exit.  head must be zero at launch.
template <int RT>
__global__ void __launch_bounds__(64 * (1 + kPcMaxTiles))
    k_b_dots_pc(const BSolve* __restrict__ sys, const uint4* __restrict__ items, uint32_t nitems,
                uint32_t* __restrict__ head, const uint64_t* __restrict__ vt_base, uint64_t* __restrict__ part_base) {
  __shared__ uint64_t qbuf[2][kQB][64];
  __shared__ uint32_t next;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(head, 1u);
    __syncthreads();
    const uint32_t it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();  // every wave has read next before it is overwritten
    if (it >= nitems) break;
    const uint4 w = items[it];
    const BSolve& b = sys[w.x];
    VsArgs a = b.a;
    a.VT = vt_base + b.vt_off;
    a.spart = part_base + b.sp_off;
    a.hpart = part_base + b.hp_off;
    vs_dots_pc_body<RT, true>(a, w.y, w.z, b.ntile, qbuf);
  }
}

// one block of kDeltaBlock rows of one system (the row segments are counted
// in blocks of 256 = kDeltaBlock rows)
__global__ void __launch_bounds__(kDeltaBlock) k_b_delta(uint32_t n, const uint32_t* __restrict__ prefix,
                                                         const BSolve* __restrict__ sys) {
  __shared__ uint64_t sh[kDeltaBlock / 64 + 1];
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BSolve& b = sys[s];
  const uint32_t l = (blockIdx.x - prefix[s]) * kDeltaBlock + threadIdx.x;
  vs_delta_block(b.a, l, b.mL, b.winv, b.status, sh);
}

__global__ void k_b_scale(uint32_t n, const uint32_t* __restrict__ prefix, const BSolve* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BSolve& b = sys[s];
  const uint32_t lb = blockIdx.x - prefix[s], nrb = cdiv(b.a.t, 256);
  const uint32_t l = (lb % nrb) * 256 + threadIdx.x;
  if (l < b.a.t) vs_scale_body(b.a, l, lb / nrb, b.winv, b.out, b.a.t);
}

// Small systems packed into shared wavefronts: lane i of item w handles row
// lanes[w][i] = (system, row) or nothing; the systems of one item have similar
// sizes.  No chunking: each lane runs its row's whole chain, loading its
// system's packed rows with vector loads.
template <int RT>
__global__ void __launch_bounds__(64) k_b_dots_packed(const BSolve* __restrict__ sys, const uint2* __restrict__ lanes,
                                                      uint32_t tile) {
  constexpr int LDV = (3 * RT + 2 + 15) & ~15;
  const uint2 me = lanes[(size_t)blockIdx.x * 64 + threadIdx.x];
  const bool live = me.x != 0xFFFFFFFFu;
  const uint32_t s = live ? me.x : lanes[(size_t)blockIdx.x * 64].x;
  const VsArgs& a = sys[s].a;
  const zr_mod M = a.M;
  const uint32_t t = a.t;
  const uint32_t l = live ? me.y : 0;
  const uint64_t m = a.mono[l], mp = a.mono_p[l];
  const bool horner = tile == 0;
  Acc6 acc[RT];
#pragma unroll
  for (int j = 0; j < RT; ++j) acc6_zero(acc[j]);
  uint64_t q = 1 % M.p, h = 0;
  const uint32_t* rows = (const uint32_t*)a.VT + (size_t)tile * t * LDV;
  const bool has_tile = tile < sys[s].ntile;
  const uint32_t steps = (live && has_tile) ? t : 0;
  // longest chain in the wave
  uint32_t tmax = steps;
  for (int o = 32; o >= 1; o >>= 1) tmax = max(tmax, (uint32_t)__shfl_xor((int)tmax, o));
  uint32_t since = 0;
  for (uint32_t u = 0; u < tmax; ++u) {
    if (u < steps) {
      const uint32_t* row = rows + (size_t)(t - 1 - u) * LDV;
      const uint32_t q0 = (uint32_t)q, q1 = (uint32_t)(q >> 32);
#pragma unroll
      for (int jj = 0; jj < RT; ++jj) acc6_mac(acc[jj], q0, q1, row[3 * jj], row[3 * jj + 1], row[3 * jj + 2]);
      const uint64_t Mr = ((uint64_t)row[3 * RT + 1] << 32) | row[3 * RT];
      if (horner) h = zr_add(M, zr_shoup(M, h, m, mp), q);
      q = zr_add(M, zr_shoup(M, q, m, mp), Mr);
      if (++since == kFold) {
#pragma unroll
        for (int j = 0; j < RT; ++j) acc6_fold(acc[j], M);
        since = 0;
      }
    }
  }
  if (!live || !has_tile) return;
  const uint32_t j0 = tile * RT;
#pragma unroll
  for (int j = 0; j < RT; ++j)
    if (j0 + j < a.R) a.spart[(size_t)(j0 + j) * t + l] = acc6_reduce(M, acc[j]);
  if (horner) a.hpart[l] = h;
}

// ---- master polynomial -------------------------------------------------------------

struct BMaster {
  uint32_t t, big;
  const uint64_t* mono;
  uint64_t* buf[2];  // buf[0] = Mc
  uint4* limbs[2];
  uint64_t* part;    // [nic][t]
};

__global__ void __launch_bounds__(64) k_b_master_small(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix,
                                                       const BMaster* __restrict__ sys) {
  __shared__ uint64_t buf[128];
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BMaster& b = sys[s];
  master_small_body(M, b.t, (blockIdx.x - prefix[s]) * 64, b.mono, b.buf[0], b.limbs[0], buf);
}

// level with factors of degree `half` (>= 64), chunks of IC: reads buffer r, writes r ^ 1
__global__ void __launch_bounds__(64) k_b_master_conv(zr_mod M, uint32_t half, uint32_t IC, uint32_t r, uint32_t n,
                                                      const uint32_t* __restrict__ prefix,
                                                      const BMaster* __restrict__ sys) {
  extern __shared__ uint64_t win[];  // 64 + IC + 8 words
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BMaster& b = sys[s];
  const uint32_t nic = cdiv(half, IC);
  const uint32_t lb = blockIdx.x - prefix[s], nrb = cdiv(b.t, 64);
  master_conv_body(M, b.t, half, IC, nic, (lb % nrb) * 64, lb / nrb, b.buf[r], b.limbs[r], b.part, b.t, b.buf[r ^ 1],
                   b.limbs[r ^ 1], win);
}

// the same for factors of degree half >= 128 with four waves (256
// coefficients) sharing each window
__global__ void __launch_bounds__(256) k_b_master_conv4(zr_mod M, uint32_t half, uint32_t IC, uint32_t r, uint32_t n,
                                                        const uint32_t* __restrict__ prefix,
                                                        const BMaster* __restrict__ sys) {
  extern __shared__ uint64_t win[];  // 256 + IC + 8 words
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BMaster& b = sys[s];
  const uint32_t nic = cdiv(half, IC);
  const uint32_t lb = blockIdx.x - prefix[s], nrb = cdiv(b.t, 256);
  master_conv_body<4>(M, b.t, half, IC, nic, (lb % nrb) * 256, lb / nrb, b.buf[r], b.limbs[r], b.part, b.t,
                      b.buf[r ^ 1], b.limbs[r ^ 1], win);
}

__global__ void k_b_master_sum(zr_mod M, uint32_t half, uint32_t nic, uint32_t r, uint32_t n,
                               const uint32_t* __restrict__ prefix, const BMaster* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BMaster& b = sys[s];
  const uint32_t g = (blockIdx.x - prefix[s]) * blockDim.x + threadIdx.x;
  if (g < b.t) master_sum_body(M, b.t, half, nic, g, b.buf[r], b.part, b.t, b.buf[r ^ 1], b.limbs[r ^ 1]);
}

// systems whose last level landed in buf[1]: copy to Mc
__global__ void k_b_master_fix(uint32_t n, const uint32_t* __restrict__ prefix, const BMaster* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BMaster& b = sys[s];
  const uint32_t g = (blockIdx.x - prefix[s]) * blockDim.x + threadIdx.x;
  if (g < b.t) b.buf[0][g] = b.buf[1][g];
}

// ---- Newton matrices -------------------------------------------------------------------

struct BConsts {
  uint32_t D1;
  uint32_t xoff;  // first node in the concatenated node array
  uint64_t yk;
  uint32_t* Wl;
  uint64_t* ypow;
};

// One workgroup per node set.  P(z) = prod_j (z - x_j) is built in LDS one
// factor at a time; column i of W = V^{-1} holds the coefficients of the
// Lagrange basis polynomial P(z) / ((z - x_i) P'(x_i)), obtained by synthetic
// division (the same closed form as the solve, at the size of the node set).
constexpr uint32_t kMaxD1 = 1024;

__global__ void __launch_bounds__(256) k_b_consts(zr_mod M, const BConsts* __restrict__ sys,
                                                 const uint64_t* __restrict__ nodes) {
  __shared__ uint64_t P[kMaxD1 + 1];
  const BConsts& b = sys[blockIdx.x];
  const uint32_t D1 = b.D1;
  const uint64_t* X = nodes + b.xoff;
  for (uint32_t d = threadIdx.x; d <= D1; d += blockDim.x) P[d] = d == 0 ? 1 % M.p : 0;
  __syncthreads();
  for (uint32_t j = 0; j < D1; ++j) {
    // P <- P (z - x_j): new P_d = P_{d-1} - x_j P_d, for d = j+1 .. 0
    const uint64_t nx = zr_neg(M, X[j]);
    uint64_t v[kMaxD1 / 256 + 1];
    uint32_t cnt = 0;
    for (uint32_t d = threadIdx.x; d <= j + 1; d += blockDim.x, ++cnt)
      v[cnt] = zr_add(M, d ? P[d - 1] : 0, zr_mul(M, nx, P[d]));
    __syncthreads();
    cnt = 0;
    for (uint32_t d = threadIdx.x; d <= j + 1; d += blockDim.x, ++cnt) P[d] = v[cnt];
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < D1; i += blockDim.x) {
    const uint64_t x = X[i];
    // q_{D1-1} = 1, q_{r-1} = P_r + x q_r; den = sum_r q_r x^r (Horner)
    uint64_t q = 1 % M.p, den = 0;
    const uint64_t xp = zr_shoup_pre(M, x);
    for (uint32_t r = D1 - 1;; --r) {
      den = zr_add(M, zr_shoup(M, den, x, xp), q);
      if (r == 0) break;
      q = zr_add(M, P[r], zr_shoup(M, q, x, xp));
    }
    const uint64_t inv = zr_inv(M, den);
    q = 1 % M.p;
    for (uint32_t r = D1 - 1;; --r) {
      const uint64_t w = zr_mul(M, q, inv);
      uint32_t* o = b.Wl + ((size_t)i * D1 + r) * 3;
      o[0] = (uint32_t)(w & 0x3FFFFF);
      o[1] = (uint32_t)((w >> 22) & 0x3FFFFF);
      o[2] = (uint32_t)(w >> 44);
      if (r == 0) break;
      q = zr_add(M, P[r], zr_shoup(M, q, x, xp));
    }
  }
  if (threadIdx.x == 0) {
    uint64_t a = 1 % M.p;
    const uint64_t ykp = zr_shoup_pre(M, b.yk);
    for (uint32_t d = 0; d < D1; ++d) {
      b.ypow[d] = a;
      b.ypow[D1 + d] = zr_shoup_pre(M, a);
      a = zr_shoup(M, a, b.yk, ykp);
    }
  }
  // padding read by the Newton kernel's look-ahead
  for (uint32_t e = threadIdx.x; e < 24; e += blockDim.x) b.Wl[(size_t)D1 * D1 * 3 + e] = 0;
}

// ---- Newton lift and expansion --------------------------------------------------------

struct BLift {
  uint32_t t, D1, kvar, nvars;
  uint32_t base;  // offset of the system's terms in the concatenated counts
  uint32_t pad;
  const int32_t* status;  // may be null
  const uint64_t* vals;
  const uint32_t* Wl;
  const uint64_t* ypow;
  uint64_t* g;
  const uint16_t* exps_old;
  const uint64_t* mono_old;
  uint16_t* exps_new;
  uint64_t* coef_new;
  uint64_t* mono_new;
  uint32_t ld_new;
};

__global__ void __launch_bounds__(64) k_b_newton(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix,
                                                 const BLift* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BLift& b = sys[s];
  const uint32_t lb = blockIdx.x - prefix[s], nrb = cdiv(b.t, 64);
  newton_body(M, b.t, b.D1, lb % nrb, (lb / nrb) * kNewtonDB, b.vals, b.Wl, b.g);
}

__global__ void k_b_count(uint32_t n, const uint32_t* __restrict__ prefix, const BLift* __restrict__ sys,
                          uint32_t* __restrict__ cnt) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BLift& b = sys[s];
  const uint32_t l = (blockIdx.x - prefix[s]) * blockDim.x + threadIdx.x;
  if (l < b.t) cnt[b.base + l] = count_nz(b.t, b.D1, b.g, l);
}

// new skeleton sizes and the systems' statuses, side by side for one read-back
__global__ void k_b_totals(uint32_t n, const BLift* __restrict__ sys, const uint32_t* __restrict__ off,
                           int32_t* __restrict__ out) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) {
    out[s] = (int32_t)(off[sys[s].base + sys[s].t] - off[sys[s].base]);
    out[n + s] = sys[s].status ? *sys[s].status : 0;
  }
}

__global__ void k_b_expand(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix, const BLift* __restrict__ sys,
                           const uint32_t* __restrict__ off) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BLift& b = sys[s];
  const uint32_t lb = blockIdx.x - prefix[s], nrb = cdiv(b.t, 256);
  const uint32_t l = (lb % nrb) * 256 + threadIdx.x;
  if (l < b.t)
    expand_body(M, b.t, b.kvar, b.nvars, l, lb / nrb, b.exps_old, b.t, b.mono_old, b.g,
                off[b.base + l] - off[b.base], b.ypow, b.ypow + b.D1, b.exps_new, b.coef_new, b.mono_new, b.ld_new);
}

// ---- evaluation at points --------------------------------------------------------------

struct BEval {
  uint32_t t, nvars, ldtab, pad;
  const uint16_t* exps;
  const uint64_t* coef;
  const uint64_t* tab;
  uint64_t* result;
};

__global__ void __launch_bounds__(256) k_b_eval(zr_mod M, const BEval* __restrict__ sys) {
  __shared__ uint64_t sh[256];
  const BEval& b = sys[blockIdx.x];
  uint64_t acc = 0;
  for (uint32_t l = threadIdx.x; l < b.t; l += blockDim.x) {
    uint64_t v = b.coef[l];
    for (uint32_t j = 0; j < b.nvars; ++j) v = zr_mul(M, v, b.tab[(size_t)j * b.ldtab + b.exps[(size_t)j * b.t + l]]);
    acc = zr_add(M, acc, v);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = zr_add(M, sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *b.result = sh[0];
}

// ---- copies ------------------------------------------------------------------------------

struct BCopy {
  const uint16_t* src;
  uint16_t* dst;
  uint64_t n;  // 16-bit units
};

__global__ void k_b_copy16(uint32_t n, const uint32_t* __restrict__ prefix, const BCopy* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const BCopy& b = sys[s];
  const uint64_t i = (uint64_t)(blockIdx.x - prefix[s]) * blockDim.x + threadIdx.x;
  if (i < b.n) b.dst[i] = b.src[i];
}

// seeded values in [lo, p): SplitMix64 output i of stream `seed`, reduced mod (p - lo)
__global__ void k_rand_mod(uint64_t* __restrict__ x, size_t n, uint64_t seed, uint64_t p, uint64_t lo) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  x[i] = lo + z % (p - lo);
}

// ===========================================================================================
// host side
// ===========================================================================================

// Pinned staging buffers, each reused once the copy that last read it has
// completed (checked without blocking), so uploads never wait on the stream.
namespace {
struct Staging {
  char* p = nullptr;
  size_t n = 0;
  hipEvent_t done = nullptr;
};
std::mutex g_staging_mu;
std::vector<Staging>& staging_pool() {
  static std::vector<Staging>* v = new std::vector<Staging>();  // kept until exit
  return *v;
}
}  // namespace

char* Blob::upload(DevArena& A, hipStream_t s) {
  if (bytes_.empty()) return nullptr;
  Staging* st = nullptr;
  {
    std::lock_guard<std::mutex> g(g_staging_mu);
    for (auto& x : staging_pool())
      if (x.n >= bytes_.size() && hipEventQuery(x.done) == hipSuccess) {
        st = &x;
        break;
      }
    if (!st) {
      Staging x;
      x.n = std::max<size_t>(bytes_.size(), 1 << 20);
      void* p = nullptr;
      check(hipHostMalloc(&p, x.n, hipHostMallocDefault));
      x.p = (char*)p;
      check(hipEventCreateWithFlags(&x.done, hipEventDisableTiming));
      staging_pool().push_back(x);
      st = &staging_pool().back();
    }
    memcpy(st->p, bytes_.data(), bytes_.size());
    char* d = A.alloc<char>(bytes_.size());
    check(hipMemcpyAsync(d, st->p, bytes_.size(), hipMemcpyHostToDevice, s));
    check(hipEventRecord(st->done, s));
    return d;
  }
}

// ---- graphs --------------------------------------------------------------------------
namespace {
std::mutex g_graph_mu;
bool g_graphs = false;
struct Retired {
  hipStream_t s;
  hipGraph_t g;
  hipGraphExec_t ge;
};
std::vector<Retired>& retired() {
  static std::vector<Retired>* v = new std::vector<Retired>();
  return *v;
}
}  // namespace

// one non-blocking stream per device, default priority, for graph capture
hipStream_t capture_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {nullptr};
  int dev = 0;
  check(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(ZR_EDEVICE);
  std::lock_guard<std::mutex> l(mu);
  if (!streams[dev]) check(hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking));
  return streams[dev];
}

bool graphs_enabled() {
  std::lock_guard<std::mutex> l(g_graph_mu);
  return g_graphs;
}
void set_graphs(bool on) {
  std::lock_guard<std::mutex> l(g_graph_mu);
  g_graphs = on;
}
// a launched graph is destroyed once its stream has been synchronised
void retire_graph(hipStream_t s, hipGraph_t g, hipGraphExec_t ge) {
  std::lock_guard<std::mutex> l(g_graph_mu);
  retired().push_back(Retired{s, g, ge});
}
void release_graphs(hipStream_t s) {
  std::lock_guard<std::mutex> l(g_graph_mu);
  auto& v = retired();
  for (size_t i = 0; i < v.size();) {
    if (v[i].s == s) {
      (void)hipGraphExecDestroy(v[i].ge);
      (void)hipGraphDestroy(v[i].g);
      v[i] = v.back();
      v.pop_back();
    } else {
      ++i;
    }
  }
}

uint32_t band_of(uint32_t t) {
  if (t < 64) return 0;
  if (t < 256) return 1;
  if (t < 1024) return 2;
  if (t < 4096) return 3;
  return 4;
}

Tuning& tuning() {
  static Tuning T = [] {
    Tuning x;
    for (int b = 0; b < kBands; ++b) x.band[b] = BandTuning{b == 0 ? 1u : 0u, 512u};
    x.tuned = 0;
    return x;
  }();
  return T;
}

void autotune(const zr_mod& M, hipStream_t s) {
  struct Case {
    uint32_t nsys, tlo, thi;
  };
  // synthetic systems of each band, R = 30 right-hand sides
  const Case cases[kBands] = {{1024, 8, 63}, {256, 64, 255}, {64, 256, 1023}, {16, 1024, 4095}, {4, 4096, 8192}};
  const uint32_t R = 30;
  Tuning& T = tuning();
  hipEvent_t e0, e1;
  check(hipEventCreate(&e0));
  check(hipEventCreate(&e1));
  uint64_t lcg = 12345;
  for (int b = 0; b < kBands; ++b) {
    DevArena A(s);
    const Case& c = cases[b];
    std::vector<uint32_t> ts(c.nsys);
    size_t tt = 0;
    for (auto& t : ts) {
      lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
      t = c.tlo + (uint32_t)((lcg >> 33) % (c.thi - c.tlo + 1));
      tt += t;
    }
    uint64_t* mono = A.alloc<uint64_t>(tt);
    uint64_t* rhs = A.alloc<uint64_t>(tt * R);
    int32_t* st = A.alloc<int32_t>(c.nsys);
    hipLaunchKernelGGL(k_rand_mod, dim3(cdiv(tt, 256)), dim3(256), 0, s, mono, tt, 1000 + b, M.p, 2);
    std::vector<SolveJob> jobs;
    size_t o = 0;
    for (uint32_t i = 0; i < c.nsys; ++i) {
      jobs.push_back(SolveJob{ts[i], R, mono + o, rhs + o * R, st + i});
      o += ts[i];
    }
    std::vector<BandTuning> cand;
    if (b == 0) cand = {{1, 512}, {0, 512}};
    else cand = {{0, 128}, {0, 512}, {0, 2048}, {0, 1u << 30}};
    float best = 1e30f;
    BandTuning pick = T.band[b];
    for (const BandTuning& x : cand) {
      T.band[b] = x;
      float ms = 0;
      for (int rep = 0; rep < 2; ++rep) {
        hipLaunchKernelGGL(k_rand_mod, dim3(cdiv(tt * R, 256)), dim3(256), 0, s, rhs, tt * R, 2000 + b, M.p, 0);
        check(hipEventRecord(e0, s));
        batched_solve(M, jobs, s);
        check(hipEventRecord(e1, s));
        check(hipEventSynchronize(e1));
        check(hipEventElapsedTime(&ms, e0, e1));
      }
      if (ms < best) {
        best = ms;
        pick = x;
      }
    }
    T.band[b] = pick;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  T.tuned = 1;
}

namespace {

typedef void (*BDotsKernel)(const BSolve*, const uint4*, uint32_t, uint32_t*, const uint64_t*, uint64_t*);
typedef void (*BPackedKernel)(const BSolve*, const uint2*, uint32_t);

template <int RT>
BDotsKernel bdots_ptr() {
  return k_b_dots<RT>;
}
template <int RT>
BPackedKernel bpacked_ptr() {
  return k_b_dots_packed<RT>;
}

BDotsKernel bdots_kernel(uint32_t RT) {
  static const BDotsKernel table[kMaxRT + 1] = {
      nullptr,         bdots_ptr<1>(),  bdots_ptr<2>(),  bdots_ptr<3>(),  bdots_ptr<4>(),  bdots_ptr<5>(),
      bdots_ptr<6>(),  bdots_ptr<7>(),  bdots_ptr<8>(),  bdots_ptr<9>(),  bdots_ptr<10>(), bdots_ptr<11>(),
      bdots_ptr<12>(), bdots_ptr<13>(), bdots_ptr<14>(), bdots_ptr<15>(), bdots_ptr<16>(), bdots_ptr<17>(),
      bdots_ptr<18>(), bdots_ptr<19>(), bdots_ptr<20>()};
  return RT >= 1 && RT <= kMaxRT ? table[RT] : nullptr;
}

typedef void (*BDotsPcKernel)(const BSolve*, const uint4*, uint32_t, uint32_t*, const uint64_t*, uint64_t*);
template <int RT>
BDotsPcKernel bdots_pc_ptr() {
  return k_b_dots_pc<RT>;
}
BDotsPcKernel bdots_pc_kernel(uint32_t RT) {
  static const BDotsPcKernel table[kPcRT + 1] = {
      nullptr,           bdots_pc_ptr<1>(), bdots_pc_ptr<2>(), bdots_pc_ptr<3>(), bdots_pc_ptr<4>(), bdots_pc_ptr<5>(),
      bdots_pc_ptr<6>(), bdots_pc_ptr<7>(), bdots_pc_ptr<8>(), bdots_pc_ptr<9>(), bdots_pc_ptr<10>()};
  return RT >= 1 && RT <= kPcRT ? table[RT] : nullptr;
}

// Workgroups of the persistent producer/consumer pass resident per CU with
// 1 + ntile waves each.
uint32_t bdots_pc_blocks_per_cu(uint32_t RT, uint32_t ntile) {
  static int cache[kPcRT + 1][kPcMaxTiles + 1] = {{0}};
  if (RT < 1 || RT > kPcRT || ntile < 1 || ntile > kPcMaxTiles) return 1;
  if (!cache[RT][ntile]) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bdots_pc_kernel(RT), 64 * (1 + ntile), 0) != hipSuccess ||
        nb <= 0)
      nb = 1;
    cache[RT][ntile] = nb;
  }
  return (uint32_t)cache[RT][ntile];
}

BPackedKernel bpacked_kernel(uint32_t RT) {
  static const BPackedKernel table[kMaxRT + 1] = {
      nullptr,           bpacked_ptr<1>(),  bpacked_ptr<2>(),  bpacked_ptr<3>(),  bpacked_ptr<4>(),
      bpacked_ptr<5>(),  bpacked_ptr<6>(),  bpacked_ptr<7>(),  bpacked_ptr<8>(),  bpacked_ptr<9>(),
      bpacked_ptr<10>(), bpacked_ptr<11>(), bpacked_ptr<12>(), bpacked_ptr<13>(), bpacked_ptr<14>(),
      bpacked_ptr<15>(), bpacked_ptr<16>(), bpacked_ptr<17>(), bpacked_ptr<18>(), bpacked_ptr<19>(),
      bpacked_ptr<20>()};
  return RT >= 1 && RT <= kMaxRT ? table[RT] : nullptr;
}

uint32_t bdots_waves_per_cu(uint32_t RT) {
  static int cache[kMaxRT + 1] = {0};
  if (RT < 1 || RT > kMaxRT) return 8;
  if (!cache[RT]) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bdots_kernel(RT), 64, 0) != hipSuccess || nb <= 0) nb = 8;
    cache[RT] = nb;
  }
  return (uint32_t)cache[RT];
}

// prefix array of per-system block counts
struct Segs {
  std::vector<uint32_t> prefix{0};
  void add(uint64_t blocks) { prefix.push_back(prefix.back() + (uint32_t)blocks); }
  uint32_t total() const { return prefix.back(); }
  uint32_t n() const { return (uint32_t)prefix.size() - 1; }
};

}  // namespace

// Per-system plan inside a batch: tile split of R as in the one-system solve;
// chunking only where a system's own work would otherwise outlast the
// batch's share per wave slot.
struct BPlan {
  uint32_t t, R, RT, ntile, ldv, L, S, packed, pc;
};

// With the producer/consumer pass selected, systems of more than kPcMinR
// right-hand sides that are not packed take its tiling (pc_tiles_for: at most
// kPcRT per consumer wave, workgroups of a multiple of four waves) and go to
// the persistent producer/consumer queue.
static BPlan bplan(uint32_t t, uint32_t R, double cap, const Tuning& T) {
  BPlan P;
  P.t = t;
  P.R = R;
  const BandTuning& bt = T.band[band_of(t)];
  P.packed = bt.packed && t < 64 ? 1 : 0;
  P.pc = !P.packed && R > kPcMinR && pc_tiles_for(R) && vsolve_uses_pc() ? 1 : 0;
  P.ntile = P.pc ? pc_tiles_for(R) : cdiv(R, kMaxRT);
  P.RT = cdiv(R, P.ntile);
  P.ldv = P.pc ? pc_ldv(P.RT) : (3 * P.RT + 2 + 15) & ~15u;  // as in the one-system solve
  uint32_t S = 1;
  if (!P.packed) {
    const double item = 64.0 * t * P.RT;  // one wave's work for an unsplit row block
    if (item > cap) S = (uint32_t)std::ceil(item / cap);
    S = std::min<uint32_t>(S, std::max<uint32_t>(1, t / std::max<uint32_t>(bt.min_chunk, 1)));
    S = std::min<uint32_t>(S, 256);
  }
  P.L = std::max<uint32_t>(1, cdiv(t, S));
  P.S = std::max<uint32_t>(1, cdiv(t, P.L));
  return P;
}

void batched_solve(const zr_mod& M, const std::vector<SolveJob>& jobs_in, hipStream_t s) {
  std::vector<SolveJob> jobs;
  for (const auto& j : jobs_in) {
    if (!j.t || !j.R) continue;
    jobs.push_back(j);
  }
  if (jobs.empty()) return;
  const uint32_t n = (uint32_t)jobs.size();
  const Tuning& T = tuning();
  const uint32_t cus = device_cus();
  // per-item work cap: a quarter of the batch's work per wave slot
  double total = 0;
  for (const auto& j : jobs) total += (double)j.t * j.t * j.R;
  const double cap = std::max(64.0 * 128 * kMaxRT, total / (4.0 * cus * 8));
  std::vector<BPlan> plan(n);
  for (uint32_t i = 0; i < n; ++i) plan[i] = bplan(jobs[i].t, jobs[i].R, cap, T);

  DevArena A(s);
  // ---- master polynomials; chunk length of each product-tree level from the
  // level's total number of row blocks
  std::vector<BMaster> bm(n);
  Segs small, fix;
  uint32_t halfmax = 0;
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t h = 64; h < jobs[i].t; h *= 2) halfmax = std::max(halfmax, h);
  std::vector<uint32_t> level_ic;
  for (uint32_t h = 64; h <= halfmax; h *= 2) {
    uint64_t blocks = 0;
    for (uint32_t i = 0; i < n; ++i)
      if (jobs[i].t > h) blocks += cdiv(jobs[i].t, 64);
    level_ic.push_back(conv_ic(h, blocks));
  }
  for (uint32_t i = 0; i < n; ++i) {
    const uint32_t t = jobs[i].t;
    uint32_t big = 0;
    for (uint32_t h = 64; h < t; h *= 2) ++big;
    BMaster& b = bm[i];
    b.t = t;
    b.big = big;
    b.mono = jobs[i].mono;
    b.buf[0] = A.alloc<uint64_t>(t);
    b.buf[1] = A.alloc<uint64_t>(t);
    b.limbs[0] = A.alloc<uint4>(t + 16);
    b.limbs[1] = A.alloc<uint4>(t + 16);
    uint32_t nic_max = 1;
    for (uint32_t h = 64, lv = 0; h < t; h *= 2, ++lv) nic_max = std::max(nic_max, cdiv(h, level_ic[lv]));
    b.part = nic_max > 1 ? A.alloc<uint64_t>((size_t)nic_max * t) : nullptr;
    small.add(cdiv(t, 64));
    fix.add(big % 2 ? cdiv(t, 256) : 0);
  }
  // ---- solve workspaces; packed rows and partial sums of all systems in two
  // shared allocations
  std::vector<BSolve> bs(n);
  Segs pack, chain, scan, rows, scale;
  size_t vt_words = 0, part_words = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const BPlan& P = plan[i];
    const size_t t = P.t, S = P.S;
    bs[i].vt_off = vt_words;
    vt_words += (P.ntile * t * (P.ldv / 2) + 7) & ~(size_t)7;
    bs[i].sp_off = part_words;
    part_words += S * (size_t)P.R * t;
    bs[i].hp_off = part_words;
    part_words += S * t;
  }
  uint64_t* vt_base = A.alloc<uint64_t>(std::max<size_t>(vt_words, 1));
  uint64_t* part_base = A.alloc<uint64_t>(std::max<size_t>(part_words, 1));
  for (uint32_t i = 0; i < n; ++i) {
    const BPlan& P = plan[i];
    const size_t t = P.t, S = P.S;
    BSolve& b = bs[i];
    b.a.M = M;
    b.a.t = P.t;
    b.a.L = P.L;
    b.a.S = P.S;
    b.a.Sd = P.S;
    b.a.R = P.R;
    b.a.ldv = P.ldv;
    for (uint32_t k = 0; k < 8; ++k) b.a.tw[k] = (uint8_t)(k < P.ntile ? P.RT : 0);  // uniform tiles
    b.a.mono = jobs[i].mono;
    b.a.VT = vt_base + b.vt_off;
    b.a.mono_p = A.alloc<uint64_t>(t);
    b.a.Mc = bm[i].buf[0];
    b.a.Bc = S > 1 ? A.alloc<uint64_t>((S - 1) * t) : nullptr;
    b.qstart = S > 1 ? A.alloc<uint64_t>(S * t) : nullptr;
    b.a.qstart = b.qstart;
    b.mL = S > 1 ? A.alloc<uint64_t>(t) : nullptr;
    b.a.spart = part_base + b.sp_off;
    b.a.hpart = part_base + b.hp_off;
    b.winv = A.alloc<uint64_t>(2 * t);
    b.rhs = jobs[i].rhs;
    b.out = jobs[i].rhs;
    b.status = jobs[i].status;
    b.RT = P.RT;
    b.ntile = P.ntile;
    pack.add(cdiv(std::max<size_t>(P.ntile * t * P.ldv, t), 256));
    chain.add(S > 1 ? (size_t)cdiv(t, 256) * (S - 1) : 0);
    scan.add(S > 1 ? cdiv(t, 256) : 0);
    rows.add(cdiv(t, kDeltaBlock));
    scale.add((size_t)cdiv(t, 256) * P.R);
  }
  // conv levels
  std::vector<Segs> conv, csum;
  for (uint32_t h = 64, lv = 0; h <= halfmax; h *= 2, ++lv) {
    Segs c, su;
    const uint32_t nic = cdiv(h, level_ic[lv]);
    for (uint32_t i = 0; i < n; ++i) {
      const uint32_t t = jobs[i].t;
      c.add(t > h ? (size_t)cdiv(t, h >= 128 ? 256 : 64) * nic : 0);  // workgroups of 4 or 1 waves
      su.add(t > h && nic > 1 ? cdiv(t, 256) : 0);
    }
    conv.push_back(c);
    csum.push_back(su);
  }
  // work queues of the dots pass: wave-per-row-block items per RT class
  // (largest chunk first) and packed lane tables per RT class
  std::vector<std::vector<uint4>> items(kMaxRT + 1);
  std::vector<std::vector<uint32_t>> order(kMaxRT + 1);
  for (uint32_t i = 0; i < n; ++i) order[plan[i].RT].push_back(i);
  std::vector<std::vector<uint2>> lanes(kMaxRT + 1);
  std::vector<uint32_t> max_tiles(kMaxRT + 1, 0);
  std::vector<std::vector<uint4>> items_pc(kPcRT + 1);  // producer/consumer items per RT class
  std::vector<uint32_t> pc_tiles(kPcRT + 1, 0);         // consumer waves per workgroup of the class
  for (uint32_t RT = 1; RT <= kMaxRT; ++RT) {
    auto& ord = order[RT];
    std::stable_sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return plan[x].L > plan[y].L; });
    std::vector<uint32_t> pk;
    for (uint32_t i : ord) {
      const BPlan& P = plan[i];
      if (P.packed) {
        pk.push_back(i);
        max_tiles[RT] = std::max(max_tiles[RT], P.ntile);
        continue;
      }
      if (P.pc) {
        pc_tiles[RT] = std::max(pc_tiles[RT], P.ntile);
        for (uint32_t c = 0; c < P.S; ++c)
          for (uint32_t rb = 0; rb < cdiv(P.t, 64); ++rb) items_pc[RT].push_back(make_uint4(i, rb, c, 0));
        continue;
      }
      for (uint32_t c = 0; c < P.S; ++c)
        for (uint32_t tile = 0; tile < P.ntile; ++tile)
          for (uint32_t rb = 0; rb < cdiv(P.t, 64); ++rb) items[RT].push_back(make_uint4(i, rb, c, tile));
    }
    // packed: systems sorted by size, rows dealt to 64-lane groups without
    // splitting a system across groups
    std::sort(pk.begin(), pk.end(), [&](uint32_t x, uint32_t y) { return plan[x].t > plan[y].t; });
    std::vector<uint2>& ln = lanes[RT];
    uint32_t fill = 64;
    for (uint32_t i : pk) {
      const uint32_t t = plan[i].t;
      if (fill + t > 64) {
        ln.resize(ln.size() + 64, make_uint2(0xFFFFFFFFu, 0));
        fill = 0;
      }
      for (uint32_t r = 0; r < t; ++r) ln[ln.size() - 64 + fill + r] = make_uint2(i, r);
      fill += t;
    }
  }
  // ---- one upload of all descriptors and tables
  Blob blob;
  const size_t o_bm = blob.add(bm), o_bs = blob.add(bs);
  const size_t o_small = blob.add(small.prefix), o_fix = blob.add(fix.prefix);
  const size_t o_pack = blob.add(pack.prefix), o_chain = blob.add(chain.prefix), o_scan = blob.add(scan.prefix);
  const size_t o_rows = blob.add(rows.prefix), o_scale = blob.add(scale.prefix);
  std::vector<size_t> o_conv, o_csum;
  for (size_t i = 0; i < conv.size(); ++i) {
    o_conv.push_back(blob.add(conv[i].prefix));
    o_csum.push_back(blob.add(csum[i].prefix));
  }
  std::vector<size_t> o_items(kMaxRT + 1, 0), o_lanes(kMaxRT + 1, 0);
  for (uint32_t RT = 1; RT <= kMaxRT; ++RT) {
    if (!items[RT].empty()) o_items[RT] = blob.add(items[RT]);
    if (!lanes[RT].empty()) o_lanes[RT] = blob.add(lanes[RT]);
  }
  std::vector<size_t> o_items_pc(kPcRT + 1, 0);
  for (uint32_t RT = 1; RT <= kPcRT; ++RT)
    if (!items_pc[RT].empty()) o_items_pc[RT] = blob.add(items_pc[RT]);
  // queue heads: [0, kMaxRT] one-wave items, [kMaxRT + 1, kMaxRT + 1 + kPcRT] producer/consumer items
  std::vector<uint32_t> zeros(kMaxRT + 2 + kPcRT, 0);
  const size_t o_heads = blob.add(zeros);
  char* d = blob.upload(A, s);
  auto P32 = [&](size_t o) { return (const uint32_t*)(d + o); };
  const BMaster* d_bm = (const BMaster*)(d + o_bm);
  const BSolve* d_bs = (const BSolve*)(d + o_bs);
  uint32_t* d_heads = (uint32_t*)(d + o_heads);

  // the device-side sequence below (every input already resident) is recorded
  // as one graph and launched as one unit when graphs are on
  std::vector<uint32_t> grid(kMaxRT + 1, 0);  // persistent grid per class, queried before any capture
  for (uint32_t RT = 1; RT <= kMaxRT; ++RT)
    if (!items[RT].empty()) grid[RT] = std::min<uint32_t>((uint32_t)items[RT].size(), cus * bdots_waves_per_cu(RT));
  std::vector<uint32_t> grid_pc(kPcRT + 1, 0);
  for (uint32_t RT = 1; RT <= kPcRT; ++RT)
    if (!items_pc[RT].empty())
      grid_pc[RT] = std::min<uint32_t>((uint32_t)items_pc[RT].size(), cus * bdots_pc_blocks_per_cu(RT, pc_tiles[RT]));
  // (captured on a library stream, since the caller's may be the null stream,
  // which cannot be captured; the graph is then launched on the caller's)
  const bool graph = graphs_enabled();
  const hipStream_t ls = graph ? capture_stream() : s;
  if (graph) check(hipStreamBeginCapture(ls, hipStreamCaptureModeThreadLocal));
  {
    TimedLaunch tl("batch_master", ls);
    hipLaunchKernelGGL(k_b_master_small, dim3(small.total()), dim3(64), 0, ls, M, n, P32(o_small), d_bm);
    uint32_t r = 0;
    for (size_t lv = 0; lv < conv.size(); ++lv, r ^= 1) {
      const uint32_t h = 64u << lv, IC = level_ic[lv];
      if (conv[lv].total() && h >= 128)
        hipLaunchKernelGGL(k_b_master_conv4, dim3(conv[lv].total()), dim3(256), (256 + IC + 8) * 8, ls, M, h, IC, r,
                           n, P32(o_conv[lv]), d_bm);
      else if (conv[lv].total())
        hipLaunchKernelGGL(k_b_master_conv, dim3(conv[lv].total()), dim3(64), (64 + IC + 8) * 8, ls, M, h, IC, r, n,
                           P32(o_conv[lv]), d_bm);
      if (csum[lv].total())
        hipLaunchKernelGGL(k_b_master_sum, dim3(csum[lv].total()), dim3(256), 0, ls, M, h, cdiv(h, IC), r, n,
                           P32(o_csum[lv]), d_bm);
    }
    if (fix.total()) hipLaunchKernelGGL(k_b_master_fix, dim3(fix.total()), dim3(256), 0, ls, n, P32(o_fix), d_bm);
  }
  {
    TimedLaunch tl("batch_pack", ls);
    hipLaunchKernelGGL(k_b_pack, dim3(pack.total()), dim3(256), 0, ls, n, P32(o_pack), d_bs);
  }
  if (chain.total()) {
    TimedLaunch tl("batch_chain", ls);
    hipLaunchKernelGGL(k_b_chain, dim3(chain.total()), dim3(256), 0, ls, n, P32(o_chain), d_bs);
    hipLaunchKernelGGL(k_b_scan, dim3(scan.total()), dim3(256), 0, ls, n, P32(o_scan), d_bs);
  }
  {
    TimedLaunch tl("batch_dots", ls);
    for (uint32_t RT = 1; RT <= kPcRT; ++RT)
      if (!items_pc[RT].empty())
        hipLaunchKernelGGL(bdots_pc_kernel(RT), dim3(grid_pc[RT]), dim3(64 * (1 + pc_tiles[RT])), 0, ls, d_bs,
                           (const uint4*)(d + o_items_pc[RT]), (uint32_t)items_pc[RT].size(),
                           d_heads + kMaxRT + 1 + RT, (const uint64_t*)vt_base, part_base);
    for (uint32_t RT = 1; RT <= kMaxRT; ++RT) {
      if (!items[RT].empty()) {
        const uint32_t ni = (uint32_t)items[RT].size();
        hipLaunchKernelGGL(bdots_kernel(RT), dim3(grid[RT]), dim3(64), 0, ls, d_bs, (const uint4*)(d + o_items[RT]), ni,
                           d_heads + RT, (const uint64_t*)vt_base, part_base);
      }
      if (!lanes[RT].empty())
        for (uint32_t tile = 0; tile < max_tiles[RT]; ++tile)
          hipLaunchKernelGGL(bpacked_kernel(RT), dim3((uint32_t)(lanes[RT].size() / 64)), dim3(64), 0, ls, d_bs,
                             (const uint2*)(d + o_lanes[RT]), tile);
    }
  }
  {
    TimedLaunch tl("batch_finish", ls);
    hipLaunchKernelGGL(k_b_delta, dim3(rows.total()), dim3(kDeltaBlock), 0, ls, n, P32(o_rows), d_bs);
    hipLaunchKernelGGL(k_b_scale, dim3(scale.total()), dim3(256), 0, ls, n, P32(o_scale), d_bs);
  }
  if (graph) {
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(ls, &g);
    if (e != hipSuccess || !g) throw Error(ZR_EDEVICE);
    hipGraphExec_t ge = nullptr;
    if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      throw Error(ZR_EDEVICE);
    }
    check(hipGraphLaunch(ge, s));
    retire_graph(s, g, ge);
  }
  check(hipGetLastError());
  for (const auto& j : jobs) count_solve(j.t, j.R);
}

size_t newton_W_words(uint32_t D1) { return (size_t)D1 * D1 * 3 + 24; }

void batched_consts(const zr_mod& M, const std::vector<ConstsJob>& jobs, hipStream_t s) {
  if (jobs.empty()) return;
  DevArena A(s);
  std::vector<uint64_t> nodes;
  std::vector<size_t> off;
  for (const auto& j : jobs) {
    if (j.D1 == 0 || j.D1 > kMaxD1) throw Error(ZR_EINVAL);
    off.push_back(nodes.size());
    nodes.insert(nodes.end(), j.h_nodes, j.h_nodes + j.D1);
  }
  std::vector<BConsts> bc(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i)
    bc[i] = BConsts{jobs[i].D1, (uint32_t)off[i], jobs[i].yk, jobs[i].Wl, jobs[i].ypow};
  Blob b;
  const size_t o_nodes = b.add(nodes), o_bc = b.add(bc);
  char* d = b.upload(A, s);
  hipLaunchKernelGGL(k_b_consts, dim3((uint32_t)jobs.size()), dim3(256), 0, s, M, (const BConsts*)(d + o_bc),
                     (const uint64_t*)(d + o_nodes));
  check(hipGetLastError());
}

std::vector<int32_t> batched_lift(const zr_mod& M, const std::vector<LiftJob>& jobs, DevArena& keep, hipStream_t s) {
  const uint32_t n = (uint32_t)jobs.size();
  std::vector<int32_t> status(n, 0);
  if (n == 0) return status;
  DevArena A(s);
  std::vector<BLift> bl(n);
  Segs newton, rows;
  uint32_t base = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const LiftJob& j = jobs[i];
    const uint32_t t = j.old->t;
    BLift& b = bl[i];
    b.t = t;
    b.D1 = j.D1;
    b.kvar = j.kvar;
    b.nvars = j.old->nvars;
    b.base = base;
    b.pad = 0;
    b.status = j.d_status;
    b.vals = j.vals;
    b.Wl = j.Wl;
    b.ypow = j.ypow;
    b.g = A.alloc<uint64_t>((size_t)j.D1 * std::max<uint32_t>(t, 1));
    b.exps_old = j.old->exps;
    b.mono_old = j.old->mono;
    base += t;
    newton.add((size_t)cdiv(t, 64) * cdiv(j.D1, kNewtonDB));
    rows.add(cdiv(t, 256));
  }
  const uint32_t T = base;
  uint32_t* cnt = A.alloc<uint32_t>(std::max<uint32_t>(T, 1));
  uint32_t* off = A.alloc<uint32_t>((size_t)T + 1);
  uint32_t* tmp = A.alloc<uint32_t>(scan_tmp_words(T));
  int32_t* tot = A.alloc<int32_t>(2 * (size_t)n);
  Blob blob;
  const size_t o_bl = blob.add(bl), o_newton = blob.add(newton.prefix), o_rows = blob.add(rows.prefix);
  char* d = blob.upload(A, s);
  const BLift* d_bl = (const BLift*)(d + o_bl);
  {
    TimedLaunch tl("batch_newton", s);
    if (newton.total())
      hipLaunchKernelGGL(k_b_newton, dim3(newton.total()), dim3(64), 0, s, M, n, (const uint32_t*)(d + o_newton), d_bl);
    if (rows.total())
      hipLaunchKernelGGL(k_b_count, dim3(rows.total()), dim3(256), 0, s, n, (const uint32_t*)(d + o_rows), d_bl, cnt);
  }
  if (T == 0) check(fill_i32((int32_t*)off, 0, 1, s));
  else check(exclusive_scan(T, cnt, off, tmp, s));
  hipLaunchKernelGGL(k_b_totals, dim3(cdiv(n, 256)), dim3(256), 0, s, n, d_bl, off, tot);
  check(hipGetLastError());
  // one read-back: new sizes and statuses
  std::vector<int32_t> h(2 * (size_t)n);
  check(hipMemcpyAsync(h.data(), tot, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
  check(hipStreamSynchronize(s));
  release_graphs(s);
  // the new skeletons share one block of `keep`
  size_t words = 0;
  for (uint32_t i = 0; i < n; ++i) {
    const size_t tn = std::max<int32_t>(h[i], 1);
    words += 2 * ((tn + 31) & ~(size_t)31) + ((jobs[i].old->nvars * tn + 127) & ~(size_t)127) / 4;
  }
  uint64_t* blk = keep.alloc<uint64_t>(std::max<size_t>(words, 1));
  Segs expand;
  for (uint32_t i = 0; i < n; ++i) {
    const LiftJob& j = jobs[i];
    count_newton(j.old->t, j.D1);
    status[i] = h[n + i];
    const uint32_t tn = (uint32_t)h[i];
    const size_t tp = std::max<uint32_t>(tn, 1);
    Skeleton& o = *j.out;
    o.nvars = j.old->nvars;
    o.t = tn;
    o.coef = blk;
    o.mono = blk + ((tp + 31) & ~(size_t)31);
    o.exps = (uint16_t*)(o.mono + ((tp + 31) & ~(size_t)31));
    blk = (uint64_t*)o.exps + ((o.nvars * tp + 127) & ~(size_t)127) / 4;
    bl[i].exps_new = o.exps;
    bl[i].coef_new = o.coef;
    bl[i].mono_new = o.mono;
    bl[i].ld_new = (uint32_t)tp;
    expand.add(status[i] == 0 ? (size_t)cdiv(j.old->t, 256) * j.D1 : 0);
  }
  if (expand.total()) {
    Blob b2;
    const size_t o2 = b2.add(bl), o2p = b2.add(expand.prefix);
    char* d2 = b2.upload(A, s);
    TimedLaunch tl("batch_expand", s);
    hipLaunchKernelGGL(k_b_expand, dim3(expand.total()), dim3(256), 0, s, M, n, (const uint32_t*)(d2 + o2p),
                       (const BLift*)(d2 + o2), off);
    check(hipGetLastError());
  }
  return status;
}

void batched_copy(const std::vector<CopyJob>& jobs, hipStream_t s) {
  std::vector<BCopy> bc;
  Segs seg;
  for (const auto& j : jobs) {
    if (j.bytes % 2) throw Error(ZR_EINVAL);
    if (!j.bytes) continue;
    bc.push_back(BCopy{(const uint16_t*)j.src, (uint16_t*)j.dst, j.bytes / 2});
    seg.add(cdiv(j.bytes / 2, 256));
  }
  if (bc.empty()) return;
  DevArena A(s);
  Blob b;
  const size_t o = b.add(bc), op = b.add(seg.prefix);
  char* d = b.upload(A, s);
  hipLaunchKernelGGL(k_b_copy16, dim3(seg.total()), dim3(256), 0, s, seg.n(), (const uint32_t*)(d + op),
                     (const BCopy*)(d + o));
  check(hipGetLastError());
}

__global__ void k_b_exps_to_terms(uint32_t n, const uint32_t* __restrict__ prefix,
                                  const TransposeJob* __restrict__ sys) {
  const uint32_t s = seg_find(prefix, n, blockIdx.x);
  const TransposeJob& b = sys[s];
  const uint64_t i = (uint64_t)(blockIdx.x - prefix[s]) * blockDim.x + threadIdx.x;  // l * nvars + v
  if (i < (uint64_t)b.t * b.nvars) {
    const uint64_t l = i / b.nvars, v = i % b.nvars;
    b.dst[i] = b.src[v * b.t + l];
  }
}

void batched_exps_to_terms(const std::vector<TransposeJob>& jobs, hipStream_t s) {
  std::vector<TransposeJob> tj;
  Segs seg;
  for (const auto& j : jobs) {
    if (!j.t || !j.nvars) continue;
    tj.push_back(j);
    seg.add(cdiv((uint64_t)j.t * j.nvars, 256));
  }
  if (tj.empty()) return;
  DevArena A(s);
  Blob b;
  const size_t o = b.add(tj), op = b.add(seg.prefix);
  char* d = b.upload(A, s);
  hipLaunchKernelGGL(k_b_exps_to_terms, dim3(seg.total()), dim3(256), 0, s, seg.n(), (const uint32_t*)(d + op),
                     (const TransposeJob*)(d + o));
  check(hipGetLastError());
}

__global__ void k_b_powers(zr_mod M, uint32_t n, const PowJob* __restrict__ jobs) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PowJob& j = jobs[i];
  for (uint32_t v = 0; v < j.nv; ++v) {
    const uint64_t x = j.pt[v];
    uint64_t a = 1 % M.p;
    for (uint32_t d = 0; d < j.ld; ++d) {
      j.tab[(size_t)v * j.ld + d] = a;
      a = zr_mul(M, a, x);
    }
  }
}

void batched_power_tables(const zr_mod& M, const std::vector<PowJob>& jobs, hipStream_t s) {
  if (jobs.empty()) return;
  DevArena A(s);
  Blob b;
  const size_t o = b.add(jobs);
  char* d = b.upload(A, s);
  hipLaunchKernelGGL(k_b_powers, dim3(cdiv((uint32_t)jobs.size(), 64u)), dim3(64), 0, s, M, (uint32_t)jobs.size(),
                     (const PowJob*)(d + o));
  check(hipGetLastError());
}

void batched_eval(const zr_mod& M, const std::vector<EvalJob>& jobs, hipStream_t s) {
  if (jobs.empty()) return;
  DevArena A(s);
  std::vector<BEval> be(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) {
    const Skeleton& P = *jobs[i].poly;
    be[i] = BEval{P.t, P.nvars, jobs[i].ldtab, 0, P.exps, P.coef, jobs[i].tab, jobs[i].result};
  }
  Blob b;
  const size_t o = b.add(be);
  char* d = b.upload(A, s);
  hipLaunchKernelGGL(k_b_eval, dim3((uint32_t)jobs.size()), dim3(256), 0, s, M, (const BEval*)(d + o));
  check(hipGetLastError());
}

}  // namespace zr
