// Host driver of the Zippel reconstruction and the C ABI declared in zippel.h.
// The host runs the stage loop (one stage per variable, §1) and talks to the
// black box; every O(t^2) and O(t D^2) step runs in the gfx950 kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <stdexcept>
#include <vector>

#include "../../include/zippel.h"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"

namespace zr {

// ---------------------------------------------------------------------------
// device memory: stream-ordered allocations from the device's default pool,
// which keeps freed memory cached so repeated calls do not reach the driver.

static std::mutex g_pool_mu;
static std::vector<int> g_pool_ready;

static void ensure_pool(int dev) {
  std::lock_guard<std::mutex> g(g_pool_mu);
  if (std::find(g_pool_ready.begin(), g_pool_ready.end(), dev) != g_pool_ready.end()) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  g_pool_ready.push_back(dev);
}

DevArena::DevArena(hipStream_t st) : s(st) {
  int dev = 0;
  hipGetDevice(&dev);
  ensure_pool(dev);
}

DevArena::~DevArena() {
  for (void* p : ptrs) hipFreeAsync(p, s);
}

void* DevArena::raw(size_t bytes) {
  void* p = nullptr;
  bytes = std::max<size_t>(bytes, 256);
  bytes = (bytes + 255) & ~(size_t)255;
  if (hipMallocAsync(&p, bytes, s) != hipSuccess || !p) throw Error(ZR_ENOMEM);
  ptrs.push_back(p);
  return p;
}

void check(hipError_t e) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) throw Error(ZR_ENOMEM);
    throw Error(ZR_EDEVICE);
  }
}

void h2d(void* d, const void* h, size_t bytes, hipStream_t s) {
  if (bytes) check(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
}

void d2h_sync(void* h, const void* d, size_t bytes, hipStream_t s) {
  if (bytes) check(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s));
  check(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// schedule (SplitMix64)

struct SplitMix {
  uint64_t st;
  explicit SplitMix(uint64_t seed) : st(seed) {}
  uint64_t next() {
    st += 0x9E3779B97F4A7C15ull;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  uint64_t uniform(uint64_t lo, uint64_t hi) {
    const uint64_t n = hi - lo;
    const zr_u128 lim = (((zr_u128)1 << 64) / n) * n;
    for (;;) {
      const uint64_t u = next();
      if ((zr_u128)u < lim) return lo + u % n;
    }
  }
};

void make_schedule(uint64_t p, uint32_t nvars, const uint32_t* nnodes, uint64_t seed, uint32_t nprobes,
                   uint64_t* y, uint64_t* anchor, uint64_t* nodes, uint64_t* probes) {
  SplitMix g(seed);
  for (uint32_t v = 0; v < nvars; ++v) y[v] = g.uniform(2, p - 1);
  for (uint32_t v = 0; v < nvars; ++v) anchor[v] = g.uniform(1, p);
  size_t off = 0;
  for (uint32_t v = 0; v < nvars; ++v) {
    std::vector<uint64_t> used{anchor[v]};
    for (uint32_t j = 0; j < nnodes[v];) {
      const uint64_t x = g.uniform(1, p);
      if (std::find(used.begin(), used.end(), x) != used.end()) continue;
      used.push_back(x);
      nodes[off + j] = x;
      ++j;
    }
    off += nnodes[v];
  }
  for (uint32_t q = 0; q < nprobes; ++q)
    for (uint32_t v = 0; v < nvars; ++v) probes[(size_t)q * nvars + v] = g.uniform(1, p);
}

bool is_prime_u64(uint64_t n) {
  static const uint64_t B[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t b : B)
    if (n % b == 0) return n == b;
  if (n >= ((uint64_t)1 << 63)) return false;  // beyond the library's field range
  const zr_mod M = zr_mod_make(n);
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : B) {
    uint64_t x = zr_pow(M, a, d);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = zr_mul(M, x, x);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

// Validated parameters with the schedule materialised on the host.
Params::Params(const zr_params* P, bool balanced) {
  if (!P) throw Error(ZR_EINVAL);
  p = P->p;
  nvars = P->nvars;
  if (p < 3 || p >= ((uint64_t)1 << 63) || nvars == 0 || nvars > 64 || !P->deg) throw Error(ZR_EINVAL);
  if (!is_prime_u64(p)) throw Error(ZR_ENOTPRIME);
  M = zr_mod_make(p);
  deg.assign(P->deg, P->deg + nvars);
  if (balanced) {
    if (!P->deg_den) throw Error(ZR_EINVAL);
    deg_den.assign(P->deg_den, P->deg_den + nvars);
  }
  for (uint32_t v = 0; v < nvars; ++v) {
    if (deg[v] > 127) throw Error(ZR_EINVAL);
    if (balanced && deg_den[v] > 127) throw Error(ZR_EINVAL);
  }
  need.resize(nvars);
  for (uint32_t v = 0; v < nvars; ++v) need[v] = balanced ? zr_thiele_nodes(deg[v], deg_den[v]) : deg[v];
  last = (P->last_stage == 0 || P->last_stage > nvars) ? nvars : P->last_stage;
  nprobes = P->nprobes;
  const bool explicit_sched = P->y && P->anchor && P->nodes && P->nnodes;
  if (explicit_sched) {
    y.assign(P->y, P->y + nvars);
    anchor.assign(P->anchor, P->anchor + nvars);
    nnodes.assign(P->nnodes, P->nnodes + nvars);
    size_t tot = 0;
    for (uint32_t v = 0; v < nvars; ++v) tot += nnodes[v];
    nodes.assign(P->nodes, P->nodes + tot);
  } else {
    nnodes = need;
    size_t tot = 0;
    for (uint32_t v = 0; v < nvars; ++v) tot += nnodes[v];
    y.resize(nvars);
    anchor.resize(nvars);
    nodes.resize(tot);
    std::vector<uint64_t> pr((size_t)nprobes * nvars);
    make_schedule(p, nvars, nnodes.data(), P->seed, nprobes, y.data(), anchor.data(), nodes.data(), pr.data());
    if (!P->probes) probes = pr;
  }
  if (nprobes && P->probes) probes.assign(P->probes, P->probes + (size_t)nprobes * nvars);
  if (nprobes && probes.empty()) {
    // explicit schedule without probe points: draw them from the seed
    std::vector<uint64_t> yy(nvars), aa(nvars), pr((size_t)nprobes * nvars);
    std::vector<uint32_t> zero(nvars, 0);
    make_schedule(p, nvars, zero.data(), P->seed, nprobes, yy.data(), aa.data(), nullptr, pr.data());
    probes = pr;
  }
  node_off.resize(nvars + 1, 0);
  for (uint32_t v = 0; v < nvars; ++v) {
    if (nnodes[v] < need[v]) throw Error(ZR_EINVAL);
    node_off[v + 1] = node_off[v] + nnodes[v];
  }
  // value checks
  for (uint32_t v = 0; v < nvars; ++v) {
    if (y[v] >= p || y[v] < 2 || anchor[v] >= p) throw Error(ZR_EINVAL);
    for (uint32_t j = 0; j < nnodes[v]; ++j) {
      const uint64_t x = nodes[node_off[v] + j];
      if (x >= p || x == anchor[v]) throw Error(ZR_EINVAL);
      for (uint32_t i = 0; i < j; ++i)
        if (nodes[node_off[v] + i] == x) throw Error(ZR_EINVAL);
    }
  }
  for (uint64_t x : probes)
    if (x >= p) throw Error(ZR_EINVAL);
}

std::vector<uint64_t> Params::node_list(uint32_t v, uint32_t count) const {
  std::vector<uint64_t> X(count);
  X[0] = anchor[v];
  for (uint32_t j = 1; j < count; ++j) X[j] = nodes[node_off[v] + j - 1];
  return X;
}

// Newton constants for nodes X[0..D1): x, x', 1/(x_i - x_{i-j}) and Shoup constants.
std::vector<uint64_t> newton_consts(const zr_mod& M, const std::vector<uint64_t>& X) {
  const size_t D1 = X.size();
  std::vector<uint64_t> c(2 * D1 + 2 * D1 * D1, 0);
  for (size_t i = 0; i < D1; ++i) {
    c[i] = X[i];
    c[D1 + i] = zr_shoup_pre(M, X[i]);
  }
  uint64_t* invd = c.data() + 2 * D1;
  uint64_t* invdp = invd + D1 * D1;
  for (size_t j = 1; j < D1; ++j)
    for (size_t i = j; i < D1; ++i) {
      const uint64_t d = zr_sub(M, X[i], X[i - j]);
      const uint64_t iv = zr_inv(M, d);
      invd[j * D1 + i] = iv;
      invdp[j * D1 + i] = zr_shoup_pre(M, iv);
    }
  return c;
}

// ---------------------------------------------------------------------------
// per-thread counters

static thread_local zr_counters g_counters;
zr_counters& counters() { return g_counters; }

void count_solve(uint64_t t, uint64_t R) {
  const uint64_t w = R * t * t + 2 * t * (t ? t - 1 : 0) + t * (t ? t - 1 : 0) / 2 + t * (R + 3);
  g_counters.mulmods += w;
  g_counters.solve_mulmods += R * t * t + 2 * t * (t ? t - 1 : 0);
  g_counters.vsolve_terms += t * R;
  g_counters.max_t = std::max<uint64_t>(g_counters.max_t, t);
}

void count_newton(uint64_t t, uint64_t D1) { g_counters.mulmods += t * (D1 ? D1 - 1 : 0) * D1; }

// ---------------------------------------------------------------------------
// black-box call

void call_bb(zr_blackbox_fn bb, void* ctx, const Params& P, uint32_t k, uint64_t ni, const uint64_t* y,
             const uint64_t* xk, uint64_t nj, uint64_t* d_vals, hipStream_t s) {
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
  if (ni == 0 || nj == 0) return;
  if (bb(ctx, &pts, d_vals, s) != 0) throw Error(ZR_EBLACKBOX);
}

// ---------------------------------------------------------------------------
// Skeleton lift: Newton over x_k for each term + expansion into the new skeleton.

void Skeleton::alloc(DevArena& A, uint32_t nv, uint32_t n) {
  nvars = nv;
  t = n;
  exps = A.alloc<uint16_t>((size_t)nv * std::max<uint32_t>(n, 1));
  coef = A.alloc<uint64_t>(std::max<uint32_t>(n, 1));
  mono = A.alloc<uint64_t>(std::max<uint32_t>(n, 1));
}

// vals [D1][t] (row 0 = coefficients at the anchor) -> new skeleton in `out`
// (allocated from `keep`).  Returns the new size.
uint32_t lift_stage(const Params& P, uint32_t kvar, const Skeleton& S, const uint64_t* d_vals, uint32_t D1,
                    const std::vector<uint64_t>& X, DevArena& keep, Skeleton& out, hipStream_t s,
                    int32_t* d_status, int32_t* h_status_out) {
  DevArena A(s);
  const uint32_t t = S.t;
  std::vector<uint64_t> nc = newton_consts(P.M, X);
  uint64_t* d_nc = A.alloc<uint64_t>(nc.size());
  h2d(d_nc, nc.data(), nc.size() * 8, s);
  uint64_t* g = A.alloc<uint64_t>((size_t)D1 * std::max<uint32_t>(t, 1));
  uint32_t* cnt = A.alloc<uint32_t>(std::max<uint32_t>(t, 1));
  uint32_t* off = A.alloc<uint32_t>((size_t)t + 1);
  uint32_t* tmp = A.alloc<uint32_t>(scan_tmp_words(t));
  check(newton_lift(P.M, t, D1, d_vals, d_nc, g, cnt, s));
  count_newton(t, D1);
  if (t == 0) check(fill_i32((int32_t*)off, 0, 1, s));
  else check(exclusive_scan(t, cnt, off, tmp, s));
  struct {
    uint32_t total;
    int32_t status;
  } h;
  check(hipMemcpyAsync(&h.total, off + t, 4, hipMemcpyDeviceToHost, s));
  check(hipMemcpyAsync(&h.status, d_status, 4, hipMemcpyDeviceToHost, s));
  check(hipStreamSynchronize(s));
  if (h_status_out) *h_status_out = h.status;
  if (h.status != 0) throw Error(h.status);
  // powers of y_k for the monomial values of the next stage
  std::vector<uint64_t> yp(2 * D1);
  uint64_t acc = 1 % P.p;
  for (uint32_t d = 0; d < D1; ++d) {
    yp[d] = acc;
    yp[D1 + d] = zr_shoup_pre(P.M, acc);
    acc = zr_mul(P.M, acc, P.y[kvar]);
  }
  uint64_t* d_yp = A.alloc<uint64_t>(2 * D1);
  h2d(d_yp, yp.data(), yp.size() * 8, s);
  out.alloc(keep, P.nvars, h.total);
  check(expand(P.M, t, D1, kvar, P.nvars, S.exps, S.mono, g, off, d_yp, d_yp + D1, out.exps, out.coef, out.mono,
               std::max<uint32_t>(h.total, 1), s));
  // keep host inputs alive until the enqueued copies have run
  check(hipStreamSynchronize(s));
  return h.total;
}

// One polynomial Zippel stage k >= 2 (0-based kvar = k-1) for a given skeleton
// and right-hand sides already in vals[1..R] (rows of length t).
void solve_stage(const Params& P, const Skeleton& S, uint64_t* vals, uint32_t R, hipStream_t s, int32_t* d_status) {
  const uint32_t t = S.t;
  if (t == 0 || R == 0) return;
  DevArena A(s);
  uint64_t* Mc = A.alloc<uint64_t>(t);
  uint64_t* tmp = A.alloc<uint64_t>(t);
  check(master_poly(P.M, t, S.mono, Mc, tmp, s));
  VsolvePlan plan = vsolve_plan(t, R, target_waves());
  uint64_t* work = A.alloc<uint64_t>(vsolve_workspace_words(plan));
  check(vsolve(P.M, plan, S.mono, Mc, vals + t, t, vals + t, t, work, d_status, s));
  count_solve(t, R);
}

uint32_t target_waves() {
  static uint32_t cached = 0;
  if (cached) return cached;
  int dev = 0, cus = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const char* env = getenv("ZR_TARGET_WAVES_PER_CU");
  const uint32_t per = env ? (uint32_t)atoi(env) : 8;
  cached = (uint32_t)cus * std::max<uint32_t>(per, 1);
  return cached;
}

// Download a skeleton into a zr_poly (row-major exponents).
void download(const Skeleton& S, hipStream_t s, zr_poly* out) {
  out->nvars = S.nvars;
  out->nterms = S.t;
  out->exps = (uint16_t*)malloc(sizeof(uint16_t) * std::max<size_t>((size_t)S.t * S.nvars, 1));
  out->coeffs = (uint64_t*)malloc(sizeof(uint64_t) * std::max<uint32_t>(S.t, 1));
  if (!out->exps || !out->coeffs) {
    free(out->exps);
    free(out->coeffs);
    out->exps = nullptr;
    out->coeffs = nullptr;
    throw Error(ZR_ENOMEM);
  }
  std::vector<uint16_t> soa((size_t)S.t * S.nvars);
  if (S.t) {
    check(hipMemcpyAsync(soa.data(), S.exps, soa.size() * 2, hipMemcpyDeviceToHost, s));
    check(hipMemcpyAsync(out->coeffs, S.coef, (size_t)S.t * 8, hipMemcpyDeviceToHost, s));
  }
  check(hipStreamSynchronize(s));
  for (uint32_t l = 0; l < S.t; ++l)
    for (uint32_t v = 0; v < S.nvars; ++v) out->exps[(size_t)l * S.nvars + v] = soa[(size_t)v * S.t + l];
}

// Value of a device skeleton at an explicit point (host result).
uint64_t eval_at(const Params& P, const Skeleton& S, const uint64_t* pt, const std::vector<uint32_t>& maxdeg,
                 hipStream_t s) {
  DevArena A(s);
  uint32_t ld = 1;
  for (uint32_t v = 0; v < P.nvars; ++v) ld = std::max(ld, maxdeg[v] + 1);
  std::vector<uint64_t> tab((size_t)P.nvars * ld, 0);
  for (uint32_t v = 0; v < P.nvars; ++v) {
    uint64_t acc = 1 % P.p;
    for (uint32_t d = 0; d <= maxdeg[v]; ++d) {
      tab[(size_t)v * ld + d] = acc;
      acc = zr_mul(P.M, acc, pt[v]);
    }
  }
  uint64_t* d_tab = A.alloc<uint64_t>(tab.size());
  uint64_t* d_res = A.alloc<uint64_t>(1);
  h2d(d_tab, tab.data(), tab.size() * 8, s);
  if (S.t == 0) check(fill_u64(d_res, 0, 1, s));
  else check(poly_eval_point(P.M, S.t, P.nvars, S.exps, S.t, S.coef, d_tab, ld, d_res, s));
  uint64_t r = 0;
  d2h_sync(&r, d_res, 8, s);
  return r;
}

uint64_t bb_at(const Params& P, zr_blackbox_fn bb, void* ctx, const uint64_t* pt, hipStream_t s) {
  DevArena A(s);
  uint64_t* d = A.alloc<uint64_t>(1);
  call_bb(bb, ctx, P, P.nvars, 1, pt, pt + (P.nvars - 1), 1, d, s);
  uint64_t r = 0;
  d2h_sync(&r, d, 8, s);
  return r;
}

// ---------------------------------------------------------------------------
// polynomial Zippel

static void reconstruct_poly(const zr_params* params, zr_blackbox_fn bb, void* ctx, hipStream_t s, zr_poly* out) {
  Params P(params, false);
  g_counters = zr_counters{};
  DevArena keep(s);
  std::vector<std::unique_ptr<DevArena>> arenas;
  int32_t* d_status = keep.alloc<int32_t>(1);
  check(fill_i32(d_status, 0, 1, s));
  // stage 1: Newton in x_1 from D_1 + 1 samples
  Skeleton root;
  root.alloc(keep, P.nvars, 1);
  check(fill_u64(root.mono, 1 % P.p, 1, s));
  check(fill_u64(root.coef, 1 % P.p, 1, s));
  {
    std::vector<uint16_t> z(P.nvars, 0);
    h2d(root.exps, z.data(), z.size() * 2, s);
    check(hipStreamSynchronize(s));
  }
  uint32_t D1 = P.deg[0] + 1;
  std::vector<uint64_t> X = P.node_list(0, D1);
  Skeleton cur;
  {
    DevArena A(s);
    uint64_t* vals = A.alloc<uint64_t>(D1);
    call_bb(bb, ctx, P, 1, 1, P.y.data(), X.data(), D1, vals, s);
    DevArena* kp = new DevArena(s);
    lift_stage(P, 0, root, vals, D1, X, *kp, cur, s, d_status, nullptr);
    arenas.emplace_back(kp);
  }
  g_counters.stages = 1;
  for (uint32_t k = 2; k <= P.last; ++k) {
    const uint32_t kvar = k - 1;
    const uint32_t R = P.deg[kvar];
    D1 = R + 1;
    X = P.node_list(kvar, D1);
    const uint32_t t = cur.t;
    Skeleton nxt;
    DevArena* kp = new DevArena(s);
    {
      DevArena A(s);
      uint64_t* vals = A.alloc<uint64_t>((size_t)D1 * std::max<uint32_t>(t, 1));
      check(copy_u64(vals, cur.coef, t, s));
      call_bb(bb, ctx, P, k, t, P.y.data(), X.data() + 1, R, vals + t, s);
      solve_stage(P, cur, vals, R, s, d_status);
      lift_stage(P, kvar, cur, vals, D1, X, *kp, nxt, s, d_status, nullptr);
    }
    // the previous skeleton's arena can go once the new one is built
    arenas.front().reset();
    arenas.erase(arenas.begin());
    arenas.emplace_back(kp);
    cur = nxt;
    g_counters.stages = k;
  }
  if (P.last == P.nvars && P.nprobes) {
    for (uint32_t q = 0; q < P.nprobes; ++q) {
      const uint64_t* pt = P.probes.data() + (size_t)q * P.nvars;
      const uint64_t want = bb_at(P, bb, ctx, pt, s);
      const uint64_t got = eval_at(P, cur, pt, P.deg, s);
      if (want != got) throw Error(ZR_EPROBE);
    }
  }
  download(cur, s, out);
}

}  // namespace zr

// ===========================================================================
// C ABI
// ===========================================================================

using namespace zr;

extern "C" {

const char* zr_strerror(int st) {
  switch (st) {
    case ZR_OK: return "ok";
    case ZR_EINVAL: return "invalid argument";
    case ZR_ENOTPRIME: return "modulus is not prime";
    case ZR_ESINGULAR: return "singular Zippel system (colliding or zero monomial values)";
    case ZR_EDEGEN: return "degenerate interpolation";
    case ZR_EPROBE: return "probe mismatch or samples exhausted";
    case ZR_ENORM: return "denominator has no constant term";
    case ZR_ENOMEM: return "out of memory";
    case ZR_EDEVICE: return "HIP runtime error";
    case ZR_EBLACKBOX: return "black box failed";
    default: return "unknown status";
  }
}

void zr_poly_free(zr_poly* poly) {
  if (!poly) return;
  free(poly->exps);
  free(poly->coeffs);
  poly->exps = nullptr;
  poly->coeffs = nullptr;
  poly->nterms = 0;
}

uint32_t zr_thiele_nodes(uint32_t a, uint32_t b) {
  uint32_t m = a > 0 ? 2 * a - 1 : 0;
  m = std::max(m, 2 * b);
  return m + 1;
}

int zr_is_prime(uint64_t n) { return is_prime_u64(n) ? 1 : 0; }

zr_status zr_schedule(uint64_t p, uint32_t nvars, const uint32_t* nnodes, uint64_t seed, uint32_t nprobes,
                      uint64_t* y, uint64_t* anchor, uint64_t* nodes, uint64_t* probes) {
  if (p < 5 || p >= ((uint64_t)1 << 63) || nvars == 0 || !nnodes || !y || !anchor) return ZR_EINVAL;
  make_schedule(p, nvars, nnodes, seed, nprobes, y, anchor, nodes, probes);
  return ZR_OK;
}

zr_status zippel_reconstruct(const zr_params* params, zr_blackbox_fn bb, void* ctx, hipStream_t stream,
                             zr_poly* out) {
  if (!out || !bb) return ZR_EINVAL;
  out->nvars = 0;
  out->nterms = 0;
  out->exps = nullptr;
  out->coeffs = nullptr;
  try {
    reconstruct_poly(params, bb, ctx, stream, out);
    return ZR_OK;
  } catch (const Error& e) {
    zr_poly_free(out);
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    zr_poly_free(out);
    return ZR_ENOMEM;
  }
}

zr_status zr_copy_h2d(void* d, const void* h, size_t bytes, hipStream_t s) {
  if (bytes == 0) return ZR_OK;
  if (hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return ZR_EDEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? ZR_OK : ZR_EDEVICE;
}
zr_status zr_copy_d2h(void* h, const void* d, size_t bytes, hipStream_t s) {
  if (bytes == 0) return ZR_OK;
  if (hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, s) != hipSuccess) return ZR_EDEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? ZR_OK : ZR_EDEVICE;
}
zr_status zr_copy_d2d(void* d, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return ZR_OK;
  return hipMemcpyAsync(d, src, bytes, hipMemcpyDeviceToDevice, s) == hipSuccess ? ZR_OK : ZR_EDEVICE;
}

void zr_last_counters(zr_counters* out) {
  if (out) *out = zr::g_counters;
}

// ---- record / replay black box ----------------------------------------------

struct zr_recorder {
  zr_blackbox_fn inner;
  void* inner_ctx;
  int replay;
  size_t idx;
  struct Rec {
    uint32_t k;
    uint64_t ni, nj;
    uint64_t* d;
  };
  std::vector<Rec> recs;
};

zr_status zr_recorder_create(zr_recorder** rec, zr_blackbox_fn inner, void* inner_ctx) {
  if (!rec) return ZR_EINVAL;
  zr_recorder* r = new (std::nothrow) zr_recorder();
  if (!r) return ZR_ENOMEM;
  r->inner = inner;
  r->inner_ctx = inner_ctx;
  r->replay = 0;
  r->idx = 0;
  *rec = r;
  return ZR_OK;
}

void zr_recorder_destroy(zr_recorder* rec) {
  if (!rec) return;
  for (auto& r : rec->recs) hipFree(r.d);
  delete rec;
}

void zr_recorder_rewind(zr_recorder* rec) {
  if (rec) rec->idx = 0;
}

void zr_recorder_set_replay(zr_recorder* rec, int replay) {
  if (rec) {
    rec->replay = replay;
    rec->idx = 0;
  }
}

int zr_recorder_blackbox(void* ctx, const zr_points* pts, uint64_t* d_vals, hipStream_t stream) {
  zr_recorder* rec = (zr_recorder*)ctx;
  const size_t n = (size_t)pts->ni * pts->nj;
  if (rec->replay) {
    if (rec->idx >= rec->recs.size()) return 2;
    const auto& r = rec->recs[rec->idx++];
    if (r.k != pts->k || r.ni != pts->ni || r.nj != pts->nj) return 3;
    return hipMemcpyAsync(d_vals, r.d, n * 8, hipMemcpyDeviceToDevice, stream) == hipSuccess ? 0 : 4;
  }
  if (!rec->inner) return 5;
  int st = rec->inner(rec->inner_ctx, pts, d_vals, stream);
  if (st) return st;
  zr_recorder::Rec r;
  r.k = pts->k;
  r.ni = pts->ni;
  r.nj = pts->nj;
  r.d = nullptr;
  if (hipMalloc(&r.d, std::max<size_t>(n, 1) * 8) != hipSuccess) return 6;
  if (hipMemcpyAsync(r.d, d_vals, n * 8, hipMemcpyDeviceToDevice, stream) != hipSuccess) return 7;
  if (hipStreamSynchronize(stream) != hipSuccess) return 8;
  rec->recs.push_back(r);
  return 0;
}

}  // extern "C"
