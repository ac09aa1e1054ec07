// Host driver of the Zippel reconstruction and the C ABI declared in zippel.h.
// The host runs the stage loop (one stage per variable, §1) and talks to the
// black box; every O(t^2) and O(t D^2) step runs in the gfx950 kernels.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <stdexcept>
#include <vector>

#include "../../include/zippel.h"
#include "batch.hpp"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"

namespace zr {

// ---------------------------------------------------------------------------
// device memory: a stream-ordered block cache.  Blocks released by a call on a
// stream go to that stream's free list and are handed out again only to later
// work on the same stream, which runs after every earlier user of the block;
// so neither allocation nor release ever waits for the device.  Blocks are
// kept until the process ends (sizes are rounded up to powers of two).

namespace {
struct BlockCache {
  std::mutex mu;
  std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void*>> free;
};
BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();  // never destroyed: blocks live until exit
  return *c;
}
size_t size_class(size_t bytes) {
  size_t c = 256;
  while (c < bytes) c <<= 1;
  return c;
}
}  // namespace

// The arena keeps a pointer to its (device, stream) free list: entries of the
// cache's map are never removed, so the pointer stays valid.
DevArena::DevArena(hipStream_t st) : s(st) {
  (void)hipGetDevice(&dev);
  BlockCache& C = block_cache();
  std::lock_guard<std::mutex> g(C.mu);
  free_list = &C.free[{dev, s}];
}

DevArena::~DevArena() {
  BlockCache& C = block_cache();
  std::lock_guard<std::mutex> g(C.mu);
  auto& fl = *free_list;
  for (auto& b : blocks) fl.emplace(b.second, b.first);
}

void* DevArena::raw(size_t bytes) {
  const size_t cls = size_class(std::max<size_t>(bytes, 256));
  BlockCache& C = block_cache();
  {
    std::lock_guard<std::mutex> g(C.mu);
    auto& fl = *free_list;
    auto it = fl.find(cls);
    if (it != fl.end()) {
      void* p = it->second;
      fl.erase(it);
      blocks.emplace_back(p, cls);
      return p;
    }
  }
  void* p = nullptr;
  const hipError_t e = hipMallocAsync(&p, cls, s);
  if (e != hipSuccess || !p) {
    note_error("hipMallocAsync(%zu bytes for %zu requested) failed: %s", cls, bytes, hipGetErrorString(e));
    (void)hipGetLastError();
    throw Error(ZR_ENOMEM);
  }
  blocks.emplace_back(p, cls);
  return p;
}

static thread_local char g_last_error[512] = "";

void note_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
}

void check_at(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    const char* base = strrchr(file, '/');
    note_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), base ? base + 1 : file, line);
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
  // resumption from a stage's result: shape, bounds, order and values
  first = P->first_stage <= 1 ? 1 : P->first_stage;
  if (first > 1) {
    start = P->start;
    if (balanced || first > last || !start || start->nvars != nvars || start->nterms >= ((uint64_t)1 << 31) ||
        (start->nterms && (!start->exps || !start->coeffs)))
      throw Error(ZR_EINVAL);
    const uint32_t kv = first - 1;  // variables x_1..x_{k-1} are reached
    for (uint64_t l = 0; l < start->nterms; ++l) {
      const uint16_t* e = start->exps + l * nvars;
      if (start->coeffs[l] >= p) throw Error(ZR_EINVAL);
      for (uint32_t v = 0; v < nvars; ++v)
        if (v < kv ? e[v] > deg[v] : e[v] != 0) throw Error(ZR_EINVAL);
      if (l > 0 && !std::lexicographical_compare(e - nvars, e, e, e + nvars)) throw Error(ZR_EINVAL);
    }
  }
}

std::vector<uint64_t> Params::node_list(uint32_t v, uint32_t count) const {
  std::vector<uint64_t> X(count);
  X[0] = anchor[v];
  for (uint32_t j = 1; j < count; ++j) X[j] = nodes[node_off[v] + j - 1];
  return X;
}

// Matrix of Newton interpolation at nodes X[0..D1): the interpolant of values
// a_i is sum_i a_i L_i(z) with the Lagrange basis L_i = Q_i / Q_i(x_i),
// Q_i = prod_{j != i} (z - x_j) = MX(z) / (z - x_i), MX = prod_j (z - x_j); so
// W[d][i] = coefficient d of L_i.  Q_i comes from MX by synthetic division, the
// D1 denominators are inverted together (one inversion and 3 D1 products).
// Returned as 22-bit limbs laid out [i][d][3] for the lift kernel.
static std::vector<uint32_t> newton_matrix_limbs_uncached(const zr_mod& M, const std::vector<uint64_t>& X) {
  const size_t D1 = X.size();
  std::vector<uint64_t> MX(D1 + 1, 0);
  MX[0] = 1 % M.p;
  for (size_t j = 0; j < D1; ++j) {
    MX[j + 1] = MX[j];
    for (size_t r = j; r >= 1; --r) MX[r] = zr_sub(M, MX[r - 1], zr_mul(M, X[j], MX[r]));
    MX[0] = zr_neg(M, zr_mul(M, X[j], MX[0]));
  }
  std::vector<uint64_t> Q(D1 * D1), den(D1), pre(D1 + 1);
  for (size_t i = 0; i < D1; ++i) {
    uint64_t* q = &Q[i * D1];
    q[D1 - 1] = MX[D1];
    for (size_t r = D1 - 1; r >= 1; --r) q[r - 1] = zr_add(M, MX[r], zr_mul(M, X[i], q[r]));
    uint64_t h = 0;
    for (size_t r = D1; r-- > 0;) h = zr_add(M, zr_mul(M, h, X[i]), q[r]);
    den[i] = h;
  }
  // batch inversion of the denominators (nonzero: the nodes are distinct)
  pre[0] = 1 % M.p;
  for (size_t i = 0; i < D1; ++i) pre[i + 1] = zr_mul(M, pre[i], den[i]);
  uint64_t inv_all = zr_inv(M, pre[D1]);
  std::vector<uint64_t> inv(D1);
  for (size_t i = D1; i-- > 0;) {
    inv[i] = zr_mul(M, inv_all, pre[i]);
    inv_all = zr_mul(M, inv_all, den[i]);
  }
  std::vector<uint32_t> W(D1 * D1 * 3, 0);
  for (size_t i = 0; i < D1; ++i)
    for (size_t d = 0; d < D1; ++d) {
      const uint64_t c = zr_mul(M, Q[i * D1 + d], inv[i]);
      uint32_t* w = &W[(i * D1 + d) * 3];
      w[0] = (uint32_t)(c & 0x3FFFFF);
      w[1] = (uint32_t)((c >> 22) & 0x3FFFFF);
      w[2] = (uint32_t)(c >> 44);
    }
  return W;
}

std::vector<uint32_t> newton_matrix_limbs(const zr_mod& M, const std::vector<uint64_t>& X) {
  // the same node lists recur across reconstructions that share a schedule
  static std::mutex mu;
  static std::vector<std::pair<std::vector<uint64_t>, std::vector<uint32_t>>> cache;
  std::vector<uint64_t> key(X);
  key.push_back(M.p);
  {
    std::lock_guard<std::mutex> g(mu);
    for (auto& e : cache)
      if (e.first == key) return e.second;
  }
  std::vector<uint32_t> W = newton_matrix_limbs_uncached(M, X);
  std::lock_guard<std::mutex> g(mu);
  if (cache.size() >= 64) cache.erase(cache.begin());
  cache.emplace_back(std::move(key), W);
  return W;
}

// Device copies of the per-variable constants a stage needs: the Newton matrix
// for D1 nodes and the powers y_v^d (with Shoup constants) for d < D1.
StageConsts::StageConsts(const Params& P, DevArena& A, const std::vector<uint32_t>& D1s, hipStream_t s) {
  const uint32_t n = (uint32_t)D1s.size();
  woff.resize(n);
  yoff.resize(n);
  size_t words = 0;  // in 32-bit units, 8-byte aligned pieces
  std::vector<std::vector<uint32_t>> Ws(n);
  for (uint32_t v = 0; v < n; ++v) {
    if (!D1s[v]) continue;
    Ws[v] = newton_matrix_limbs(P.M, P.node_list(v, D1s[v]));
    woff[v] = words;
    // zero padding: the lift kernel fetches whole groups of limbs ahead of use
    words += (Ws[v].size() + 3 * 8 + 1) & ~(size_t)1;
    yoff[v] = words;
    words += 4 * (size_t)D1s[v];
  }
  std::vector<uint32_t> host(std::max<size_t>(words, 2), 0);
  for (uint32_t v = 0; v < n; ++v) {
    if (!D1s[v]) continue;
    std::copy(Ws[v].begin(), Ws[v].end(), host.begin() + woff[v]);
    uint64_t* yp = (uint64_t*)(host.data() + yoff[v]);
    uint64_t acc = 1 % P.p;
    for (uint32_t d = 0; d < D1s[v]; ++d) {
      yp[d] = acc;
      yp[D1s[v] + d] = zr_shoup_pre(P.M, acc);
      acc = zr_mul(P.M, acc, P.y[v]);
    }
  }
  // through pinned staging, so the upload stays asynchronous
  Blob b;
  b.add(host);
  base = (uint32_t*)b.upload(A, s);
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
  g_counters.dot_products += R * t * t;
  g_counters.chain_steps += t * (t ? t - 1 : 0);
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
  pts.nexpr = 1;
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
// (allocated from `keep`).  One host synchronisation: the new size.
uint32_t lift_stage(const Params& P, uint32_t kvar, const Skeleton& S, const uint64_t* d_vals, uint32_t D1,
                    const uint32_t* d_W, const uint64_t* d_ypow, DevArena& keep, Skeleton& out, hipStream_t s,
                    int32_t* d_status) {
  DevArena A(s);
  const uint32_t t = S.t;
  uint64_t* g = A.alloc<uint64_t>((size_t)D1 * std::max<uint32_t>(t, 1));
  uint32_t* cnt = A.alloc<uint32_t>(std::max<uint32_t>(t, 1));
  uint32_t* off = A.alloc<uint32_t>((size_t)t + 1);
  uint32_t* tmp = A.alloc<uint32_t>(scan_tmp_words(t));
  check(newton_lift(P.M, t, D1, d_vals, d_W, g, cnt, s));
  count_newton(t, D1);
  if (t == 0) check(fill_i32((int32_t*)off, 0, 1, s));
  else check(exclusive_scan(t, cnt, off, tmp, s));
  int32_t* h = host_scratch();
  check(hipMemcpyAsync(&h[0], off + t, 4, hipMemcpyDeviceToHost, s));
  check(hipMemcpyAsync(&h[1], d_status, 4, hipMemcpyDeviceToHost, s));
  check(hipStreamSynchronize(s));
  const uint32_t total = (uint32_t)h[0];
  if (h[1] != 0) throw Error(h[1]);
  out.alloc(keep, P.nvars, total);
  check(expand(P.M, t, D1, kvar, P.nvars, S.exps, S.mono, g, off, d_ypow, d_ypow + D1, out.exps, out.coef, out.mono,
               std::max<uint32_t>(total, 1), s));
  return total;
}

int32_t* host_words(size_t n) {
  static thread_local int32_t* buf = nullptr;
  static thread_local size_t cap = 0;
  if (n > cap) {
    if (buf) check(hipHostFree(buf));
    buf = nullptr;
    cap = 0;
    const size_t want = std::max<size_t>(n, 1 << 14);
    void* p = nullptr;
    check(hipHostMalloc(&p, want * 4, hipHostMallocDefault));
    buf = (int32_t*)p;
    cap = want;
  }
  return buf;
}

// Pinned host words for the per-stage size read-back.
int32_t* host_scratch() {
  static thread_local int32_t* buf = nullptr;
  if (!buf) {
    void* p = nullptr;
    check(hipHostMalloc(&p, 64, hipHostMallocDefault));
    buf = (int32_t*)p;
  }
  return buf;
}

// One polynomial Zippel stage k >= 2 (0-based kvar = k-1) for a given skeleton
// and right-hand sides already in vals[1..R] (rows of length t).
void solve_stage(const Params& P, const Skeleton& S, uint64_t* vals, uint32_t R, hipStream_t s, int32_t* d_status) {
  const uint32_t t = S.t;
  if (t == 0 || R == 0) return;
  DevArena A(s);
  uint64_t* Mc = A.alloc<uint64_t>(t);
  uint64_t* tmp = A.alloc<uint64_t>(master_tmp_words(t));
  check(master_poly(P.M, t, S.mono, Mc, tmp, s));
  VsolvePlan plan = vsolve_plan(t, R, device_cus());
  uint64_t* work = A.alloc<uint64_t>(vsolve_workspace_words(plan));
  check(vsolve(P.M, plan, S.mono, Mc, vals + t, t, vals + t, t, work, d_status, s));
  count_solve(t, R);
}

uint32_t device_cus() {
  static uint32_t cached = 0;
  if (cached) return cached;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  cached = (uint32_t)std::max(cus, 1);
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

void upload_start(const Params& P, const StageConsts& K, DevArena& keep, Skeleton& S, hipStream_t s) {
  const uint32_t t = (uint32_t)P.start->nterms, nv = P.nvars, kv = P.first - 1;
  S.alloc(keep, nv, t);
  if (t == 0) return;
  std::vector<uint16_t> soa((size_t)nv * t);
  for (uint32_t l = 0; l < t; ++l)
    for (uint32_t v = 0; v < nv; ++v) soa[(size_t)v * t + l] = P.start->exps[(size_t)l * nv + v];
  h2d(S.exps, soa.data(), soa.size() * 2, s);
  h2d(S.coef, P.start->coeffs, (size_t)t * 8, s);
  MonoTables T{};
  const uint64_t* tabs = (const uint64_t*)K.base;
  for (uint32_t v = 0; v < kv; ++v) T.off[v] = (uint32_t)(K.yoff[v] / 2);
  check(mono_values(P.M, t, kv, S.exps, t, tabs, T, S.mono, s));
  // the host arrays above are pageable: the copies have completed on return
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
  std::vector<uint32_t> D1s(P.nvars);
  for (uint32_t v = 0; v < P.nvars; ++v) D1s[v] = v < P.last ? P.deg[v] + 1 : 0;
  StageConsts K(P, keep, D1s, s);
  // stage 1: Newton in x_1 from D_1 + 1 samples
  Skeleton root;
  root.alloc(keep, P.nvars, 1);
  check(fill_u64(root.mono, 1 % P.p, 1, s));
  check(fill_u64(root.coef, 1 % P.p, 1, s));
  check(fill_u64((uint64_t*)root.exps, 0, (P.nvars * 2 + 7) / 8, s));
  uint32_t D1 = D1s[0];
  std::vector<uint64_t> X;
  Skeleton cur;
  if (P.first > 1) {
    DevArena* kp = new DevArena(s);
    arenas.emplace_back(kp);
    upload_start(P, K, *kp, cur, s);
  } else {
    X = P.node_list(0, D1);
    DevArena A(s);
    uint64_t* vals = A.alloc<uint64_t>(D1);
    call_bb(bb, ctx, P, 1, 1, P.y.data(), X.data(), D1, vals, s);
    DevArena* kp = new DevArena(s);
    arenas.emplace_back(kp);
    lift_stage(P, 0, root, vals, D1, K.W(0), K.ypow(0), *kp, cur, s, d_status);
  }
  const uint32_t k0 = P.first > 1 ? P.first : 2;
  g_counters.stages = k0 - 1;
  for (uint32_t k = k0; k <= P.last; ++k) {
    const uint32_t kvar = k - 1;
    const uint32_t R = P.deg[kvar];
    D1 = D1s[kvar];
    X = P.node_list(kvar, D1);
    const uint32_t t = cur.t;
    Skeleton nxt;
    DevArena* kp = new DevArena(s);
    arenas.emplace_back(kp);
    {
      DevArena A(s);
      uint64_t* vals = A.alloc<uint64_t>((size_t)D1 * std::max<uint32_t>(t, 1));
      check(copy_u64(vals, cur.coef, t, s));
      call_bb(bb, ctx, P, k, t, P.y.data(), X.data() + 1, R, vals + t, s);
      solve_stage(P, cur, vals, R, s, d_status);
      lift_stage(P, kvar, cur, vals, D1, K.W(kvar), K.ypow(kvar), *kp, nxt, s, d_status);
    }
    // the previous skeleton's arena can go once the new one is built
    arenas.erase(arenas.begin());
    cur = nxt;
    g_counters.stages = k;
  }
  if (P.last == P.nvars && P.nprobes) check_probes(P, bb, ctx, cur, nullptr, s);
  download(cur, s, out);
}

// Compare the black box with the reconstruction (num / den when den != NULL)
// at the probe points: all black-box calls and evaluations are enqueued, then
// one read-back.
void check_probes(const Params& P, zr_blackbox_fn bb, void* ctx, const Skeleton& N, const Skeleton* D,
                  hipStream_t s) {
  DevArena A(s);
  const uint32_t np = P.nprobes, nv = P.nvars;
  uint32_t ld = 1;
  for (uint32_t v = 0; v < nv; ++v) ld = std::max(ld, std::max(P.deg[v], D ? P.deg_den[v] : 0u) + 1);
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
  uint64_t* d_res = A.alloc<uint64_t>(3 * (size_t)np);
  uint64_t* d_part = A.alloc<uint64_t>(2 * (size_t)np * kPolyEvalBlocks);
  h2d(d_tab, tab.data(), tab.size() * 8, s);
  for (uint32_t q = 0; q < np; ++q) {
    const uint64_t* pt = P.probes.data() + (size_t)q * nv;
    call_bb(bb, ctx, P, nv, 1, pt, pt + (nv - 1), 1, d_res + q, s);
    const uint64_t* tq = d_tab + (size_t)q * nv * ld;
    uint64_t* pq = d_part + (size_t)2 * q * kPolyEvalBlocks;
    if (N.t) check(poly_eval_point(P.M, N.t, nv, N.exps, N.t, N.coef, tq, ld, d_res + np + q, pq, s));
    else check(fill_u64(d_res + np + q, 0, 1, s));
    if (D) {
      if (D->t)
        check(poly_eval_point(P.M, D->t, nv, D->exps, D->t, D->coef, tq, ld, d_res + 2 * np + q,
                              pq + kPolyEvalBlocks, s));
      else check(fill_u64(d_res + 2 * np + q, 0, 1, s));
    }
  }
  std::vector<uint64_t> r(3 * (size_t)np);
  d2h_sync(r.data(), d_res, r.size() * 8, s);
  for (uint32_t q = 0; q < np; ++q) {
    const uint64_t f = r[q], nvl = r[np + q];
    if (D ? nvl != zr_mul(P.M, f, r[2 * np + q]) : nvl != f) throw Error(ZR_EPROBE);
  }
}

}  // namespace zr

// ===========================================================================
// C ABI
// ===========================================================================

using namespace zr;

extern "C" {

const char* zr_last_error(void) { return g_last_error; }

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

zr_status zr_vandermonde_solve(uint64_t p, uint32_t t, uint32_t R, const uint64_t* d_mono, const uint64_t* d_rhs,
                               uint64_t* d_out, int32_t* d_status, hipStream_t stream) {
  if (p < 3 || p >= ((uint64_t)1 << 63) || !d_status || t >= ((uint32_t)1 << 31)) return ZR_EINVAL;
  if (t && R && (!d_mono || !d_rhs || !d_out)) return ZR_EINVAL;
  if (!is_prime_u64(p)) return ZR_ENOTPRIME;
  try {
    check(fill_i32(d_status, 0, 1, stream));
    if (t == 0 || R == 0) return ZR_OK;
    const zr_mod M = zr_mod_make(p);
    DevArena A(stream);
    uint64_t* Mc = A.alloc<uint64_t>(t);
    uint64_t* tmp = A.alloc<uint64_t>(master_tmp_words(t));
    check(master_poly(M, t, d_mono, Mc, tmp, stream));
    VsolvePlan plan = vsolve_plan(t, R, device_cus());
    uint64_t* work = A.alloc<uint64_t>(vsolve_workspace_words(plan));
    check(vsolve(M, plan, d_mono, Mc, d_rhs, t, d_out, t, work, d_status, stream));
    return ZR_OK;
  } catch (const Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    return ZR_ENOMEM;
  }
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
  for (auto& r : rec->recs) (void)hipFree(r.d);  // nothing to report to: the handle is gone either way
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
  const size_t n = (size_t)pts->ni * pts->nj * std::max<uint32_t>(pts->nexpr, 1);
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
