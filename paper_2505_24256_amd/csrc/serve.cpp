// Served form: a request loop for reconstructions that arrive over time (the
// coefficients of a modular reduction stream out one by one and each one is a
// black box to reconstruct, Introduction).  Requests are admitted while their
// estimated device footprint fits the budget and a slot is free; every step
// advances each active request by one stage, with the stage's transposed
// Vandermonde solves (§1, §2.2), Newton matrices and lifts of all active
// requests batched into one launch sequence, so requests admitted at a step
// boundary share the device with those already running (continuous batching).
// Skeletons stay on the device between steps.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <unordered_set>
#include <memory>
#include <vector>

#include "../../include/zippel.h"
#include "batch.hpp"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"

struct zr_server;

namespace zr {

namespace {

struct Request {
  uint64_t id = 0;
  bool balanced = false;
  std::unique_ptr<Params> P;
  zr_blackbox_fn bb = nullptr;
  void* ctx = nullptr;
  uint64_t footprint = 0;  // estimate for the next stage (stage_footprint)
  uint64_t cap = 0;        // bound on any skeleton's size used by the estimate
  uint32_t k = 0;          // stages done
  Skeleton SN, SD;
  std::shared_ptr<DevArena> arena;  // holds SN, SD
  int32_t* d_status = nullptr;
  int32_t status = ZR_OK;
  bool finished = false;
  zr_poly num{0, 0, nullptr, nullptr}, den{0, 0, nullptr, nullptr};
  uint64_t admitted_step = 0, finished_step = 0;
};

// Footprint model of a request's next stage (stage k + 1 after k stages
// done), from its live skeleton sizes.  Per term of a skeleton of t terms and
// D1 nodes of the new variable: the value table [D1][t], the Newton output of
// the same size and the solve's packed rows and partial sums (about 2 D1 words
// in all), and the skeleton itself; plus the next skeleton, at most t D1
// terms, capped by `cap` (the caller's expected final size, or the degree
// bounds' monomial count), at four words a term.  The balanced path has a
// numerator and a denominator and adds the per-slice Thiele tables (samples and
// two coefficient tables of nk + 1 rows for T = max(tN, tD) slices).
uint64_t monomial_count(const Params& P) {
  uint64_t c = 1;
  for (uint32_t v = 0; v < P.nvars; ++v) {
    c *= (uint64_t)P.deg[v] + 1;
    if (c > ((uint64_t)1 << 32)) return (uint64_t)1 << 32;
  }
  return c;
}

uint64_t stage_footprint(const Params& P, bool balanced, uint32_t k, uint64_t tN, uint64_t tD, uint64_t cap) {
  if (k >= P.last) return 0;
  const uint64_t D1 = (uint64_t)P.need[k] + 1;
  auto words = [&](uint64_t t) {
    t = std::max<uint64_t>(t, 1);
    return t * (4 * D1 + 12) + std::min(t * D1, cap) * 4;
  };
  if (!balanced) return 8 * words(tN);
  const uint64_t T = std::max<uint64_t>(std::max(tN, tD), 1);
  return 8 * (words(tN) + words(tD) + 3 * (D1 + 1) * T);
}

}  // namespace

struct Server {
  hipStream_t s;
  uint64_t p;
  zr_mod M;
  uint64_t budget, used = 0;
  uint32_t max_active;
  uint64_t next_id = 1, steps = 0;
  std::unique_ptr<DevArena> status_arena;
  std::vector<int32_t*> free_status;  // status words of retired requests, reused by new ones
  std::deque<Request*> pending;
  std::vector<Request*> active;
  std::map<uint64_t, Request*> done;
  std::unordered_set<uint64_t> waiting;  // ids submitted and not yet finished
  std::vector<uint64_t> newly_done;      // finished since the last zr_server_finished
  zr_server_stats stats{};
  int32_t* hbuf = nullptr;  // pinned read-back buffer
  size_t hcap = 0;
  void* dbuf = nullptr;  // pinned read-back buffer of finishing requests
  size_t dcap = 0;
  ~Server() {
    if (hbuf) (void)hipHostFree(hbuf);
    if (dbuf) (void)hipHostFree(dbuf);
    for (Request* r : pending) delete r;
    for (Request* r : active) delete r;
    for (auto& kv : done) {
      zr_poly_free(&kv.second->num);
      zr_poly_free(&kv.second->den);
      delete kv.second;
    }
  }
};

namespace {

// Device parts of finishing the requests that ended at a step, batched over
// them: the constant term of each balanced denominator (zero when that
// skeleton has no constant monomial; skeletons are in lexicographic order, so
// it can only be the first term), then the scaling of each result by one
// constant.
struct ConstTermJob {
  const uint16_t* exps;  // SoA [nvars][t]
  const uint64_t* coef;
  uint32_t t, nvars;
  uint64_t* out;
};

__global__ void k_const_terms(uint32_t n, const ConstTermJob* __restrict__ jobs) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const ConstTermJob& j = jobs[i];
  bool zero = j.t > 0;
  for (uint32_t v = 0; v < j.nvars; ++v) zero = zero && j.exps[(size_t)v * j.t] == 0;
  *j.out = zero ? j.coef[0] : 0;
}

struct ScaleJob {
  uint64_t* v;
  uint64_t n;
  uint64_t c, cp;  // the factor and its Shoup quotient
};

// one workgroup per job
__global__ void k_scale_jobs(zr_mod M, const ScaleJob* __restrict__ jobs) {
  const ScaleJob& j = jobs[blockIdx.x];
  for (uint64_t i = threadIdx.x; i < j.n; i += blockDim.x) j.v[i] = zr_shoup(M, j.v[i], j.c, j.cp);
}

// Host memory for one step's read-backs, pinned, grown as needed.
void* pinned(Server& S, size_t bytes) {
  if (S.dcap < bytes) {
    if (S.dbuf) check(hipHostFree(S.dbuf));
    S.dbuf = nullptr;
    S.dcap = 0;
    const size_t n = std::max<size_t>(bytes, 1 << 20);
    check(hipHostMalloc(&S.dbuf, n, hipHostMallocDefault));
    S.dcap = n;
  }
  return S.dbuf;
}

// The results of every request that ended at this step (its last stage done,
// or failed).  Per request this is what the one-request paths do after their
// last stage (balanced_finish, check_probes, download), with the same
// black-box calls in the same order, but the device work of all requests is
// enqueued together and read back in three host synchronisations per step
// instead of up to nine per request.
void finish_batch(Server& S, const std::vector<Request*>& ended) {
  hipStream_t s = S.s;
  DevArena A(s);
  auto fail = [](Request& r, int32_t code) {
    zr_poly_free(&r.num);
    zr_poly_free(&r.den);
    r.status = code;
  };
  std::vector<Request*> ok;
  for (Request* r : ended)
    if (r->status == ZR_OK) ok.push_back(r);
  // ---- normalisation of complete balanced results: D(0) = 1
  std::vector<Request*> norm;
  for (Request* r : ok)
    if (r->balanced && r->P->last == r->P->nvars) norm.push_back(r);
  if (!norm.empty()) {
    uint64_t* d_c0 = A.alloc<uint64_t>(norm.size());
    std::vector<ConstTermJob> cj;
    for (size_t q = 0; q < norm.size(); ++q) cj.push_back(ConstTermJob{norm[q]->SD.exps, norm[q]->SD.coef,
                                                                       norm[q]->SD.t, norm[q]->SD.nvars, d_c0 + q});
    Blob b;
    const size_t o = b.add(cj);
    char* d = b.upload(A, s);
    hipLaunchKernelGGL(k_const_terms, dim3(((uint32_t)cj.size() + 63) / 64), dim3(64), 0, s, (uint32_t)cj.size(),
                       (const ConstTermJob*)(d + o));
    check(hipGetLastError());
    uint64_t* c0 = (uint64_t*)pinned(S, norm.size() * 8);
    check(hipMemcpyAsync(c0, d_c0, norm.size() * 8, hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    std::vector<ScaleJob> sc;
    for (size_t q = 0; q < norm.size(); ++q) {
      Request& r = *norm[q];
      if (c0[q] == 0) {
        fail(r, ZR_ENORM);
        continue;
      }
      const uint64_t ci = zr_inv(S.M, c0[q]), cip = zr_shoup_pre(S.M, ci);
      if (r.SN.t) sc.push_back(ScaleJob{r.SN.coef, r.SN.t, ci, cip});
      if (r.SD.t) sc.push_back(ScaleJob{r.SD.coef, r.SD.t, ci, cip});
    }
    if (!sc.empty()) {
      Blob sb;
      const size_t so = sb.add(sc);
      char* ds = sb.upload(A, s);
      hipLaunchKernelGGL(k_scale_jobs, dim3((uint32_t)sc.size()), dim3(256), 0, s, S.M, (const ScaleJob*)(ds + so));
      check(hipGetLastError());
    }
  }
  // ---- probes: black-box values and the results' values at the probe points
  struct ProbeSet {
    Request* r;
    size_t off;  // first of 3 np result words
  };
  std::vector<ProbeSet> ps;
  size_t pwords = 0;
  for (Request* r : ok)
    if (r->status == ZR_OK && r->P->last == r->P->nvars && r->P->nprobes) {
      ps.push_back(ProbeSet{r, pwords});
      pwords += 3 * (size_t)r->P->nprobes;
    }
  if (!ps.empty()) {
    uint64_t* d_res = A.alloc<uint64_t>(pwords);
    check(fill_u64(d_res, 0, pwords, s));
    // the probe points go up once; their power tables are built on the device
    Blob pb;
    std::vector<size_t> poff(ps.size()), toff(ps.size());
    std::vector<uint32_t> lds(ps.size());
    size_t twords = 0;
    for (size_t e = 0; e < ps.size(); ++e) {
      const Params& P = *ps[e].r->P;
      const bool bal = ps[e].r->balanced;
      uint32_t ld = 1;
      for (uint32_t v = 0; v < P.nvars; ++v) ld = std::max(ld, std::max(P.deg[v], bal ? P.deg_den[v] : 0u) + 1);
      lds[e] = ld;
      poff[e] = pb.add(P.probes);
      toff[e] = twords;
      twords += (size_t)P.nprobes * P.nvars * ld;
    }
    char* dpts = pb.upload(A, s);
    uint64_t* d_tabs = A.alloc<uint64_t>(twords);
    std::vector<PowJob> pj;
    for (size_t e = 0; e < ps.size(); ++e) {
      const Params& P = *ps[e].r->P;
      for (uint32_t q = 0; q < P.nprobes; ++q)
        pj.push_back(PowJob{(const uint64_t*)(dpts + poff[e]) + (size_t)q * P.nvars,
                            d_tabs + toff[e] + (size_t)q * P.nvars * lds[e], P.nvars, lds[e]});
    }
    batched_power_tables(S.M, pj, s);
    for (size_t e = 0; e < ps.size(); ++e) {
      Request& r = *ps[e].r;
      const Params& P = *r.P;
      const Skeleton* D = r.balanced ? &r.SD : nullptr;
      const uint32_t np = P.nprobes, nv = P.nvars, ld = lds[e];
      const uint64_t* d_tab = d_tabs + toff[e];
      uint64_t* d_part = A.alloc<uint64_t>(2 * (size_t)np * kPolyEvalBlocks);
      uint64_t* res = d_res + ps[e].off;
      try {
        for (uint32_t q = 0; q < np; ++q) {
          const uint64_t* pt = P.probes.data() + (size_t)q * nv;
          call_bb(r.bb, r.ctx, P, nv, 1, pt, pt + (nv - 1), 1, res + q, s);
          const uint64_t* tq = d_tab + (size_t)q * nv * ld;
          uint64_t* pq = d_part + (size_t)2 * q * kPolyEvalBlocks;
          if (r.SN.t)
            check(poly_eval_point(P.M, r.SN.t, nv, r.SN.exps, r.SN.t, r.SN.coef, tq, ld, res + np + q, pq, s));
          if (D && D->t)
            check(poly_eval_point(P.M, D->t, nv, D->exps, D->t, D->coef, tq, ld, res + 2 * np + q,
                                  pq + kPolyEvalBlocks, s));
        }
      } catch (const Error& x) {
        fail(r, x.code);
      }
    }
    uint64_t* h = (uint64_t*)pinned(S, pwords * 8);
    check(hipMemcpyAsync(h, d_res, pwords * 8, hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    for (ProbeSet& e : ps) {
      Request& r = *e.r;
      if (r.status != ZR_OK) continue;
      const uint32_t np = r.P->nprobes;
      const uint64_t* res = h + e.off;
      for (uint32_t q = 0; q < np; ++q) {
        const uint64_t f = res[q], nvl = res[np + q];
        if (r.balanced ? nvl != zr_mul(r.P->M, f, res[2 * np + q]) : nvl != f) {
          fail(r, ZR_EPROBE);
          break;
        }
      }
    }
  }
  // ---- results: every skeleton gathered into one buffer, one read-back
  struct Out {
    const Skeleton* S;
    zr_poly* dst;
    Request* r;
    size_t eoff, coff;  // bytes into the gathered buffer
  };
  std::vector<Out> outs;
  size_t bytes = 0;
  auto align8 = [](size_t x) { return (x + 7) & ~(size_t)7; };
  for (Request* r : ok) {
    if (r->status != ZR_OK) continue;
    outs.push_back(Out{&r->SN, &r->num, r, 0, 0});
    if (r->balanced) outs.push_back(Out{&r->SD, &r->den, r, 0, 0});
  }
  if (outs.empty()) return;
  std::vector<CopyJob> cp;
  for (Out& o : outs) {
    o.eoff = bytes;
    bytes = align8(bytes + (size_t)o.S->t * o.S->nvars * 2);
    o.coff = bytes;
    bytes += (size_t)o.S->t * 8;
  }
  char* d_all = (char*)A.alloc<uint64_t>(std::max<size_t>(bytes / 8, 1));
  for (Out& o : outs) {
    cp.push_back(CopyJob{o.S->exps, d_all + o.eoff, (size_t)o.S->t * o.S->nvars * 2});
    cp.push_back(CopyJob{o.S->coef, d_all + o.coff, (size_t)o.S->t * 8});
  }
  batched_copy(cp, s);
  char* h = (char*)pinned(S, std::max<size_t>(bytes, 8));
  check(hipMemcpyAsync(h, d_all, std::max<size_t>(bytes, 8), hipMemcpyDeviceToHost, s));
  check(hipStreamSynchronize(s));
  for (Out& o : outs) {
    Request& r = *o.r;
    if (r.status != ZR_OK) continue;
    const uint32_t t = o.S->t, nv = o.S->nvars;
    zr_poly* out = o.dst;
    out->nvars = nv;
    out->nterms = t;
    out->exps = (uint16_t*)malloc(sizeof(uint16_t) * std::max<size_t>((size_t)t * nv, 1));
    out->coeffs = (uint64_t*)malloc(sizeof(uint64_t) * std::max<uint32_t>(t, 1));
    if (!out->exps || !out->coeffs) {
      fail(r, ZR_ENOMEM);
      continue;
    }
    const uint16_t* soa = (const uint16_t*)(h + o.eoff);
    for (uint32_t l = 0; l < t; ++l)
      for (uint32_t v = 0; v < nv; ++v) out->exps[(size_t)l * nv + v] = soa[(size_t)v * t + l];
    if (t) memcpy(out->coeffs, h + o.coff, (size_t)t * 8);
  }
}

// Bookkeeping of a request that ended: its slot, status word and footprint.
void retire(Server& S, Request& r) {
  r.finished = true;
  r.finished_step = S.steps;
  r.arena.reset();
  // every device use of the status word has been read back by now; a later
  // request clears it on the same stream before its first use
  S.free_status.push_back(r.d_status);
  r.d_status = nullptr;
  S.used -= r.footprint;
  r.footprint = 0;
  S.stats.completed += 1;
  if (r.status != ZR_OK) S.stats.failed += 1;
}

// Stage 1 of the balanced requests admitted at this step, all in one pass:
// each request's samples on x_1 (its own black-box call), one Thiele launch
// over all of them, one read-back of their degrees, statuses and coefficients,
// and one upload of the new skeletons, which are copied into each request's
// own arena.  Per request the arithmetic is that of balanced_stage1, which
// takes three host synchronisations and two uploads per request instead.
void stage1_batch(Server& S, const std::vector<Request*>& fresh, DevArena& A) {
  hipStream_t s = S.s;
  const size_t nf = fresh.size();
  std::vector<uint32_t> n1(nf);
  std::vector<std::vector<uint64_t>> X(nf);
  std::vector<size_t> xo(nf), co(nf);
  Blob xb;
  size_t cwords = 0;
  for (size_t q = 0; q < nf; ++q) {
    const Params& P = *fresh[q]->P;
    n1[q] = P.nnodes[0] + 1;
    X[q] = P.node_list(0, n1[q]);
    xo[q] = xb.add(X[q]);
    co[q] = cwords;  // A then B, n1 + 1 coefficients each
    cwords += 2 * ((size_t)n1[q] + 1);
  }
  char* dx = xb.upload(A, s);
  uint64_t* coef = A.alloc<uint64_t>(std::max<size_t>(cwords, 1));
  int32_t* flags = A.alloc<int32_t>(3 * nf);
  std::vector<ThieleJob> tj;
  std::vector<size_t> jq;  // fresh index of each job
  for (size_t q = 0; q < nf; ++q) {
    Request& r = *fresh[q];
    uint64_t* F = A.alloc<uint64_t>(n1[q]);
    const size_t sw = thiele_scratch_words(1, n1[q]);
    uint64_t* scr = sw ? A.alloc<uint64_t>(sw) : nullptr;
    try {
      call_bb(r.bb, r.ctx, *r.P, 1, 1, r.P->y.data(), X[q].data(), n1[q], F, s);
    } catch (const Error& e) {
      r.status = e.code;
      continue;
    }
    tj.push_back(ThieleJob{1, n1[q], (const uint64_t*)(dx + xo[q]), F, coef + co[q], coef + co[q] + n1[q] + 1,
                           flags + 3 * q, flags + 3 * q + 1, flags + 3 * q + 2, scr});
    jq.push_back(q);
  }
  if (tj.empty()) return;
  {
    uint32_t max_nk = 0;
    for (const ThieleJob& j : tj) max_nk = std::max(max_nk, j.nk);
    const uint32_t per = thiele_slices_per_block(max_nk);
    std::vector<uint32_t> tprefix{0};
    for (const ThieleJob& j : tj) tprefix.push_back(tprefix.back() + (j.T + per - 1) / per);
    Blob tb;
    const size_t oj = tb.add(tj), op = tb.add(tprefix);
    char* dt = tb.upload(A, s);
    check(thiele_slices_batch(S.M, (uint32_t)tj.size(), (const uint32_t*)(dt + op), tprefix.back(), max_nk,
                              (const ThieleJob*)(dt + oj), s));
  }
  std::vector<int32_t> hf(3 * nf);
  std::vector<uint64_t> hc(std::max<size_t>(cwords, 1));
  check(hipMemcpyAsync(hf.data(), flags, hf.size() * 4, hipMemcpyDeviceToHost, s));
  d2h_sync(hc.data(), coef, hc.size() * 8, s);
  // the skeletons of every request, uploaded together
  Blob sb;
  struct Put {
    size_t off;
    void* dst;
    size_t bytes;
  };
  std::vector<Put> puts;
  auto put = [&](const Params& P, const std::vector<uint64_t>& c, DevArena& keep, Skeleton& Sk) {
    std::vector<uint16_t> e;
    std::vector<uint64_t> cf, mo;
    const uint32_t t = stage1_skeleton_host(P, c, e, cf, mo);
    Sk.alloc(keep, P.nvars, t);
    if (!t) return;
    puts.push_back(Put{sb.add(e.data(), (size_t)P.nvars * t), Sk.exps, (size_t)P.nvars * t * 2});
    puts.push_back(Put{sb.add(cf.data(), t), Sk.coef, (size_t)t * 8});
    puts.push_back(Put{sb.add(mo.data(), t), Sk.mono, (size_t)t * 8});
  };
  for (size_t q : jq) {
    Request& r = *fresh[q];
    const Params& P = *r.P;
    int32_t rn, rd;
    try {
      check_slices({hf[3 * q + 2]}, {hf[3 * q]}, {hf[3 * q + 1]}, P.deg[0], P.deg_den[0], rn, rd);
    } catch (const Error& e) {
      r.status = e.code;
      continue;
    }
    const uint64_t* ca = hc.data() + co[q];
    const uint64_t* cb = ca + n1[q] + 1;
    r.arena = std::make_shared<DevArena>(s);
    put(P, std::vector<uint64_t>(ca, ca + rn + 1), *r.arena, r.SN);
    put(P, std::vector<uint64_t>(cb, cb + rd + 1), *r.arena, r.SD);
    r.k = 1;
  }
  if (!puts.empty()) {
    char* ds = sb.upload(A, s);
    std::vector<CopyJob> cp;
    for (const Put& u : puts) cp.push_back(CopyJob{ds + u.off, u.dst, u.bytes});
    batched_copy(cp, s);
  }
}

void advance(Server& S) {
  const zr_mod& M = S.M;
  hipStream_t s = S.s;
  DevArena A(s);
  std::vector<Request*> act;
  for (Request* r : S.active)
    if (r->status == ZR_OK) act.push_back(r);
  // ---- balanced requests at stage 1: univariate Thiele (small, per request);
  // they take part in the batched stages from the next step on
  std::vector<Request*> fresh;
  for (Request* r : act)
    if (r->balanced && r->k == 0) fresh.push_back(r);
  if (!fresh.empty()) stage1_batch(S, fresh, A);
  // ---- polynomial requests at stage 1 start from the constant skeleton
  {
    std::vector<uint32_t> nv;
    std::vector<Skeleton*> ptr;
    for (Request* r : act)
      if (!r->balanced && r->k == 0 && r->status == ZR_OK) {
        nv.push_back(r->P->nvars);
        ptr.push_back(&r->SN);
      }
    if (!ptr.empty()) {
      auto g = std::make_shared<DevArena>(s);
      constant_skeletons(*g, nv, ptr, S.p, s);
      for (Request* r : act)
        if (!r->balanced && r->k == 0 && r->status == ZR_OK) r->arena = g;
    }
  }
  // ---- balanced stage k >= 2, part 1: samples, per-slice Thiele, N and D at y^i
  struct Bal {
    Request* r;
    uint32_t kvar, T, nk;
    std::vector<uint64_t> X;
    uint64_t *dX, *F, *cA, *cB, *nprev, *dprev;
    int32_t *dgA, *dgB, *dst;
    size_t hoff;
    int32_t rhoN, rhoD;
  };
  std::vector<Bal> bal;
  for (Request* r : act) {
    if (!r->balanced || r->status != ZR_OK || r->k < 1 || r->k >= r->P->last) continue;
    if (std::find(fresh.begin(), fresh.end(), r) != fresh.end()) continue;
    Bal b;
    b.r = r;
    b.kvar = r->k;
    b.T = std::max(r->SN.t, r->SD.t);
    b.nk = r->P->nnodes[b.kvar] + 1;
    b.X = r->P->node_list(b.kvar, b.nk);
    bal.push_back(std::move(b));
  }
  std::vector<int32_t> hflags;
  if (!bal.empty()) {
    Blob xb;
    std::vector<size_t> xo;
    for (auto& b : bal) xo.push_back(xb.add(b.X));
    char* dxb = xb.upload(A, s);
    // every request's slice degrees and statuses in one device block, so that
    // one copy reads them back
    size_t hwords = 0;
    for (auto& b : bal) {
      b.hoff = hwords;
      hwords += 3 * (size_t)std::max<uint32_t>(b.T, 1);
    }
    int32_t* dflags = A.alloc<int32_t>(hwords);
    std::vector<ThieleJob> tj;
    std::vector<VapplyJob> vj;
    for (size_t q = 0; q < bal.size(); ++q) {
      Bal& b = bal[q];
      Request& r = *b.r;
      const uint32_t T1 = std::max<uint32_t>(b.T, 1);
      b.dX = (uint64_t*)(dxb + xo[q]);
      b.F = A.alloc<uint64_t>((size_t)b.nk * T1);
      b.cA = A.alloc<uint64_t>((size_t)(b.nk + 1) * T1);
      b.cB = A.alloc<uint64_t>((size_t)(b.nk + 1) * T1);
      b.dgA = dflags + b.hoff;
      b.dgB = b.dgA + T1;
      b.dst = b.dgB + T1;
      b.nprev = A.alloc<uint64_t>(T1);
      b.dprev = A.alloc<uint64_t>(T1);
      const size_t sw = thiele_scratch_words(b.T, b.nk);
      uint64_t* scr = sw ? A.alloc<uint64_t>(sw) : nullptr;
      try {
        call_bb(r.bb, r.ctx, *r.P, r.k + 1, b.T, r.P->y.data(), b.X.data(), b.nk, b.F, s);
      } catch (const Error& e) {
        r.status = e.code;
        continue;
      }
      // the slices of every request go through one Thiele launch below
      tj.push_back(ThieleJob{b.T, b.nk, b.dX, b.F, b.cA, b.cB, b.dgA, b.dgB, b.dst, scr});
      // N_{k-1} and D_{k-1} at y^i: applies of all requests go through two launches below
      vj.push_back(VapplyJob{r.SN.t, b.T, r.SN.mono, r.SN.coef, b.nprev,
                             A.alloc<uint64_t>(vapply_work_words(r.SN.t, b.T))});
      vj.push_back(VapplyJob{r.SD.t, b.T, r.SD.mono, r.SD.coef, b.dprev,
                             A.alloc<uint64_t>(vapply_work_words(r.SD.t, b.T))});
      counters().mulmods += (uint64_t)b.T * (r.SN.t + r.SD.t);
    }
    if (!vj.empty()) {
      std::vector<uint32_t> pre{0}, spre{0};
      for (const VapplyJob& j : vj) {
        pre.push_back(pre.back() + vapply_batch_blocks(j.t, j.T));
        spre.push_back(spre.back() + (j.T + 255) / 256);
      }
      Blob vb;
      const size_t oj = vb.add(vj), op = vb.add(pre), os = vb.add(spre);
      char* dv = vb.upload(A, s);
      check(vapply_batch(M, (uint32_t)vj.size(), (const uint32_t*)(dv + op), pre.back(), (const uint32_t*)(dv + os),
                         spre.back(), (const VapplyJob*)(dv + oj), s));
    }
    if (!tj.empty()) {
      uint32_t max_nk = 0;
      for (const ThieleJob& j : tj) max_nk = std::max(max_nk, j.nk);
      const uint32_t per = thiele_slices_per_block(max_nk);
      std::vector<uint32_t> tprefix{0};
      for (const ThieleJob& j : tj) tprefix.push_back(tprefix.back() + (j.T + per - 1) / per);
      Blob tb;
      const size_t oj = tb.add(tj), op = tb.add(tprefix);
      char* dt = tb.upload(A, s);
      check(thiele_slices_batch(M, (uint32_t)tj.size(), (const uint32_t*)(dt + op), tprefix.back(), max_nk,
                                (const ThieleJob*)(dt + oj), s));
    }
    // one read-back of every slice's degrees and status
    if (S.hcap < hwords) {
      if (S.hbuf) check(hipHostFree(S.hbuf));
      S.hbuf = nullptr;
      S.hcap = 0;
      check(hipHostMalloc((void**)&S.hbuf, std::max<size_t>(hwords, 1 << 16) * 4, hipHostMallocDefault));
      S.hcap = std::max<size_t>(hwords, 1 << 16);
    }
    int32_t* hbuf = S.hbuf;
    // (the blocks of requests whose black box failed are read too, and ignored)
    check(hipMemcpyAsync(hbuf, dflags, hwords * 4, hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    hflags.assign(hbuf, hbuf + hwords);
  }
  // ---- part 2: balanced right-hand sides; then every request's solve jobs
  std::vector<SolveJob> sj;
  std::vector<ConstsJob> cj;
  struct LiftPlan {
    Request* r;
    bool den;
    uint32_t kvar, D1;
    uint64_t* vals;
    std::vector<uint64_t> X;
  };
  std::vector<LiftPlan> lp;
  std::vector<BalanceJob> bj;
  std::vector<CopyJob> copies;
  for (auto& b : bal) {
    Request& r = *b.r;
    if (r.status != ZR_OK) continue;
    const uint32_t T1 = std::max<uint32_t>(b.T, 1);
    std::vector<int32_t> dA(hflags.begin() + b.hoff, hflags.begin() + b.hoff + b.T);
    std::vector<int32_t> dB(hflags.begin() + b.hoff + T1, hflags.begin() + b.hoff + T1 + b.T);
    std::vector<int32_t> st(hflags.begin() + b.hoff + 2 * T1, hflags.begin() + b.hoff + 2 * T1 + b.T);
    try {
      check_slices(st, dA, dB, r.P->deg[b.kvar], r.P->deg_den[b.kvar], b.rhoN, b.rhoD);
    } catch (const Error& e) {
      r.status = e.code;
      continue;
    }
    const uint32_t tN = r.SN.t, tD = r.SD.t;
    const uint32_t D1N = (uint32_t)b.rhoN + 1, D1D = (uint32_t)b.rhoD + 1;
    uint64_t* valsN = A.alloc<uint64_t>((size_t)D1N * std::max<uint32_t>(tN, 1));
    uint64_t* valsD = A.alloc<uint64_t>((size_t)D1D * std::max<uint32_t>(tD, 1));
    // row 0 of the Newton input is the previous skeleton; the balancing of all
    // requests runs in two launches below
    copies.push_back(CopyJob{r.SN.coef, valsN, (size_t)tN * 8});
    copies.push_back(CopyJob{r.SD.coef, valsD, (size_t)tD * 8});
    bj.push_back(BalanceJob{b.T, tN, tD, b.rhoN, b.rhoD, b.dX, b.cA, b.cB, b.dgA, b.dgB, b.nprev, b.dprev,
                            A.alloc<uint64_t>(T1), valsN + tN, tN, valsD + tD, tD, r.d_status});
    sj.push_back(SolveJob{tN, (uint32_t)b.rhoN, r.SN.mono, valsN + tN, r.d_status});
    sj.push_back(SolveJob{tD, (uint32_t)b.rhoD, r.SD.mono, valsD + tD, r.d_status});
    lp.push_back(LiftPlan{&r, false, b.kvar, D1N, valsN, std::vector<uint64_t>(b.X.begin(), b.X.begin() + D1N)});
    lp.push_back(LiftPlan{&r, true, b.kvar, D1D, valsD, std::vector<uint64_t>(b.X.begin(), b.X.begin() + D1D)});
  }
  if (!bj.empty()) {
    batched_copy(copies, s);
    std::vector<uint32_t> bpre{0}, rpre{0};
    for (const BalanceJob& j : bj) {
      bpre.push_back(bpre.back() + balance_beta_blocks(j.T));
      rpre.push_back(rpre.back() + balance_rhs_blocks(j.tN, j.tD, j.rhoN, j.rhoD));
    }
    Blob bb;
    const size_t oj = bb.add(bj), ob = bb.add(bpre), orh = bb.add(rpre);
    char* db = bb.upload(A, s);
    check(balance_batch(M, (uint32_t)bj.size(), (const uint32_t*)(db + ob), bpre.back(), (const uint32_t*)(db + orh),
                        rpre.back(), (const BalanceJob*)(db + oj), s));
  }
  // polynomial requests: samples at the Zippel points, then the same jobs
  for (Request* rp : act) {
    Request& r = *rp;
    if (r.balanced || r.status != ZR_OK || r.k >= r.P->last) continue;
    const uint32_t kvar = r.k, k = r.k + 1;
    const uint32_t D1 = r.P->deg[kvar] + 1, t = r.SN.t;
    std::vector<uint64_t> X = r.P->node_list(kvar, D1);
    uint64_t* vals = A.alloc<uint64_t>((size_t)D1 * std::max<uint32_t>(t, 1));
    try {
      if (k == 1) call_bb(r.bb, r.ctx, *r.P, 1, 1, r.P->y.data(), X.data(), D1, vals, s);
      else {
        check(copy_u64(vals, r.SN.coef, t, s));
        call_bb(r.bb, r.ctx, *r.P, k, t, r.P->y.data(), X.data() + 1, D1 - 1, vals + t, s);
      }
    } catch (const Error& e) {
      r.status = e.code;
      continue;
    }
    if (k > 1) sj.push_back(SolveJob{t, D1 - 1, r.SN.mono, vals + t, r.d_status});
    lp.push_back(LiftPlan{&r, false, kvar, D1, vals, std::move(X)});
  }
  // Newton matrices, solves, lifts of all requests
  std::vector<uint64_t*> cw(lp.size());
  for (size_t q = 0; q < lp.size(); ++q) {
    const uint32_t D1 = lp[q].D1;
    cw[q] = A.alloc<uint64_t>(newton_W_words(D1) / 2 + 2 + 2 * (size_t)D1);
    cj.push_back(ConstsJob{D1, lp[q].X.data(), lp[q].r->P->y[lp[q].kvar], (uint32_t*)cw[q],
                           cw[q] + newton_W_words(D1) / 2 + 1});
  }
  batched_consts(M, cj, s);
  batched_solve(M, sj, s);
  std::vector<LiftJob> lj;
  std::vector<Skeleton> nxt(lp.size());
  std::vector<size_t> lj_idx;
  for (size_t q = 0; q < lp.size(); ++q) {
    Request& r = *lp[q].r;
    if (r.status != ZR_OK) continue;
    lj.push_back(LiftJob{lp[q].kvar, lp[q].D1, lp[q].den ? &r.SD : &r.SN, lp[q].vals, cj[q].Wl, cj[q].ypow,
                         r.d_status, &nxt[q]});
    lj_idx.push_back(q);
  }
  auto g = std::make_shared<DevArena>(s);
  const std::vector<int32_t> lst = batched_lift(M, lj, *g, s);
  for (size_t u = 0; u < lj_idx.size(); ++u) {
    LiftPlan& L = lp[lj_idx[u]];
    Request& r = *L.r;
    if (lst[u] != 0 && r.status == ZR_OK) r.status = lst[u];
    (L.den ? r.SD : r.SN) = nxt[lj_idx[u]];
  }
  // requests that lifted advance; their skeletons now live in g
  for (size_t u = 0; u < lj_idx.size(); ++u) {
    Request& r = *lp[lj_idx[u]].r;
    if (r.arena != g) {
      r.arena = g;
      r.k += 1;
    }
  }
}

}  // namespace

}  // namespace zr

using namespace zr;

struct zr_server {
  Server impl;
};

extern "C" {

zr_status zr_server_create(zr_server** out, uint64_t p, uint64_t hbm_budget, uint32_t max_active,
                           hipStream_t stream) {
  if (!out || p < 3 || p >= ((uint64_t)1 << 63) || max_active == 0) return ZR_EINVAL;
  if (!is_prime_u64(p)) return ZR_ENOTPRIME;
  try {
    zr_server* srv = new zr_server();
    Server& S = srv->impl;
    S.s = stream;
    S.p = p;
    S.M = zr_mod_make(p);
    S.budget = hbm_budget;
    S.max_active = max_active;
    S.status_arena.reset(new DevArena(stream));
    *out = srv;
    return ZR_OK;
  } catch (const Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    return ZR_ENOMEM;
  }
}

void zr_server_destroy(zr_server* srv) {
  if (!srv) return;
  (void)hipStreamSynchronize(srv->impl.s);
  delete srv;
}

zr_status zr_server_submit(zr_server* srv, const zr_params* params, int balanced, uint64_t expected_terms,
                           zr_blackbox_fn bb, void* ctx, uint64_t* id) {
  if (!srv || !params || !bb || !id) return ZR_EINVAL;
  Server& S = srv->impl;
  try {
    std::unique_ptr<Request> r(new Request());
    r->P.reset(new Params(params, balanced != 0));
    if (r->P->p != S.p || r->P->first > 1) return ZR_EINVAL;
    r->balanced = balanced != 0;
    r->bb = bb;
    r->ctx = ctx;
    r->cap = expected_terms ? expected_terms : monomial_count(*r->P);
    r->footprint = stage_footprint(*r->P, r->balanced, 0, 1, 1, r->cap);
    r->id = S.next_id++;
    if (!S.free_status.empty()) {
      r->d_status = S.free_status.back();
      S.free_status.pop_back();
    } else {
      r->d_status = S.status_arena->alloc<int32_t>(1);
    }
    check(fill_i32(r->d_status, 0, 1, S.s));
    *id = r->id;
    S.waiting.insert(r->id);
    S.pending.push_back(r.release());
    S.stats.submitted += 1;
    return ZR_OK;
  } catch (const Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    return ZR_ENOMEM;
  }
}

zr_status zr_server_step(zr_server* srv, uint32_t* n_active, uint32_t* n_pending, uint32_t* n_finished) {
  if (!srv) return ZR_EINVAL;
  Server& S = srv->impl;
  uint32_t fin = 0;
  try {
    // admission: first come, first served, while slots and the budget allow
    // (a request larger than the budget still runs when nothing else does)
    while (!S.pending.empty() && S.active.size() < S.max_active) {
      Request* r = S.pending.front();
      if (!S.active.empty() && S.used + r->footprint > S.budget) break;
      S.pending.pop_front();
      S.used += r->footprint;
      r->admitted_step = S.steps;
      S.active.push_back(r);
      S.stats.admitted += 1;
    }
    S.stats.peak_footprint = std::max(S.stats.peak_footprint, S.used);
    S.stats.peak_active = std::max<uint64_t>(S.stats.peak_active, S.active.size());
    if (!S.active.empty()) {
      advance(S);
      S.steps += 1;
      S.stats.steps = S.steps;
      std::vector<Request*> keep, ended;
      for (Request* r : S.active)
        if (r->status != ZR_OK || r->k >= r->P->last) ended.push_back(r);
      if (!ended.empty()) finish_batch(S, ended);
      for (Request* r : S.active) {
        if (r->status != ZR_OK || r->k >= r->P->last) {
          retire(S, *r);
          S.done[r->id] = r;
          S.waiting.erase(r->id);
          S.newly_done.push_back(r->id);
          // a caller that only polls never drains the list: drop the ids
          // already collected once they outnumber the uncollected ones
          if (S.newly_done.size() > 2 * S.done.size() + 4096) {
            std::vector<uint64_t> keep_ids;
            for (uint64_t x : S.newly_done)
              if (S.done.count(x)) keep_ids.push_back(x);
            S.newly_done.swap(keep_ids);
          }
          ++fin;
        } else {
          // the next stage's estimate from the skeletons just built
          S.used -= r->footprint;
          r->footprint = stage_footprint(*r->P, r->balanced, r->k, r->SN.t, r->SD.t, r->cap);
          S.used += r->footprint;
          keep.push_back(r);
        }
      }
      S.active.swap(keep);
      S.stats.peak_footprint = std::max(S.stats.peak_footprint, S.used);
    }
  } catch (const Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    return ZR_ENOMEM;
  }
  if (n_active) *n_active = (uint32_t)S.active.size();
  if (n_pending) *n_pending = (uint32_t)S.pending.size();
  if (n_finished) *n_finished = fin;
  return ZR_OK;
}

int zr_server_poll(zr_server* srv, uint64_t id, int32_t* status, zr_poly* num, zr_poly* den) {
  if (!srv) return ZR_EINVAL;
  Server& S = srv->impl;
  auto it = S.done.find(id);
  if (it == S.done.end()) return S.waiting.count(id) ? 1 : ZR_EINVAL;
  Request* r = it->second;
  if (status) *status = r->status;
  if (num) *num = r->num;
  else zr_poly_free(&r->num);
  if (den) *den = r->den;
  else zr_poly_free(&r->den);
  S.done.erase(it);
  delete r;
  return 0;
}

uint32_t zr_server_finished(zr_server* srv, uint64_t* ids, uint32_t cap) {
  if (!srv || (!ids && cap)) return 0;
  Server& S = srv->impl;
  // ids already collected through zr_server_poll are skipped
  uint32_t n = 0;
  size_t i = 0;
  for (; i < S.newly_done.size() && n < cap; ++i)
    if (S.done.count(S.newly_done[i])) ids[n++] = S.newly_done[i];
  S.newly_done.erase(S.newly_done.begin(), S.newly_done.begin() + i);
  return n;
}

zr_status zr_server_get_stats(zr_server* srv, zr_server_stats* out) {
  if (!srv || !out) return ZR_EINVAL;
  *out = srv->impl.stats;
  out->footprint = srv->impl.used;
  out->active = srv->impl.active.size();
  out->pending = srv->impl.pending.size();
  return ZR_OK;
}

}  // extern "C"
