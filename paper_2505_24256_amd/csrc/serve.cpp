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

#include <algorithm>
#include <deque>
#include <map>
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
  zr_server_stats stats{};
  int32_t* hbuf = nullptr;  // pinned read-back buffer
  size_t hcap = 0;
  ~Server() {
    if (hbuf) (void)hipHostFree(hbuf);
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

void finish(Server& S, Request& r) {
  if (r.status == ZR_OK) {
    try {
      if (r.balanced) {
        balanced_finish(*r.P, r.bb, r.ctx, r.SN, r.SD, S.s, &r.num, &r.den);
      } else {
        if (r.P->last == r.P->nvars && r.P->nprobes) check_probes(*r.P, r.bb, r.ctx, r.SN, nullptr, S.s);
        download(r.SN, S.s, &r.num);
      }
    } catch (const Error& e) {
      zr_poly_free(&r.num);
      zr_poly_free(&r.den);
      r.status = e.code;
    }
  }
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

// One stage for every active request (stage r.k + 1).
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
  for (Request* r : act) {
    if (!r->balanced || r->k != 0) continue;
    try {
      r->arena = std::make_shared<DevArena>(s);
      balanced_stage1(*r->P, r->bb, r->ctx, *r->arena, r->SN, r->SD, s);
      r->k = 1;
    } catch (const Error& e) {
      r->status = e.code;
    }
    fresh.push_back(r);
  }
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
    size_t hwords = 0;
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
      b.dgA = A.alloc<int32_t>(3 * (size_t)T1);
      b.dgB = b.dgA + T1;
      b.dst = b.dgB + T1;
      b.nprev = A.alloc<uint64_t>(T1);
      b.dprev = A.alloc<uint64_t>(T1);
      const size_t sw = thiele_scratch_words(b.T, b.nk);
      uint64_t* scr = sw ? A.alloc<uint64_t>(sw) : nullptr;
      b.hoff = hwords;
      hwords += 3 * (size_t)T1;
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
    for (auto& b : bal)
      if (b.r->status == ZR_OK)
        check(hipMemcpyAsync(hbuf + b.hoff, b.dgA, 3 * (size_t)std::max<uint32_t>(b.T, 1) * 4,
                             hipMemcpyDeviceToHost, s));
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
      std::vector<Request*> keep;
      for (Request* r : S.active) {
        if (r->status != ZR_OK || r->k >= r->P->last) {
          finish(S, *r);
          S.done[r->id] = r;
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
  if (it == S.done.end()) {
    for (Request* r : S.pending)
      if (r->id == id) return 1;
    for (Request* r : S.active)
      if (r->id == id) return 1;
    return ZR_EINVAL;
  }
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

zr_status zr_server_get_stats(zr_server* srv, zr_server_stats* out) {
  if (!srv || !out) return ZR_EINVAL;
  *out = srv->impl.stats;
  out->footprint = srv->impl.used;
  out->active = srv->impl.active.size();
  out->pending = srv->impl.pending.size();
  return ZR_OK;
}

}  // extern "C"
