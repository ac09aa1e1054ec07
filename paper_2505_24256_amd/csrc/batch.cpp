// Batched entry points: vandermonde_solve_batch (many transposed Vandermonde
// systems, §1 and §2.2) and zippel_reconstruct_batch (many polynomial Zippel
// reconstructions advanced stage by stage together, §1).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <memory>
#include <vector>

#include "../../include/zippel.h"
#include "batch.hpp"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"

namespace zr {

static void solve_batch(size_t nsys, uint64_t p, const uint64_t* h_sys_off, const uint64_t* d_mono,
                        const uint32_t* h_nrhs, const uint64_t* h_rhs_off, const uint64_t* d_rhs, uint64_t* d_out,
                        int32_t* d_status, hipStream_t s) {
  const zr_mod M = zr_mod_make(p);
  // graphs of earlier asynchronous calls on this stream: destroyed once it is idle
  if (hipStreamQuery(s) == hipSuccess) release_graphs(s);
  check(fill_i32(d_status, 0, nsys, s));
  if (h_rhs_off[nsys])
    check(hipMemcpyAsync(d_out, d_rhs, h_rhs_off[nsys] * 8, hipMemcpyDeviceToDevice, s));
  std::vector<SolveJob> jobs;
  jobs.reserve(nsys);
  for (size_t i = 0; i < nsys; ++i) {
    const uint32_t t = (uint32_t)(h_sys_off[i + 1] - h_sys_off[i]);
    jobs.push_back(SolveJob{t, h_nrhs[i], d_mono + h_sys_off[i], d_out + h_rhs_off[i], d_status + i});
  }
  batched_solve(M, jobs, s);
}

// ---------------------------------------------------------------------------
// batched polynomial Zippel

// The constant polynomial 1 as a skeleton for each of out.size() instances
// (stage-0 skeletons), all in one block of A.
void constant_skeletons(DevArena& A, const std::vector<uint32_t>& nvars, const std::vector<Skeleton*>& out,
                        uint64_t p, hipStream_t s) {
  const size_t n = out.size();
  std::vector<uint64_t> host;
  std::vector<size_t> off(n);
  for (size_t i = 0; i < n; ++i) {
    off[i] = host.size();
    host.resize(host.size() + 2 + (nvars[i] + 3) / 4, 0);
    host[off[i]] = 1 % p;
    host[off[i] + 1] = 1 % p;
  }
  Blob b;
  const size_t o = b.add(host);
  uint64_t* d = (uint64_t*)(b.upload(A, s) + o);
  for (size_t i = 0; i < n; ++i) {
    Skeleton& S = *out[i];
    S.nvars = nvars[i];
    S.t = 1;
    S.coef = d + off[i];
    S.mono = d + off[i] + 1;
    S.exps = (uint16_t*)(d + off[i] + 2);
  }
}

namespace {

struct Gen {  // one step's skeletons, alive while an instance refers to them
  std::unique_ptr<DevArena> arena;
  explicit Gen(hipStream_t s) : arena(new DevArena(s)) {}
};

}  // namespace

static void reconstruct_batch(uint32_t n, const zr_params* params, zr_blackbox_fn bb, void* const* ctx,
                              hipStream_t s, zr_poly* out, int32_t* st) {
  std::vector<std::unique_ptr<Params>> P(n);
  uint64_t p = 0;
  for (uint32_t i = 0; i < n; ++i) {
    try {
      P[i].reset(new Params(&params[i], false));
      if (P[i]->first > 1) throw Error(ZR_EINVAL);  // resumption is a one-reconstruction feature
      st[i] = ZR_OK;
    } catch (const Error& e) {
      st[i] = e.code;
      continue;
    }
    if (p == 0) p = P[i]->p;
    else if (P[i]->p != p) throw Error(ZR_EINVAL);
  }
  counters() = zr_counters{};
  if (p == 0) return;
  const zr_mod M = P[0] ? P[0]->M : zr_mod_make(p);
  DevArena keep(s);
  int32_t* d_status = keep.alloc<int32_t>(n);
  check(fill_i32(d_status, 0, n, s));
  // stage-0 skeletons: the constant 1
  std::vector<Skeleton> cur(n);
  std::vector<std::shared_ptr<Gen>> gen(n);
  {
    auto g0 = std::make_shared<Gen>(s);
    std::vector<uint32_t> nv;
    std::vector<Skeleton*> ptr;
    for (uint32_t i = 0; i < n; ++i) {
      if (st[i] != ZR_OK) continue;
      nv.push_back(P[i]->nvars);
      ptr.push_back(&cur[i]);
      gen[i] = g0;
    }
    constant_skeletons(*g0->arena, nv, ptr, p, s);
  }
  uint32_t kmax = 0;
  for (uint32_t i = 0; i < n; ++i)
    if (st[i] == ZR_OK) kmax = std::max(kmax, P[i]->last);
  for (uint32_t k = 1; k <= kmax; ++k) {
    const uint32_t kvar = k - 1;
    std::vector<uint32_t> live;
    for (uint32_t i = 0; i < n; ++i)
      if (st[i] == ZR_OK && P[i]->last >= k) live.push_back(i);
    if (live.empty()) break;
    DevArena A(s);
    const size_t nl = live.size();
    // per-instance stage constants and value tables
    std::vector<uint32_t> D1(nl);
    std::vector<std::vector<uint64_t>> X(nl);
    size_t vwords = 0, wwords = 0;
    std::vector<size_t> voff(nl), woff(nl);
    for (size_t q = 0; q < nl; ++q) {
      const Params& Pi = *P[live[q]];
      D1[q] = Pi.deg[kvar] + 1;
      X[q] = Pi.node_list(kvar, D1[q]);
      voff[q] = vwords;
      vwords += ((size_t)D1[q] * std::max<uint32_t>(cur[live[q]].t, 1) + 31) & ~(size_t)31;
      woff[q] = wwords;
      wwords += (newton_W_words(D1[q]) / 2 + 1 + 2 * D1[q] + 31) & ~(size_t)31;
    }
    uint64_t* vals = A.alloc<uint64_t>(std::max<size_t>(vwords, 1));
    uint64_t* cw = A.alloc<uint64_t>(std::max<size_t>(wwords, 1));
    std::vector<ConstsJob> cj(nl);
    for (size_t q = 0; q < nl; ++q) {
      uint32_t* Wl = (uint32_t*)(cw + woff[q]);
      uint64_t* ypow = cw + woff[q] + newton_W_words(D1[q]) / 2 + 1;
      cj[q] = ConstsJob{D1[q], X[q].data(), P[live[q]]->y[kvar], Wl, ypow};
    }
    batched_consts(M, cj, s);
    // samples: row 0 = current coefficients (values at the anchor), rows 1.. from the black box
    if (k > 1) {
      std::vector<CopyJob> cp;
      for (size_t q = 0; q < nl; ++q) {
        const Skeleton& S = cur[live[q]];
        cp.push_back(CopyJob{S.coef, vals + voff[q], (size_t)S.t * 8});
      }
      batched_copy(cp, s);
    }
    for (size_t q = 0; q < nl; ++q) {
      const uint32_t i = live[q];
      const Params& Pi = *P[i];
      try {
        if (k == 1) call_bb(bb, ctx ? ctx[i] : nullptr, Pi, 1, 1, Pi.y.data(), X[q].data(), D1[q], vals + voff[q], s);
        else
          call_bb(bb, ctx ? ctx[i] : nullptr, Pi, k, cur[i].t, Pi.y.data(), X[q].data() + 1, D1[q] - 1,
                  vals + voff[q] + cur[i].t, s);
      } catch (const Error& e) {
        st[i] = e.code;
      }
    }
    std::vector<SolveJob> sj;
    std::vector<LiftJob> lj;
    std::vector<uint32_t> lj_inst;
    std::vector<Skeleton> nxt(nl);
    for (size_t q = 0; q < nl; ++q) {
      const uint32_t i = live[q];
      if (st[i] != ZR_OK) continue;
      if (k > 1) sj.push_back(SolveJob{cur[i].t, D1[q] - 1, cur[i].mono, vals + voff[q] + cur[i].t, d_status + i});
      lj.push_back(LiftJob{kvar, D1[q], &cur[i], vals + voff[q], cj[q].Wl, cj[q].ypow, d_status + i, &nxt[q]});
      lj_inst.push_back(i);
    }
    batched_solve(M, sj, s);
    auto g = std::make_shared<Gen>(s);
    const std::vector<int32_t> lst = batched_lift(M, lj, *g->arena, s);
    for (size_t q = 0, r = 0; q < nl; ++q) {
      const uint32_t i = live[q];
      if (r < lj_inst.size() && lj_inst[r] == i) {
        if (lst[r] != 0) st[i] = lst[r];
        cur[i] = nxt[q];
        gen[i] = g;
        ++r;
      }
    }
  }
  // probes: black-box values and evaluations of the results, one read-back
  {
    DevArena A(s);
    std::vector<EvalJob> ej;
    std::vector<uint32_t> owner;
    std::vector<size_t> toff;
    std::vector<uint32_t> lds;
    size_t np_total = 0;
    for (uint32_t i = 0; i < n; ++i)
      if (st[i] == ZR_OK && P[i]->last == P[i]->nvars) np_total += P[i]->nprobes;
    uint64_t* d_res = A.alloc<uint64_t>(2 * std::max<size_t>(np_total, 1));
    // the probe points go up once; their power tables are built on the device
    Blob pb;
    std::vector<size_t> poff(n, 0);
    size_t twords = 0;
    for (uint32_t i = 0; i < n; ++i)
      if (st[i] == ZR_OK && P[i]->last == P[i]->nvars && P[i]->nprobes) poff[i] = pb.add(P[i]->probes);
    char* dpts = pb.upload(A, s);
    std::vector<PowJob> pj;
    size_t pi = 0;
    for (uint32_t i = 0; i < n; ++i) {
      if (st[i] != ZR_OK || P[i]->last != P[i]->nvars) continue;
      const Params& Pi = *P[i];
      const uint32_t nv = Pi.nvars;
      uint32_t ld = 1;
      for (uint32_t v = 0; v < nv; ++v) ld = std::max(ld, Pi.deg[v] + 1);
      for (uint32_t q = 0; q < Pi.nprobes; ++q, ++pi) {
        const uint64_t* pt = Pi.probes.data() + (size_t)q * nv;
        try {
          call_bb(bb, ctx ? ctx[i] : nullptr, Pi, nv, 1, pt, pt + (nv - 1), 1, d_res + pi, s);
        } catch (const Error& e) {
          st[i] = e.code;
        }
        toff.push_back(twords);
        lds.push_back(ld);
        pj.push_back(PowJob{(const uint64_t*)(dpts + poff[i]) + (size_t)q * nv, nullptr, nv, ld});
        twords += (size_t)nv * ld;
        owner.push_back(i);
      }
    }
    if (pi) {
      uint64_t* tabs = A.alloc<uint64_t>(twords);
      for (size_t q = 0; q < pi; ++q) pj[q].tab = tabs + toff[q];
      batched_power_tables(M, pj, s);
      for (size_t q = 0; q < pi; ++q) ej.push_back(EvalJob{&cur[owner[q]], tabs + toff[q], lds[q], d_res + pi + q});
      batched_eval(M, ej, s);
      std::vector<uint64_t> r(2 * pi);
      d2h_sync(r.data(), d_res, r.size() * 8, s);
      for (size_t q = 0; q < pi; ++q)
        if (st[owner[q]] == ZR_OK && r[q] != r[pi + q]) st[owner[q]] = ZR_EPROBE;
    }
  }
  // results: gather every successful skeleton into one buffer, one read-back
  {
    DevArena A(s);
    std::vector<CopyJob> cp;
    std::vector<size_t> off(n, 0);
    size_t words = 0;
    for (uint32_t i = 0; i < n; ++i) {
      if (st[i] != ZR_OK) continue;
      const Skeleton& S = cur[i];
      off[i] = words;
      words += S.t + ((size_t)S.nvars * S.t + 3) / 4;
    }
    uint64_t* d = A.alloc<uint64_t>(std::max<size_t>(words, 1));
    // coefficients as they are, exponents turned term-major on the device
    std::vector<TransposeJob> tr;
    for (uint32_t i = 0; i < n; ++i) {
      if (st[i] != ZR_OK) continue;
      const Skeleton& S = cur[i];
      cp.push_back(CopyJob{S.coef, d + off[i], (size_t)S.t * 8});
      tr.push_back(TransposeJob{S.exps, (uint16_t*)(d + off[i] + S.t), S.t, S.nvars});
    }
    batched_copy(cp, s);
    batched_exps_to_terms(tr, s);
    std::unique_ptr<uint64_t[]> h(new uint64_t[std::max<size_t>(words, 1)]);  // filled by the copy: no zeroing
    d2h_sync(h.get(), d, words * 8, s);
    for (uint32_t i = 0; i < n; ++i) {
      if (st[i] != ZR_OK) continue;
      const Skeleton& S = cur[i];
      zr_poly& o = out[i];
      o.nvars = S.nvars;
      o.nterms = S.t;
      o.exps = (uint16_t*)malloc(sizeof(uint16_t) * std::max<size_t>((size_t)S.t * S.nvars, 1));
      o.coeffs = (uint64_t*)malloc(sizeof(uint64_t) * std::max<uint32_t>(S.t, 1));
      if (!o.exps || !o.coeffs) {
        free(o.exps);
        free(o.coeffs);
        o.exps = nullptr;
        o.coeffs = nullptr;
        st[i] = ZR_ENOMEM;
        continue;
      }
      memcpy(o.coeffs, h.get() + off[i], (size_t)S.t * 8);
      memcpy(o.exps, h.get() + off[i] + S.t, (size_t)S.t * S.nvars * 2);
    }
  }
}

}  // namespace zr

using namespace zr;

extern "C" {

zr_status vandermonde_solve_batch(size_t nsys, uint64_t p, const uint64_t* d_sys_off, const uint64_t* h_sys_off,
                                  const uint64_t* d_mono, const uint32_t* h_nrhs, const uint64_t* d_rhs_off,
                                  const uint64_t* h_rhs_off, const uint64_t* d_rhs, uint64_t* d_out,
                                  int32_t* d_status, hipStream_t stream) {
  (void)d_sys_off;
  (void)d_rhs_off;
  if (nsys == 0) return ZR_OK;
  if (p < 3 || p >= ((uint64_t)1 << 63) || !h_sys_off || !h_nrhs || !h_rhs_off || !d_status) return ZR_EINVAL;
  if (!is_prime_u64(p)) return ZR_ENOTPRIME;
  for (size_t i = 0; i < nsys; ++i) {
    if (h_sys_off[i + 1] < h_sys_off[i]) return ZR_EINVAL;
    const uint64_t t = h_sys_off[i + 1] - h_sys_off[i];
    if (t >= ((uint64_t)1 << 31)) return ZR_EINVAL;
    if (h_rhs_off[i + 1] < h_rhs_off[i] || h_rhs_off[i + 1] - h_rhs_off[i] != t * h_nrhs[i]) return ZR_EINVAL;
  }
  if (h_sys_off[nsys] && (!d_mono || !d_rhs || !d_out)) return ZR_EINVAL;
  try {
    solve_batch(nsys, p, h_sys_off, d_mono, h_nrhs, h_rhs_off, d_rhs, d_out, d_status, stream);
    return ZR_OK;
  } catch (const Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    note_error("host allocation failed");
    return ZR_ENOMEM;
  } catch (...) {
    note_error("unexpected exception");
    return ZR_EDEVICE;
  }
}

// Whole-batch failure: no outputs, every instance carries the error.
static void fail_all(uint32_t n, zr_poly* out, int32_t* status, int code) {
  for (uint32_t i = 0; i < n; ++i) {
    zr_poly_free(&out[i]);
    status[i] = code;
  }
}

zr_status zippel_reconstruct_batch(uint32_t n, const zr_params* params, zr_blackbox_fn bb, void* const* ctx,
                                   hipStream_t stream, zr_poly* out, int32_t* status) {
  if (n == 0) return ZR_OK;
  if (!params || !bb || !out || !status) return ZR_EINVAL;
  for (uint32_t i = 0; i < n; ++i) out[i] = zr_poly{0, 0, nullptr, nullptr};
  try {
    reconstruct_batch(n, params, bb, ctx, stream, out, status);
    return ZR_OK;
  } catch (const Error& e) {
    fail_all(n, out, status, e.code);
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    note_error("host allocation failed");
    fail_all(n, out, status, ZR_ENOMEM);
    return ZR_ENOMEM;
  } catch (...) {
    note_error("unexpected exception");
    fail_all(n, out, status, ZR_EDEVICE);
    return ZR_EDEVICE;
  }
}

zr_status zr_autotune(uint64_t p, hipStream_t stream, zr_band_choice* table) {
  if (p < 3 || p >= ((uint64_t)1 << 63)) return ZR_EINVAL;
  if (!is_prime_u64(p)) return ZR_ENOTPRIME;
  try {
    autotune(zr_mod_make(p), stream);
  } catch (const Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    note_error("host allocation failed");
    return ZR_ENOMEM;
  } catch (...) {
    note_error("unexpected exception");
    return ZR_EDEVICE;
  }
  if (table) zr_tuning_get(table);
  return ZR_OK;
}

void zr_batch_graphs(int on) { set_graphs(on != 0); }

int zr_tuning_get(zr_band_choice* table) {
  const Tuning& T = tuning();
  if (table)
    for (int b = 0; b < kBands; ++b) table[b] = zr_band_choice{T.band[b].packed, T.band[b].min_chunk};
  return T.tuned ? 1 : 0;
}

zr_status zr_tuning_set(const zr_band_choice* table) {
  if (!table) return ZR_EINVAL;
  Tuning& T = tuning();
  for (int b = 0; b < kBands; ++b) {
    if (table[b].min_chunk == 0) return ZR_EINVAL;
    T.band[b] = BandTuning{table[b].packed ? 1u : 0u, table[b].min_chunk};
  }
  return ZR_OK;
}

}  // extern "C"
