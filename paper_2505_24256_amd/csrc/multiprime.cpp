// Host driver of the reconstruction over several primes (§1: rational numbers
// are recovered from the modular results as the last step; §2.2: the
// multi-prime Zippel routine) and its C ABI.  The first prime runs the full
// Zippel reconstruction and fixes the term set; every further prime costs one
// black-box call at the t Zippel points of all variables and one transposed
// Vandermonde solve with a single right-hand side; after each prime the
// fractions reconstructed from the primes so far are tested against the next
// prime's residues and accepted when all of them agree.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/zippel.h"
#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"
#include "multiprime.hpp"

namespace zr {
namespace {

// Prime range of the multi-prime path: the mixed-radix digits of Garner's
// method are reduced into [0, p_j) by one subtraction, which needs every
// prime above 2^62.
bool mp_prime_ok(uint64_t p) { return p > ((uint64_t)1 << 62) && p < ((uint64_t)1 << 63) && is_prime_u64(p); }

MpConsts mp_consts(const std::vector<uint64_t>& primes) {
  MpConsts C;
  memset(&C, 0, sizeof(C));
  C.J = (uint32_t)primes.size();
  for (uint32_t j = 0; j < C.J; ++j) {
    const zr_mod Mj = zr_mod_make(primes[j]);
    C.mod[j] = Mj;
    uint64_t prod = 1 % Mj.p;
    for (uint32_t i = 0; i < j; ++i) {
      C.pmod[j][i] = primes[i] % Mj.p;
      prod = zr_mul(Mj, prod, C.pmod[j][i]);
    }
    C.cinv[j] = zr_inv(Mj, prod);
  }
  // P = product of the primes, little-endian words
  C.P[0] = 1;
  uint32_t used = 1;
  for (uint32_t j = 0; j < C.J; ++j) {
    uint64_t carry = 0;
    for (uint32_t i = 0; i < used; ++i) {
      const zr_u128 pr = (zr_u128)C.P[i] * primes[j] + carry;
      C.P[i] = (uint64_t)pr;
      carry = (uint64_t)(pr >> 64);
    }
    if (carry) C.P[used++] = carry;
  }
  uint32_t bits = 0;
  for (int i = kMpWords - 1; i >= 0; --i)
    if (C.P[i]) {
      bits = 64 * i + 64 - __builtin_clzll(C.P[i]);
      break;
    }
  C.e = bits >= 2 ? (bits - 2) / 2 : 0;
  C.nw = std::max<uint32_t>(1, (C.e + 63) / 64);
  return C;
}

// Monomial values over all nvars variables at the bases y, for exponents SoA
// [nvars][t] on the device: per-variable power tables built on the host.
void all_variable_monomials(const zr_mod& M, uint32_t nvars, uint32_t t, const uint16_t* d_exps,
                            const std::vector<uint32_t>& maxe, const uint64_t* y, DevArena& A, uint64_t* mono,
                            hipStream_t s) {
  MonoTables T{};
  std::vector<uint64_t> tabs;
  for (uint32_t v = 0; v < nvars; ++v) {
    T.off[v] = (uint32_t)tabs.size();
    uint64_t acc = 1 % M.p;
    for (uint32_t d = 0; d <= maxe[v]; ++d) {
      tabs.push_back(acc);
      acc = zr_mul(M, acc, y[v]);
    }
  }
  uint64_t* d_tabs = A.alloc<uint64_t>(tabs.size());
  h2d(d_tabs, tabs.data(), tabs.size() * 8, s);
  check(mono_values(M, t, nvars, d_exps, t, d_tabs, T, mono, s));
  check(hipStreamSynchronize(s));  // the host tables above are released on return
}

// Coefficients modulo M.p of the terms d_exps from samples at the Zippel
// points of all variables (d_vals[i-1] at x_v = y_v^i, i = 1..t).
void skeleton_solve(const zr_mod& M, uint32_t nvars, uint32_t t, const uint16_t* d_exps,
                    const std::vector<uint32_t>& maxe, const uint64_t* y, const uint64_t* d_vals, uint64_t* d_out,
                    int32_t* d_status, hipStream_t s) {
  if (t == 0) return;
  DevArena A(s);
  uint64_t* mono = A.alloc<uint64_t>(t);
  all_variable_monomials(M, nvars, t, d_exps, maxe, y, A, mono, s);
  uint64_t* Mc = A.alloc<uint64_t>(t);
  uint64_t* tmp = A.alloc<uint64_t>(master_tmp_words(t));
  check(master_poly(M, t, mono, Mc, tmp, s));
  const MpSolvePlan plan = mp_solve_plan(t);
  uint64_t* work = A.alloc<uint64_t>(mp_solve_words(plan));
  check(mp_solve(M, plan, mono, Mc, d_vals, d_out, work, d_status, s));
  count_solve(t, 1);
}

std::vector<uint32_t> max_exponents(uint32_t nvars, uint64_t t, const uint16_t* h_exps) {
  std::vector<uint32_t> maxe(nvars, 0);
  for (uint64_t l = 0; l < t; ++l)
    for (uint32_t v = 0; v < nvars; ++v) maxe[v] = std::max<uint32_t>(maxe[v], h_exps[l * nvars + v]);
  return maxe;
}

uint16_t* upload_exps_soa(uint32_t nvars, uint32_t t, const uint16_t* h_exps, DevArena& A, hipStream_t s) {
  std::vector<uint16_t> soa((size_t)nvars * t);
  for (uint32_t l = 0; l < t; ++l)
    for (uint32_t v = 0; v < nvars; ++v) soa[(size_t)v * t + l] = h_exps[(size_t)l * nvars + v];
  uint16_t* d = A.alloc<uint16_t>(std::max<size_t>(soa.size(), 1));
  h2d(d, soa.data(), soa.size() * 2, s);
  check(hipStreamSynchronize(s));
  return d;
}

void reconstruct_rational(const zr_params* params, const uint64_t* primes, uint32_t nprimes, zr_blackbox_fn bb,
                          void* ctx, hipStream_t s, zr_qpoly* out) {
  if (!params || !bb || (nprimes && !primes) || 1 + nprimes > kMpMaxPrimes) throw Error(ZR_EINVAL);
  // the term set must be that of the whole polynomial
  if ((params->last_stage && params->last_stage != params->nvars) || params->first_stage > 1) throw Error(ZR_EINVAL);
  std::vector<uint64_t> all{params->p};
  for (uint32_t j = 0; j < nprimes; ++j) all.push_back(primes[j]);
  for (size_t j = 0; j < all.size(); ++j) {
    if (!mp_prime_ok(all[j])) {
      note_error("prime %zu of the multi-prime reconstruction is not a prime in (2^62, 2^63)", j);
      throw Error(is_prime_u64(all[j]) || all[j] >= ((uint64_t)1 << 63) ? ZR_EINVAL : ZR_ENOTPRIME);
    }
    for (size_t i = 0; i < j; ++i)
      if (all[i] == all[j]) throw Error(ZR_EINVAL);
  }
  // first prime: the full reconstruction fixes the term set
  zr_poly first{};
  {
    const zr_status st = zippel_reconstruct(params, bb, ctx, s, &first);
    if (st != ZR_OK) throw Error(st);
  }
  struct PolyGuard {
    zr_poly* p;
    ~PolyGuard() { zr_poly_free(p); }
  } guard{&first};
  const uint32_t n = first.nvars, t = (uint32_t)first.nterms;
  DevArena A(s);
  const uint16_t* d_exps = upload_exps_soa(n, t, first.exps, A, s);
  const std::vector<uint32_t> maxe = max_exponents(n, t, first.exps);
  const size_t tt = std::max<uint32_t>(t, 1);
  uint64_t* res = A.alloc<uint64_t>(kMpMaxPrimes * tt);
  uint64_t* num = A.alloc<uint64_t>(kMpWords * tt);
  uint64_t* den = A.alloc<uint64_t>(kMpWords * tt);
  uint32_t* neg = A.alloc<uint32_t>(tt);
  uint64_t* vals = A.alloc<uint64_t>(tt);
  int32_t* d_cnt = A.alloc<int32_t>(4);  // [0] solve status, [1] reconstruction failures, [2] mismatches
  h2d(res, first.coeffs, (size_t)t * 8, s);
  std::vector<uint64_t> used{all[0]};
  MpConsts C = mp_consts(used);
  check(fill_i32(d_cnt, 0, 4, s));
  check(mp_crt_rr(C, t, res, num, den, neg, (uint32_t*)d_cnt + 1, s));
  uint32_t confirmed = 0;
  int32_t* h = host_scratch();
  for (uint32_t j = 1; j < all.size() && !confirmed; ++j) {
    const uint64_t q = all[j];
    const zr_mod Mq = zr_mod_make(q);
    std::vector<uint64_t> y(n), anchor(n, 0);
    std::vector<uint32_t> zero(n, 0);
    make_schedule(q, n, zero.data(), params->seed + j, 0, y.data(), anchor.data(), nullptr, nullptr);
    std::fill(anchor.begin(), anchor.end(), 0);
    if (t) {
      // every variable at its Zippel power: k = nvars + 1, one value of the (absent) x_k
      const uint64_t xk0 = 0;
      zr_points pts;
      pts.nvars = n;
      pts.k = n + 1;
      pts.i_first = 1;
      pts.ni = t;
      pts.nj = 1;
      pts.y = y.data();
      pts.anchor = anchor.data();
      pts.xk = &xk0;
      pts.p = q;
      pts.nexpr = 1;
      if (bb(ctx, &pts, vals, s) != 0) throw Error(ZR_EBLACKBOX);
    }
    uint64_t* rj = res + (size_t)j * tt;
    check(fill_i32(d_cnt, 0, 4, s));
    skeleton_solve(Mq, n, t, d_exps, maxe, y.data(), vals, rj, d_cnt, s);
    check(mp_check(Mq, t, C.nw, num, den, neg, rj, (uint32_t*)d_cnt + 2, s));
    check(hipMemcpyAsync(h, d_cnt, 12, hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
    if (h[0] != 0) throw Error(h[0]);
    if (h[2] == 0) {
      confirmed = j + 1;
      break;
    }
    used.push_back(q);
    C = mp_consts(used);
    check(mp_crt_rr(C, t, res, num, den, neg, (uint32_t*)d_cnt + 1, s));
  }
  if (!confirmed) {
    note_error("no confirmation within the %zu primes given", all.size());
    throw Error(ZR_EPROBE);
  }
  // results: magnitudes [nw][t] -> [t][nw]
  const uint32_t nw = C.nw;
  std::vector<uint64_t> hn((size_t)nw * t), hd((size_t)nw * t);
  std::vector<uint32_t> hneg(t);
  if (t) {
    check(hipMemcpyAsync(hn.data(), num, hn.size() * 8, hipMemcpyDeviceToHost, s));
    check(hipMemcpyAsync(hd.data(), den, hd.size() * 8, hipMemcpyDeviceToHost, s));
    check(hipMemcpyAsync(hneg.data(), neg, (size_t)t * 4, hipMemcpyDeviceToHost, s));
  }
  check(hipStreamSynchronize(s));
  out->nvars = n;
  out->nterms = t;
  out->nwords = nw;
  out->nprimes = confirmed;
  out->exps = (uint16_t*)malloc(sizeof(uint16_t) * std::max<size_t>((size_t)t * n, 1));
  out->num = (uint64_t*)malloc(8 * std::max<size_t>((size_t)t * nw, 1));
  out->den = (uint64_t*)malloc(8 * std::max<size_t>((size_t)t * nw, 1));
  out->neg = (uint8_t*)malloc(std::max<size_t>(t, 1));
  if (!out->exps || !out->num || !out->den || !out->neg) throw Error(ZR_ENOMEM);
  memcpy(out->exps, first.exps, sizeof(uint16_t) * (size_t)t * n);
  for (uint32_t l = 0; l < t; ++l) {
    for (uint32_t w = 0; w < nw; ++w) {
      out->num[(size_t)l * nw + w] = hn[(size_t)w * t + l];
      out->den[(size_t)l * nw + w] = hd[(size_t)w * t + l];
    }
    out->neg[l] = (uint8_t)hneg[l];
  }
}

}  // namespace
}  // namespace zr

using namespace zr;

extern "C" void zr_qpoly_free(zr_qpoly* q) {
  if (!q) return;
  free(q->exps);
  free(q->num);
  free(q->den);
  free(q->neg);
  q->exps = nullptr;
  q->num = nullptr;
  q->den = nullptr;
  q->neg = nullptr;
  q->nterms = 0;
}

extern "C" zr_status zippel_reconstruct_rational(const zr_params* params, const uint64_t* primes, uint32_t nprimes,
                                                 zr_blackbox_fn bb, void* ctx, hipStream_t stream, zr_qpoly* out) {
  if (!out) return ZR_EINVAL;
  memset(out, 0, sizeof(*out));
  try {
    reconstruct_rational(params, primes, nprimes, bb, ctx, stream, out);
    return ZR_OK;
  } catch (const Error& e) {
    zr_qpoly_free(out);
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    zr_qpoly_free(out);
    return ZR_ENOMEM;
  } catch (...) {
    zr_qpoly_free(out);
    return ZR_EDEVICE;
  }
}

extern "C" zr_status zr_skeleton_solve(uint64_t p, uint32_t nvars, uint32_t t, const uint16_t* h_exps,
                                       const uint64_t* y, const uint64_t* d_vals, uint64_t* d_out, int32_t* d_status,
                                       hipStream_t stream) {
  if (p < 3 || p >= ((uint64_t)1 << 63) || nvars == 0 || nvars > 64 || !d_status || !y) return ZR_EINVAL;
  if (t && (!h_exps || !d_vals || !d_out)) return ZR_EINVAL;
  if (!is_prime_u64(p)) return ZR_ENOTPRIME;
  for (uint32_t v = 0; v < nvars; ++v)
    if (y[v] >= p) return ZR_EINVAL;
  try {
    check(fill_i32(d_status, 0, 1, stream));
    if (t == 0) return ZR_OK;
    const zr_mod M = zr_mod_make(p);
    DevArena A(stream);
    const uint16_t* d_exps = upload_exps_soa(nvars, t, h_exps, A, stream);
    skeleton_solve(M, nvars, t, d_exps, max_exponents(nvars, t, h_exps), y, d_vals, d_out, d_status, stream);
    return ZR_OK;
  } catch (const Error& e) {
    return (zr_status)e.code;
  } catch (const std::bad_alloc&) {
    return ZR_ENOMEM;
  } catch (...) {
    return ZR_EDEVICE;
  }
}
