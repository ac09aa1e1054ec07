// Arithmetic in F_p for 3 <= p < 2^63, shared by host and device code of the
// library.  Products are formed from 32x32->64 multiplies by the compiler
// (v_mad_u64_u32 on gfx950); no hardware divide is used anywhere.
//
//  * General products a*b mod p reduce the 128-bit product by division by an
//    invariant integer with a precomputed reciprocal (Moller and Granlund,
//    "Improved division by invariant integers", IEEE Trans. Computers 60(2),
//    2011, 2-by-1 division with a normalised divisor).  This is the method the
//    paper adopts in §2.1 for its fastest mulmod variant.
//  * Products by a fixed multiplier w use Shoup's precomputed quotient
//    w' = floor(w 2^64 / p): r = x w - hi(x w') p lies in [0, 2p) for any
//    64-bit x (V. Shoup, NTL; see also Harvey, "Faster arithmetic for
//    number-theoretic transforms", J. Symb. Comp. 2014).
//  * Sums of many 126-bit products are accumulated exactly in 192 bits and
//    reduced once (deferred reduction, §2.2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ZR_HD __host__ __device__ __forceinline__

typedef unsigned __int128 zr_u128;

struct zr_mod {
  uint64_t p;     // the prime
  uint64_t pn;    // p << norm, top bit set
  uint64_t v;     // floor((2^128 - 1) / pn) - 2^64
  uint32_t norm;  // number of leading zero bits of p (>= 1)
  uint32_t pad;
};

// Host-side construction (uses a 128-bit division once).
static inline zr_mod zr_mod_make(uint64_t p) {
  zr_mod M;
  M.p = p;
  M.norm = (uint32_t)__builtin_clzll(p);
  M.pn = p << M.norm;
  M.v = (uint64_t)(((((zr_u128)(~M.pn)) << 64) | ~(uint64_t)0) / M.pn);
  M.pad = 0;
  return M;
}

ZR_HD uint64_t zr_mulhi(uint64_t a, uint64_t b) { return (uint64_t)(((zr_u128)a * b) >> 64); }

// Remainder (and quotient) of (u1:u0) by the normalised divisor pn; needs u1 < pn.
ZR_HD uint64_t zr_div21(const zr_mod& M, uint64_t u1, uint64_t u0, uint64_t* quo) {
  zr_u128 q = (zr_u128)M.v * u1 + ((((zr_u128)u1) << 64) | u0);
  uint64_t q1 = (uint64_t)(q >> 64) + 1;
  uint64_t q0 = (uint64_t)q;
  uint64_t r = u0 - q1 * M.pn;
  if (r > q0) {
    q1 -= 1;
    r += M.pn;
  }
  if (r >= M.pn) {
    q1 += 1;
    r -= M.pn;
  }
  if (quo) *quo = q1;
  return r;
}

// (hi:lo) mod p for hi < p.
ZR_HD uint64_t zr_mod128(const zr_mod& M, uint64_t hi, uint64_t lo) {
  const uint32_t s = M.norm;
  uint64_t u1 = (hi << s) | (lo >> (64 - s));
  uint64_t u0 = lo << s;
  return zr_div21(M, u1, u0, nullptr) >> s;
}

ZR_HD uint64_t zr_mul(const zr_mod& M, uint64_t a, uint64_t b) {
  zr_u128 t = (zr_u128)a * b;
  return zr_mod128(M, (uint64_t)(t >> 64), (uint64_t)t);
}

ZR_HD uint64_t zr_add(const zr_mod& M, uint64_t a, uint64_t b) {
  uint64_t s = a + b;  // a, b < p < 2^63: no overflow
  return s >= M.p ? s - M.p : s;
}

ZR_HD uint64_t zr_sub(const zr_mod& M, uint64_t a, uint64_t b) { return a >= b ? a - b : a + M.p - b; }

ZR_HD uint64_t zr_neg(const zr_mod& M, uint64_t a) { return a ? M.p - a : 0; }

// Reduce x < 2p to [0, p).
ZR_HD uint64_t zr_red2p(const zr_mod& M, uint64_t x) { return x >= M.p ? x - M.p : x; }

// Shoup quotient for the fixed multiplier w < p.
ZR_HD uint64_t zr_shoup_pre(const zr_mod& M, uint64_t w) {
  uint64_t q;
  zr_div21(M, w << M.norm, 0, &q);
  return q;
}

// x*w mod p in [0, 2p) for any 64-bit x.
ZR_HD uint64_t zr_shoup_lazy(const zr_mod& M, uint64_t x, uint64_t w, uint64_t wp) {
  uint64_t qh = zr_mulhi(x, wp);
  return x * w - qh * M.p;
}

ZR_HD uint64_t zr_shoup(const zr_mod& M, uint64_t x, uint64_t w, uint64_t wp) {
  return zr_red2p(M, zr_shoup_lazy(M, x, w, wp));
}

ZR_HD uint64_t zr_pow(const zr_mod& M, uint64_t a, uint64_t e) {
  uint64_t r = 1 % M.p;
  while (e) {
    if (e & 1) r = zr_mul(M, r, a);
    a = zr_mul(M, a, a);
    e >>= 1;
  }
  return r;
}

// Inverse by Fermat's little theorem (p prime); 0 maps to 0.
ZR_HD uint64_t zr_inv(const zr_mod& M, uint64_t a) { return zr_pow(M, a, M.p - 2); }

// Exact 192-bit accumulator of products of two values below 2^64.
struct zr_acc192 {
  uint64_t lo, hi;
  uint32_t top;
};

ZR_HD void zr_acc_zero(zr_acc192& a) {
  a.lo = 0;
  a.hi = 0;
  a.top = 0;
}

ZR_HD void zr_acc_mac(zr_acc192& a, uint64_t x, uint64_t y) {
  zr_u128 pr = (zr_u128)x * y;
  zr_u128 s = ((((zr_u128)a.hi) << 64) | a.lo) + pr;
  a.top += (uint32_t)(s < pr);
  a.lo = (uint64_t)s;
  a.hi = (uint64_t)(s >> 64);
}

ZR_HD uint64_t zr_acc_reduce(const zr_mod& M, const zr_acc192& a) {
  uint64_t r = zr_mod128(M, 0, a.top);
  r = zr_mod128(M, r, a.hi);
  return zr_mod128(M, r, a.lo);
}
