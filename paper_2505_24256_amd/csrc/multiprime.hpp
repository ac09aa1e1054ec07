// Multi-prime step: coefficients of a known term set modulo a further prime
// (one transposed Vandermonde system with one right-hand side, correlation
// form), Chinese remaindering and rational reconstruction per term.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.hpp"

namespace zr {

// Primes per reconstruction (the first included) and 64-bit words of their
// product: eight primes below 2^63 fit in eight words.
constexpr int kMpWords = 8;
constexpr uint32_t kMpMaxPrimes = 8;

// Constants of the Chinese remaindering over primes p_0..p_{J-1}.
struct MpConsts {
  uint32_t J;                           // primes combined
  uint32_t e;                           // bound exponent: |num|, den < 2^e
  uint32_t nw;                          // output words per magnitude, cdiv(e, 64)
  uint32_t pad;
  zr_mod mod[kMpWords];                 // p_j
  uint64_t pmod[kMpWords][kMpWords];    // [j][i] = p_i mod p_j, i < j
  uint64_t cinv[kMpWords];              // (p_0 ... p_{j-1})^{-1} mod p_j
  uint64_t P[kMpWords];                 // p_0 ... p_{J-1}, little-endian words
};

struct MpSolvePlan {
  uint32_t t;
  uint32_t LC, C;  // correlation: chunk length and count
  uint32_t L, S;   // evaluation: chunk length and count
};
MpSolvePlan mp_solve_plan(uint32_t t);
size_t mp_solve_words(const MpSolvePlan& P);

// a_l (l < t) from samples vals[i-1] = sum_l a_l m_l^i, i = 1..t, given the
// monomial values and the master polynomial's lower coefficients Mc[t].
// status receives ZR_ESINGULAR (-3) when some m_l M'(m_l) vanishes.
hipError_t mp_solve(const zr_mod& M, const MpSolvePlan& P, const uint64_t* mono, const uint64_t* Mc,
                    const uint64_t* vals, uint64_t* out, uint64_t* work, int32_t* status, hipStream_t s);

// res [J][t] residues -> num, den [nw][t] magnitudes (words), neg [t];
// fails counts the terms with no fraction within the bound.
hipError_t mp_crt_rr(const MpConsts& C, uint32_t t, const uint64_t* res, uint64_t* num, uint64_t* den,
                     uint32_t* neg, uint32_t* fails, hipStream_t s);

// mismatches counts the terms whose fraction does not reduce to res mod p.
hipError_t mp_check(const zr_mod& M, uint32_t t, uint32_t nw, const uint64_t* num, const uint64_t* den,
                    const uint32_t* neg, const uint64_t* res, uint32_t* mismatches, hipStream_t s);

}  // namespace zr
