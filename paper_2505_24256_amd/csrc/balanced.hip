// gfx950 kernels of the balanced (rational) Zippel path: per-slice Thiele
// reconstruction (eq. 2), the transposed Vandermonde apply that evaluates the
// previous stage's numerator/denominator at the Zippel points, and the
// balancing factors that make all slices share one normalisation (§2.2).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "field.hpp"
#include "kernels.hpp"

namespace zr {

__host__ __device__ static inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// ----------------------------------------------------------------------------
// Thiele, one lane per slice.  Samples F[j][i] at nodes X[j], j < nk.
// Inverse differences phi_{s+1}(x_j) = (x_j - x_s) / (phi_s(x_j) - phi_s(x_s)),
// b_s = phi_s(x_s); stop at the first m whose continued fraction reproduces the
// sample at node m+1 (evaluated as a fraction P/Q, so without inverses).
// Then (A, B) <- (b_m, 1), (A, B) <- (b_s A + (x - x_s) B, A) for s = m-1..0,
// and scale so that the lowest nonzero coefficient of B is 1.
// Arrays are SoA [index][T] so that consecutive lanes touch consecutive words.
// ----------------------------------------------------------------------------
__device__ void thiele_body(const zr_mod& M, uint32_t T, uint32_t nk, const uint64_t* __restrict__ X,
                            const uint64_t* __restrict__ F, uint64_t* __restrict__ A, uint64_t* __restrict__ B,
                            int32_t* __restrict__ degA, int32_t* __restrict__ degB, int32_t* __restrict__ st,
                            uint64_t* __restrict__ scratch, uint32_t i) {
  uint64_t* phi = scratch;
  uint64_t* b = phi + (size_t)nk * T;
  uint64_t* NA = b + (size_t)nk * T;
#define PHI(j) phi[(size_t)(j) * T + i]
#define BB(j) b[(size_t)(j) * T + i]
#define FV(j) F[(size_t)(j) * T + i]
  for (uint32_t j = 0; j < nk; ++j) PHI(j) = FV(j);
  BB(0) = PHI(0);
  uint32_t m = 0;
  int32_t status = 0;
  for (;;) {
    if (m + 1 >= nk) {
      status = -5;  // samples exhausted without confirmation
      break;
    }
    const uint64_t x = X[m + 1];
    uint64_t P = BB(m), Q = 1 % M.p;
    bool ok = true;
    for (uint32_t s = m; s-- > 0;) {
      if (P == 0) {
        ok = false;
        break;
      }
      const uint64_t nP = zr_add(M, zr_mul(M, BB(s), P), zr_mul(M, zr_sub(M, x, X[s]), Q));
      Q = P;
      P = nP;
    }
    if (ok && P == zr_mul(M, FV(m + 1), Q)) break;
    // phi_{m+1}(x_j) for j > m, the denominators inverted together
    // (Montgomery's batch inversion: one inverse and three products each)
    const uint64_t pm = PHI(m), xm = X[m];
    uint64_t pre = 1 % M.p;
    for (uint32_t j = m + 1; j < nk; ++j) {
      const uint64_t den = zr_sub(M, PHI(j), pm);
      if (den == 0) {
        status = -4;
        break;
      }
      NA[(size_t)j * T + i] = pre;  // product of the denominators before j
      pre = zr_mul(M, pre, den);
    }
    if (status) break;
    uint64_t inv = zr_inv(M, pre);
    for (uint32_t j = nk; j-- > m + 1;) {
      const uint64_t den = zr_sub(M, PHI(j), pm);
      const uint64_t dinv = zr_mul(M, inv, NA[(size_t)j * T + i]);
      inv = zr_mul(M, inv, den);
      PHI(j) = zr_mul(M, zr_sub(M, X[j], xm), dinv);
    }
    BB(m + 1) = PHI(m + 1);
    ++m;
  }
  if (status) {
    st[i] = status;
    degA[i] = -1;
    degB[i] = -1;
    return;
  }
#define AA(r) A[(size_t)(r) * T + i]
#define BQ(r) B[(size_t)(r) * T + i]
#define NN(r) NA[(size_t)(r) * T + i]
  const uint32_t cap = nk + 1;
  for (uint32_t r = 0; r < cap; ++r) {
    AA(r) = 0;
    BQ(r) = 0;
  }
  AA(0) = BB(m);
  BQ(0) = 1 % M.p;
  for (uint32_t s = m; s-- > 0;) {
    const uint64_t bs = BB(s), xs = X[s];
    const uint32_t top = std::min(cap - 1, m + 1);
    for (uint32_t r = 0; r <= top; ++r) {
      uint64_t v = zr_sub(M, zr_mul(M, bs, AA(r)), zr_mul(M, xs, BQ(r)));
      if (r > 0) v = zr_add(M, v, BQ(r - 1));
      NN(r) = v;
    }
    for (uint32_t r = 0; r <= top; ++r) {
      BQ(r) = AA(r);
      AA(r) = NN(r);
    }
  }
  int32_t da = -1, db = -1;
  for (uint32_t r = 0; r < cap; ++r) {
    if (AA(r)) da = (int32_t)r;
    if (BQ(r)) db = (int32_t)r;
  }
  if (db < 0) {
    st[i] = -4;
    degA[i] = -1;
    degB[i] = -1;
    return;
  }
  uint32_t low = 0;
  while (BQ(low) == 0) ++low;
  const uint64_t sc = zr_inv(M, BQ(low));
  for (int32_t r = 0; r <= da; ++r) AA(r) = zr_mul(M, AA(r), sc);
  for (int32_t r = 0; r <= db; ++r) BQ(r) = zr_mul(M, BQ(r), sc);
  if (da < 0) da = 0;
  degA[i] = da;
  degB[i] = db;
  st[i] = 0;
#undef PHI
#undef BB
#undef FV
#undef AA
#undef BQ
#undef NN
}

__global__ void k_thiele(zr_mod M, uint32_t T, uint32_t nk, const uint64_t* __restrict__ X,
                         const uint64_t* __restrict__ F, uint64_t* __restrict__ A, uint64_t* __restrict__ B,
                         int32_t* __restrict__ degA, int32_t* __restrict__ degB, int32_t* __restrict__ st,
                         uint64_t* __restrict__ scratch) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < T) thiele_body(M, T, nk, X, F, A, B, degA, degB, st, scratch, i);
}

// ----------------------------------------------------------------------------
// Thiele, one wavefront per slice (nk <= 64 KPL - 1).  The same continued
// fraction as thiele_body, computed without per-step inverses: an inverse
// difference is carried as a fraction N/D,
//     phi_{m+1}(x_j) = (x_j - x_m) D_j D_m / (N_j D_m - N_m D_j),
// starting from (f_j, 1).  Every D that is used is nonzero (a zero one is the
// vanishing denominator that ends the recursion), so replacing b_s by N_s/D_s
// and clearing the D's scales the confirmation fraction P/Q and the
// polynomials (A, B) by nonzero constants: no zero test and no ratio changes,
// and the final normalisation of B removes the constant.  One inverse remains.
//   1. all recursion steps m = 0..nk-2 at once over the lanes (lane-held
//      index j = 64 k + lane), up to the first step with a zero denominator;
//   2. the confirmation test of every candidate m in parallel (lane-held m),
//      one uniform loop over s = mlast-1..0 with b_s broadcast from its lane;
//   3. the first confirmed m -> (A, B), lane-held coefficient index r.
// ----------------------------------------------------------------------------
constexpr int kThWaves = 4;      // slices (wavefronts) per workgroup
constexpr int kThMaxKpl = 8;     // values per lane: nk <= 511

// v from lane `src` (uniform) of the wavefront
__device__ __forceinline__ uint64_t bcast(uint64_t v, uint32_t src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)src);
  return ((uint64_t)hi << 32) | lo;
}

// Element idx (uniform) of the lane-held array v.  Each lane offers the entry
// it holds at idx, if any, and the owner lane's offer is broadcast; the group
// index stays a compile-time constant, so v is never indexed at run time.
template <int KPL>
__device__ __forceinline__ uint64_t held(const uint64_t (&v)[KPL], uint32_t idx, uint32_t lane) {
  uint64_t mine = 0;
#pragma unroll
  for (int k = 0; k < KPL; ++k)
    if (64 * k + lane == idx) mine = v[k];
  return bcast(mine, idx & 63);
}

template <int KPL>
__device__ void thiele_wave(const zr_mod& M, uint32_t T, uint32_t nk, const uint64_t* __restrict__ X,
                            const uint64_t* __restrict__ F, uint64_t* __restrict__ A, uint64_t* __restrict__ B,
                            int32_t* __restrict__ degA, int32_t* __restrict__ degB, int32_t* __restrict__ st,
                            uint32_t i) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t one = 1 % M.p;
  auto fail = [&](int32_t code) {
    if (lane == 0) {
      st[i] = code;
      degA[i] = -1;
      degB[i] = -1;
    }
  };
  if (nk < 2) {
    fail(-5);  // no sample to confirm with
    return;
  }
  uint64_t N[KPL], D[KPL], xv[KPL];
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    const uint32_t j = 64 * k + lane;
    const bool in = j < nk;
    xv[k] = in ? X[j] : 0;
    N[k] = in ? F[(size_t)j * T + i] : 0;
    D[k] = one;
  }
  // 1. recursion steps m = 64 g + l; zstep = first step with a zero
  //    denominator (nk: none).  Groups below g hold no index above m.
  uint32_t zstep = nk;
  bool stop = false;
#pragma unroll
  for (int g = 0; g < KPL; ++g) {
    for (uint32_t l = 0; l < 64 && !stop; ++l) {
      const uint32_t m = 64 * g + l;
      if (m + 1 >= nk) {
        stop = true;
        break;
      }
      const uint64_t Nm = bcast(N[g], l), Dm = bcast(D[g], l), xm = bcast(xv[g], l);
      bool zero = false;
#pragma unroll
      for (int k = g; k < KPL; ++k) {
        const uint32_t j = 64 * k + lane;
        if (j > m && j < nk) {
          const uint64_t dn = zr_sub(M, zr_mul(M, N[k], Dm), zr_mul(M, Nm, D[k]));
          N[k] = zr_mul(M, zr_mul(M, zr_sub(M, xv[k], xm), D[k]), Dm);
          D[k] = dn;
          zero |= dn == 0;
        }
      }
      if (__ballot(zero)) {
        zstep = m;
        stop = true;
      }
    }
  }
  // 2. candidates m <= mlast (b_0..b_m final), confirmed at node m+1;
  //    s = 64 g + l runs down from mlast-1, lane-held m updates while m > s
  const uint32_t mlast = zstep < nk - 2 ? zstep : nk - 2;
  uint64_t P[KPL], Q[KPL], xc[KPL], fc[KPL];
  bool ok[KPL];
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    const uint32_t m = 64 * k + lane;
    ok[k] = m <= mlast;
    P[k] = N[k];
    Q[k] = D[k];
    xc[k] = ok[k] ? X[m + 1] : 0;
    fc[k] = ok[k] ? F[(size_t)(m + 1) * T + i] : 0;
  }
#pragma unroll
  for (int g = KPL - 1; g >= 0; --g) {
    if (64u * g >= mlast) continue;
    const uint32_t top = mlast - 64u * g < 64u ? mlast - 64u * g : 64u;  // s < mlast
    for (uint32_t l = top; l-- > 0;) {
      const uint32_t s = 64 * g + l;
      const uint64_t Ns = bcast(N[g], l), Ds = bcast(D[g], l), xs = bcast(xv[g], l);
#pragma unroll
      for (int k = g; k < KPL; ++k) {
        const uint32_t m = 64 * k + lane;
        if (ok[k] && m > s) {
          if (P[k] == 0) {
            ok[k] = false;  // a zero tail: the nested fraction divides by zero
          } else {
            const uint64_t u = zr_mul(M, zr_sub(M, xc[k], xs), Ds);
            const uint64_t nP = zr_add(M, zr_mul(M, Ns, P[k]), zr_mul(M, u, Q[k]));
            Q[k] = zr_mul(M, Ds, P[k]);
            P[k] = nP;
          }
        }
      }
    }
  }
  uint32_t c = nk;
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    const uint64_t hit = __ballot(ok[k] && P[k] == zr_mul(M, fc[k], Q[k]));
    if (hit && c == nk) c = 64 * k + (uint32_t)__builtin_ctzll(hit);
  }
  if (c == nk) {
    fail(zstep < nk ? -4 : -5);
    return;
  }
  // 3. (A, B) <- (N_c, D_c); (A, B) <- (N_s A + (x - x_s) D_s B, D_s A) for
  //    s = c-1..0; after c - s steps the degree is at most c - s <= c
  uint64_t Ac[KPL], Bc[KPL];
  {
    const uint64_t Nc = held(N, c, lane), Dc = held(D, c, lane);
#pragma unroll
    for (int k = 0; k < KPL; ++k) {
      const bool r0 = k == 0 && lane == 0;
      Ac[k] = r0 ? Nc : 0;
      Bc[k] = r0 ? Dc : 0;
    }
  }
#pragma unroll
  for (int g = KPL - 1; g >= 0; --g) {
    if (64u * g >= c) continue;
    const uint32_t top = c - 64u * g < 64u ? c - 64u * g : 64u;  // s < c
    for (uint32_t l = top; l-- > 0;) {
      const uint64_t Ns = bcast(N[g], l), Ds = bcast(D[g], l), xs = bcast(xv[g], l);
      const uint64_t u = zr_mul(M, xs, Ds);
      uint64_t Bm[KPL];  // coefficient r-1 of B
#pragma unroll
      for (int k = 0; k < KPL; ++k) {
        const uint64_t up = __shfl_up(Bc[k], 1, 64);
        const uint64_t carry = k > 0 ? bcast(Bc[k > 0 ? k - 1 : 0], 63) : 0;
        Bm[k] = lane == 0 ? carry : up;
      }
#pragma unroll
      for (int k = 0; k < KPL; ++k) {
        if (64u * k > c) continue;  // coefficients above the final degree stay 0
        const uint64_t a =
            zr_add(M, zr_sub(M, zr_mul(M, Ns, Ac[k]), zr_mul(M, u, Bc[k])), zr_mul(M, Ds, Bm[k]));
        Bc[k] = zr_mul(M, Ds, Ac[k]);
        Ac[k] = a;
      }
    }
  }
  int32_t da = -1, db = -1, low = -1;
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    const uint64_t nzA = __ballot(Ac[k] != 0), nzB = __ballot(Bc[k] != 0);
    if (nzA) da = 64 * k + 63 - __builtin_clzll(nzA);
    if (nzB) db = 64 * k + 63 - __builtin_clzll(nzB);
    if (nzB && low < 0) low = 64 * k + __builtin_ctzll(nzB);
  }
  if (db < 0) {
    fail(-4);
    return;
  }
  const uint64_t sc = zr_inv(M, held(Bc, (uint32_t)low, lane));
  const uint32_t cap = nk + 1;
#pragma unroll
  for (int k = 0; k < KPL; ++k) {
    const uint32_t r = 64 * k + lane;
    if (r < cap) {
      A[(size_t)r * T + i] = zr_mul(M, Ac[k], sc);
      B[(size_t)r * T + i] = zr_mul(M, Bc[k], sc);
    }
  }
  if (lane == 0) {
    degA[i] = da < 0 ? 0 : da;
    degB[i] = db;
    st[i] = 0;
  }
}

template <int KPL>
__global__ void __launch_bounds__(64 * kThWaves)
    k_thiele_wave(zr_mod M, uint32_t T, uint32_t nk, const uint64_t* __restrict__ X, const uint64_t* __restrict__ F,
                  uint64_t* __restrict__ A, uint64_t* __restrict__ B, int32_t* __restrict__ degA,
                  int32_t* __restrict__ degB, int32_t* __restrict__ st) {
  const uint32_t i = blockIdx.x * kThWaves + (threadIdx.x >> 6);
  if (i < T) thiele_wave<KPL>(M, T, nk, X, F, A, B, degA, degB, st, i);
}

// block b belongs to job seg(b): the largest s with prefix[s] <= b
__device__ __forceinline__ uint32_t thiele_job_of(uint32_t n, const uint32_t* __restrict__ prefix, uint32_t b) {
  uint32_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Slices of many reconstructions in one launch, kThWaves slices per block.
template <int KPL>
__global__ void __launch_bounds__(64 * kThWaves)
    k_thiele_wave_batch(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix, const ThieleJob* __restrict__ jobs) {
  const uint32_t q = thiele_job_of(n, prefix, blockIdx.x);
  const ThieleJob& j = jobs[q];
  const uint32_t i = (blockIdx.x - prefix[q]) * kThWaves + (threadIdx.x >> 6);
  if (i < j.T) thiele_wave<KPL>(M, j.T, j.nk, j.X, j.F, j.A, j.B, j.degA, j.degB, j.st, i);
}

// The same with one lane per slice (any nk; uses the jobs' scratch), 64 slices per block.
__global__ void k_thiele_batch(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix,
                               const ThieleJob* __restrict__ jobs) {
  const uint32_t q = thiele_job_of(n, prefix, blockIdx.x);
  const ThieleJob& j = jobs[q];
  const uint32_t i = (blockIdx.x - prefix[q]) * blockDim.x + threadIdx.x;
  if (i < j.T) thiele_body(M, j.T, j.nk, j.X, j.F, j.A, j.B, j.degA, j.degB, j.st, j.scratch, i);
}

static int thiele_kpl(uint32_t nk) {
  for (int kpl = 1; kpl <= kThMaxKpl; kpl *= 2)
    if (nk + 1 <= 64u * kpl) return kpl;
  return 0;  // one lane per slice
}

uint32_t thiele_slices_per_block(uint32_t max_nk) { return thiele_kpl(max_nk) ? kThWaves : 64; }

size_t thiele_scratch_words(uint32_t T, uint32_t nk) {
  return thiele_kpl(nk) ? 0 : (size_t)(3 * nk + 1) * std::max<uint32_t>(T, 1);
}

hipError_t thiele_slices_batch(const zr_mod& M, uint32_t n, const uint32_t* d_prefix, uint32_t total_blocks,
                               uint32_t max_nk, const ThieleJob* d_jobs, hipStream_t s) {
  if (n == 0 || total_blocks == 0) return hipSuccess;
  TimedLaunch tl("thiele", s);
  const dim3 g(total_blocks), b(64 * kThWaves);
  switch (thiele_kpl(max_nk)) {
    case 1: hipLaunchKernelGGL(k_thiele_wave_batch<1>, g, b, 0, s, M, n, d_prefix, d_jobs); break;
    case 2: hipLaunchKernelGGL(k_thiele_wave_batch<2>, g, b, 0, s, M, n, d_prefix, d_jobs); break;
    case 4: hipLaunchKernelGGL(k_thiele_wave_batch<4>, g, b, 0, s, M, n, d_prefix, d_jobs); break;
    case 8: hipLaunchKernelGGL(k_thiele_wave_batch<8>, g, b, 0, s, M, n, d_prefix, d_jobs); break;
    default: hipLaunchKernelGGL(k_thiele_batch, g, dim3(64), 0, s, M, n, d_prefix, d_jobs); break;
  }
  return hipGetLastError();
}

hipError_t thiele_slices(const zr_mod& M, uint32_t T, uint32_t nk, const uint64_t* X, const uint64_t* F, uint64_t* A,
                         uint64_t* B, int32_t* degA, int32_t* degB, int32_t* st, uint64_t* scratch, hipStream_t s) {
  if (T == 0) return hipSuccess;
  TimedLaunch tl("thiele", s);
  const dim3 g(cdiv(T, kThWaves)), b(64 * kThWaves);
  switch (thiele_kpl(nk)) {
    case 1: hipLaunchKernelGGL(k_thiele_wave<1>, g, b, 0, s, M, T, nk, X, F, A, B, degA, degB, st); break;
    case 2: hipLaunchKernelGGL(k_thiele_wave<2>, g, b, 0, s, M, T, nk, X, F, A, B, degA, degB, st); break;
    case 4: hipLaunchKernelGGL(k_thiele_wave<4>, g, b, 0, s, M, T, nk, X, F, A, B, degA, degB, st); break;
    case 8: hipLaunchKernelGGL(k_thiele_wave<8>, g, b, 0, s, M, T, nk, X, F, A, B, degA, degB, st); break;
    default:
      if (!scratch) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_thiele, dim3(cdiv(T, 64)), dim3(64), 0, s, M, T, nk, X, F, A, B, degA, degB, st, scratch);
      break;
  }
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Transposed Vandermonde apply out[i] = sum_l a_l m_l^(i+1): one lane per term
// l walks its power chain over a block of i with a fixed Shoup multiplier; the
// per-i partial sums are reduced across the wave with lane shuffles and across
// the workgroup in LDS (the substitution kernel of §2.2 with its warp
// reduction, on 64-lane wavefronts).
// ----------------------------------------------------------------------------
constexpr int kApW = 4;      // waves per workgroup
constexpr int kApB = 128;    // powers i per workgroup

__device__ __forceinline__ uint64_t wave_sum_mod(const zr_mod& M, uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(v, off, 64);
    v = zr_add(M, v, o);
  }
  return v;
}

// block (bx, by): powers i0 = kApB bx .. + kApB, terms kApW*64 by .. (one partial row by)
__device__ __forceinline__ void vapply_body(const zr_mod& M, uint32_t t, const uint64_t* __restrict__ mono,
                                            const uint64_t* __restrict__ a, uint32_t T,
                                            uint64_t* __restrict__ partial, uint32_t bx, uint32_t by,
                                            uint64_t (*sh)[kApB]) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t l = by * (kApW * 64) + threadIdx.x;
  const uint32_t i0 = bx * kApB;
  const uint32_t nb = std::min<uint32_t>(kApB, T - i0);
  uint64_t m = 0, mp = 0, b = 0;
  if (l < t) {
    m = mono[l];
    mp = zr_shoup_pre(M, m);
    b = zr_mul(M, a[l], zr_pow(M, m, i0 + 1));
  }
  for (uint32_t ii = 0; ii < nb; ++ii) {
    const uint64_t s = wave_sum_mod(M, b);
    if (lane == 0) sh[wave][ii] = s;
    b = zr_shoup(M, b, m, mp);
  }
  __syncthreads();
  for (uint32_t ii = threadIdx.x; ii < nb; ii += blockDim.x) {
    uint64_t s = sh[0][ii];
    for (int w = 1; w < kApW; ++w) s = zr_add(M, s, sh[w][ii]);
    partial[(size_t)by * T + i0 + ii] = s;
  }
}

__global__ void __launch_bounds__(kApW * 64) k_vapply(zr_mod M, uint32_t t, const uint64_t* __restrict__ mono,
                                                      const uint64_t* __restrict__ a, uint32_t T,
                                                      uint64_t* __restrict__ partial) {
  __shared__ uint64_t sh[kApW][kApB];
  vapply_body(M, t, mono, a, T, partial, blockIdx.x, blockIdx.y, sh);
}

__global__ void k_vapply_sum(zr_mod M, uint32_t T, uint32_t nparts, const uint64_t* __restrict__ partial,
                             uint64_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  uint64_t s = 0;
  for (uint32_t c = 0; c < nparts; ++c) s = zr_add(M, s, partial[(size_t)c * T + i]);
  out[i] = s;
}

size_t vapply_work_words(uint32_t t, uint32_t T) {
  return (size_t)std::max<uint32_t>(1, cdiv(t, kApW * 64)) * std::max<uint32_t>(T, 1) + 64;
}

hipError_t vapply(const zr_mod& M, uint32_t t, const uint64_t* mono, const uint64_t* a, uint32_t T, uint64_t* out,
                  uint64_t* work, size_t work_words, hipStream_t s) {
  if (T == 0) return hipSuccess;
  if (t == 0) return fill_u64(out, 0, T, s);
  const uint32_t nparts = cdiv(t, kApW * 64);
  if (work_words < (size_t)nparts * T) return hipErrorInvalidValue;
  TimedLaunch tl("vapply", s);
  hipLaunchKernelGGL(k_vapply, dim3(cdiv(T, kApB), nparts), dim3(kApW * 64), 0, s, M, t, mono, a, T, work);
  hipLaunchKernelGGL(k_vapply_sum, dim3(cdiv(T, 256)), dim3(256), 0, s, M, T, nparts, work, out);
  return hipGetLastError();
}

// ---- many applies in two launches (block -> job by binary search over prefix sums)
uint32_t vapply_batch_blocks(uint32_t t, uint32_t T) { return t ? cdiv(T, kApB) * cdiv(t, kApW * 64) : 0; }

__global__ void __launch_bounds__(kApW * 64) k_vapply_batch(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix,
                                                            const VapplyJob* __restrict__ jobs) {
  __shared__ uint64_t sh[kApW][kApB];
  const uint32_t q = thiele_job_of(n, prefix, blockIdx.x);
  const VapplyJob& j = jobs[q];
  const uint32_t lb = blockIdx.x - prefix[q], nbx = cdiv(j.T, kApB);
  vapply_body(M, j.t, j.mono, j.a, j.T, j.work, lb % nbx, lb / nbx, sh);
}

__global__ void k_vapply_sum_batch(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix,
                                   const VapplyJob* __restrict__ jobs) {
  const uint32_t q = thiele_job_of(n, prefix, blockIdx.x);
  const VapplyJob& j = jobs[q];
  const uint32_t i = (blockIdx.x - prefix[q]) * blockDim.x + threadIdx.x;
  if (i >= j.T) return;
  const uint32_t nparts = j.t ? cdiv(j.t, kApW * 64) : 0;
  uint64_t s = 0;
  for (uint32_t c = 0; c < nparts; ++c) s = zr_add(M, s, j.work[(size_t)c * j.T + i]);
  j.out[i] = s;
}

hipError_t vapply_batch(const zr_mod& M, uint32_t n, const uint32_t* d_prefix, uint32_t total,
                        const uint32_t* d_sum_prefix, uint32_t sum_total, const VapplyJob* d_jobs, hipStream_t s) {
  if (n == 0) return hipSuccess;
  TimedLaunch tl("vapply", s);
  if (total) hipLaunchKernelGGL(k_vapply_batch, dim3(total), dim3(kApW * 64), 0, s, M, n, d_prefix, d_jobs);
  if (sum_total) hipLaunchKernelGGL(k_vapply_sum_batch, dim3(sum_total), dim3(256), 0, s, M, n, d_sum_prefix, d_jobs);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Balancing: beta_i = N_{k-1}(y^i) / A_i(x_0) (fallback D_{k-1}(y^i) / B_i(x_0))
// and the balanced right-hand sides beta_i A_i(x_j), beta_i B_i(x_j), j >= 1.
// ----------------------------------------------------------------------------
__device__ uint64_t horner_col(const zr_mod& M, const uint64_t* c, uint32_t T, uint32_t i, int32_t deg, uint64_t x) {
  uint64_t v = 0;
  for (int32_t r = deg; r >= 0; --r) v = zr_add(M, zr_mul(M, v, x), c[(size_t)r * T + i]);
  return v;
}

// beta_i from the two values at x_0 (one lane per slice; st[i] = -4 if neither exists)
__global__ void k_balance_beta(zr_mod M, uint32_t T, const uint64_t* __restrict__ X, const uint64_t* __restrict__ A,
                               const uint64_t* __restrict__ B, const int32_t* __restrict__ degA,
                               const int32_t* __restrict__ degB, const uint64_t* __restrict__ nprev,
                               const uint64_t* __restrict__ dprev, uint64_t* __restrict__ beta,
                               int32_t* __restrict__ st) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T) return;
  const uint64_t a0 = horner_col(M, A, T, i, degA[i], X[0]);
  const uint64_t b0 = horner_col(M, B, T, i, degB[i], X[0]);
  uint64_t b = 0;
  if (nprev[i] != 0 && a0 != 0) b = zr_mul(M, nprev[i], zr_inv(M, a0));
  else if (dprev[i] != 0 && b0 != 0) b = zr_mul(M, dprev[i], zr_inv(M, b0));
  else st[i] = -4;
  beta[i] = b;
}

// One thread per (slice i, right-hand side u): u < rhoN is beta_i A_i(x_{u+1}),
// the rest beta_i B_i(x_{u-rhoN+1}).
__global__ void k_balance_rhs(zr_mod M, uint32_t T, const uint64_t* __restrict__ X, const uint64_t* __restrict__ A,
                              const uint64_t* __restrict__ B, const int32_t* __restrict__ degA,
                              const int32_t* __restrict__ degB, const uint64_t* __restrict__ beta, uint32_t tN,
                              int32_t rhoN, uint64_t* __restrict__ vN, size_t ldN, uint32_t tD,
                              uint64_t* __restrict__ vD, size_t ldD) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t u = blockIdx.y;
  if (u < (uint32_t)rhoN) {
    if (i < tN) vN[(size_t)u * ldN + i] = zr_mul(M, beta[i], horner_col(M, A, T, i, degA[i], X[u + 1]));
  } else {
    const uint32_t j = u - (uint32_t)rhoN;
    if (i < tD) vD[(size_t)j * ldD + i] = zr_mul(M, beta[i], horner_col(M, B, T, i, degB[i], X[j + 1]));
  }
}

hipError_t balance_rhs(const zr_mod& M, uint32_t T, uint32_t nk, const uint64_t* X, const uint64_t* A,
                       const uint64_t* B, const int32_t* degA, const int32_t* degB, const uint64_t* nprev,
                       const uint64_t* dprev, uint32_t tN, int32_t rhoN, uint64_t* vN, size_t ldN, uint32_t tD,
                       int32_t rhoD, uint64_t* vD, size_t ldD, int32_t* st, uint64_t* beta, hipStream_t s) {
  (void)nk;
  if (T == 0) return hipSuccess;
  TimedLaunch tl("balance", s);
  hipLaunchKernelGGL(k_balance_beta, dim3(cdiv(T, 64)), dim3(64), 0, s, M, T, X, A, B, degA, degB, nprev, dprev,
                     beta, st);
  const uint32_t units = (uint32_t)std::max(rhoN, 0) + (uint32_t)std::max(rhoD, 0);
  const uint32_t rows = std::max(tN, tD);
  if (units && rows)
    hipLaunchKernelGGL(k_balance_rhs, dim3(cdiv(rows, 64), units), dim3(64), 0, s, M, T, X, A, B, degA, degB, beta,
                       tN, rhoN, vN, ldN, tD, vD, ldD);
  return hipGetLastError();
}

// ---- the balancing of many reconstructions in two launches
__global__ void k_balance_beta_batch(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix,
                                     const BalanceJob* __restrict__ jobs) {
  const uint32_t q = thiele_job_of(n, prefix, blockIdx.x);
  const BalanceJob& j = jobs[q];
  const uint32_t i = (blockIdx.x - prefix[q]) * blockDim.x + threadIdx.x;
  if (i >= j.T) return;
  const uint64_t a0 = horner_col(M, j.A, j.T, i, j.degA[i], j.X[0]);
  const uint64_t b0 = horner_col(M, j.B, j.T, i, j.degB[i], j.X[0]);
  uint64_t b = 0;
  if (j.nprev[i] != 0 && a0 != 0) b = zr_mul(M, j.nprev[i], zr_inv(M, a0));
  else if (j.dprev[i] != 0 && b0 != 0) b = zr_mul(M, j.dprev[i], zr_inv(M, b0));
  else *j.status = -4;  // ZR_EDEGEN for the whole reconstruction (every writer stores the same value)
  j.beta[i] = b;
}

__global__ void k_balance_rhs_batch(zr_mod M, uint32_t n, const uint32_t* __restrict__ prefix,
                                    const BalanceJob* __restrict__ jobs) {
  const uint32_t q = thiele_job_of(n, prefix, blockIdx.x);
  const BalanceJob& j = jobs[q];
  const uint32_t rows = std::max(j.tN, j.tD), nbx = cdiv(rows, 64);
  const uint32_t lb = blockIdx.x - prefix[q];
  const uint32_t i = (lb % nbx) * 64 + threadIdx.x, u = lb / nbx;
  if (u < (uint32_t)j.rhoN) {
    if (i < j.tN) j.vN[(size_t)u * j.ldN + i] = zr_mul(M, j.beta[i], horner_col(M, j.A, j.T, i, j.degA[i], j.X[u + 1]));
  } else {
    const uint32_t v = u - (uint32_t)j.rhoN;
    if (i < j.tD) j.vD[(size_t)v * j.ldD + i] = zr_mul(M, j.beta[i], horner_col(M, j.B, j.T, i, j.degB[i], j.X[v + 1]));
  }
}

uint32_t balance_beta_blocks(uint32_t T) { return cdiv(T, 64); }
uint32_t balance_rhs_blocks(uint32_t tN, uint32_t tD, int32_t rhoN, int32_t rhoD) {
  return cdiv(std::max(tN, tD), 64) * (uint32_t)(std::max(rhoN, 0) + std::max(rhoD, 0));
}

hipError_t balance_batch(const zr_mod& M, uint32_t n, const uint32_t* d_beta_prefix, uint32_t beta_total,
                         const uint32_t* d_rhs_prefix, uint32_t rhs_total, const BalanceJob* d_jobs, hipStream_t s) {
  if (n == 0) return hipSuccess;
  TimedLaunch tl("balance", s);
  if (beta_total) hipLaunchKernelGGL(k_balance_beta_batch, dim3(beta_total), dim3(64), 0, s, M, n, d_beta_prefix, d_jobs);
  if (rhs_total) hipLaunchKernelGGL(k_balance_rhs_batch, dim3(rhs_total), dim3(64), 0, s, M, n, d_rhs_prefix, d_jobs);
  return hipGetLastError();
}

// *out = code when any st[i] is nonzero (every writer stores the same value)
__global__ void k_fold_status(const int32_t* __restrict__ st, uint32_t T, int32_t* __restrict__ out, int32_t code) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < T && st[i] != 0) *out = code;
}

hipError_t fold_status(const int32_t* st, uint32_t T, int32_t* out, int32_t code, hipStream_t s) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_status, dim3(cdiv(T, 256)), dim3(256), 0, s, st, T, out, code);
  return hipGetLastError();
}

__global__ void k_scale(zr_mod M, uint64_t* v, size_t n, uint64_t c, uint64_t cp) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = zr_shoup(M, v[i], c, cp);
}

hipError_t scale_u64(const zr_mod& M, uint64_t* v, size_t n, uint64_t c, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(cdiv(n, 256)), dim3(256), 0, s, M, v, n, c, zr_shoup_pre(M, c));
  return hipGetLastError();
}

}  // namespace zr
