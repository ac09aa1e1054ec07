/* Host black box for synthetic workloads: evaluates a hidden sparse polynomial
 * (or a ratio P/Q) mod p at the structured points the reconstruction asks for.
 *
 * Input generation only.  It exploits the geometric structure of the Zippel
 * points (x_v = y_v^i for the already reconstructed variables): for each term h
 * the value at power i is w_h * Y_h^i with Y_h = prod_{v<k} y_v^e_{h,v}, so a
 * block of consecutive powers costs one multiplication per term and power plus
 * one multiply-accumulate per requested x_k value.
 *
 * Arithmetic: unsigned __int128 products reduced with %, sums kept below 2^127
 * by subtracting the largest multiple of p not above 2^127.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef unsigned __int128 u128;

typedef struct {
  uint64_t p;
  uint32_t nvars, nterms;
  const uint16_t *exps;   /* [nterms][nvars] */
  const uint64_t *coefs;  /* [nterms] */
} zs_poly;

typedef struct {
  zs_poly num, den;
  int32_t rational;
  int32_t nthreads;
} zs_box;

static inline uint64_t mm(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)(((u128)a * b) % p); }

static uint64_t pw(uint64_t a, uint64_t e, uint64_t p) {
  uint64_t r = 1 % p;
  a %= p;
  while (e) {
    if (e & 1) r = mm(r, a, p);
    a = mm(a, a, p);
    e >>= 1;
  }
  return r;
}

#define BLK 32

/* vals[jj*ni + ii] = poly at point (ii, jj) */
static void eval_poly(const zs_poly *P, uint32_t k, uint64_t i_first, uint64_t ni, const uint64_t *y,
                      const uint64_t *anchor, uint64_t nj, const uint64_t *xk, uint64_t *vals, int nthreads) {
  const uint64_t p = P->p;
  const uint32_t n = P->nvars, T = P->nterms;
  const u128 top = (u128)1 << 127;
  const u128 pbig = (top / p) * p;
  /* per-term constants */
  uint64_t *Y = (uint64_t *)malloc(sizeof(uint64_t) * (T ? T : 1));
  uint64_t *W = (uint64_t *)malloc(sizeof(uint64_t) * (T ? T : 1) * (nj ? nj : 1));
  /* k = nvars + 1: every variable at its Zippel power, no x_k (xk[0] unused) */
  const int has_xk = k <= n;
  uint32_t maxd = 0;
  for (uint32_t h = 0; h < T && has_xk; ++h)
    if (P->exps[(size_t)h * n + (k - 1)] > maxd) maxd = P->exps[(size_t)h * n + (k - 1)];
  uint64_t *xpow = (uint64_t *)malloc(sizeof(uint64_t) * (maxd + 1) * (nj ? nj : 1));
  for (uint64_t jj = 0; jj < nj; ++jj) {
    xpow[jj * (maxd + 1)] = 1 % p;
    for (uint32_t d = 1; d <= maxd; ++d) xpow[jj * (maxd + 1) + d] = mm(xpow[jj * (maxd + 1) + d - 1], xk[jj], p);
  }
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
  for (uint32_t h = 0; h < T; ++h) {
    const uint16_t *e = P->exps + (size_t)h * n;
    uint64_t yh = 1 % p, ah = P->coefs[h] % p;
    for (uint32_t v = 0; v + 1 < k && v < n; ++v) yh = mm(yh, pw(y[v], e[v], p), p);
    for (uint32_t v = k; v < n; ++v) ah = mm(ah, pw(anchor[v], e[v], p), p);
    Y[h] = yh;
    const uint32_t ek = has_xk ? e[k - 1] : 0;
    for (uint64_t jj = 0; jj < nj; ++jj) W[(size_t)h * nj + jj] = mm(ah, xpow[jj * (maxd + 1) + ek], p);
  }
  const uint64_t nblk = (ni + BLK - 1) / BLK;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
  {
    u128 *acc = (u128 *)malloc(sizeof(u128) * BLK * (nj ? nj : 1));
#pragma omp for schedule(dynamic, 1)
    for (uint64_t b = 0; b < nblk; ++b) {
      const uint64_t i0 = b * BLK;
      const uint64_t nb = (ni - i0 < BLK) ? (ni - i0) : BLK;
      memset(acc, 0, sizeof(u128) * BLK * nj);
      for (uint32_t h = 0; h < T; ++h) {
        uint64_t z = pw(Y[h], i_first + i0, p);
        const uint64_t *w = W + (size_t)h * nj;
        for (uint64_t ii = 0; ii < nb; ++ii) {
          for (uint64_t jj = 0; jj < nj; ++jj) {
            u128 *a = &acc[jj * BLK + ii];
            *a += (u128)w[jj] * z;
            if (*a >= top) *a -= pbig;
          }
          z = mm(z, Y[h], p);
        }
      }
      for (uint64_t jj = 0; jj < nj; ++jj)
        for (uint64_t ii = 0; ii < nb; ++ii) vals[jj * ni + i0 + ii] = (uint64_t)(acc[jj * BLK + ii] % p);
    }
    free(acc);
  }
  free(Y);
  free(W);
  free(xpow);
}

/* Returns 0 on success, 1 if a denominator vanishes at a requested point. */
int zs_eval_points(const void *ctx, uint32_t nvars, uint32_t k, uint64_t i_first, uint64_t ni,
                   const uint64_t *y, const uint64_t *anchor, uint64_t nj, const uint64_t *xk,
                   uint64_t *vals) {
  const zs_box *B = (const zs_box *)ctx;
  (void)nvars;
  if (ni == 0 || nj == 0) return 0;
  eval_poly(&B->num, k, i_first, ni, y, anchor, nj, xk, vals, B->nthreads);
  if (!B->rational) return 0;
  const uint64_t p = B->num.p;
  uint64_t *dv = (uint64_t *)malloc(sizeof(uint64_t) * ni * nj);
  eval_poly(&B->den, k, i_first, ni, y, anchor, nj, xk, dv, B->nthreads);
  int bad = 0;
  for (uint64_t i = 0; i < ni * nj; ++i) {
    if (dv[i] == 0) { bad = 1; break; }
    vals[i] = mm(vals[i], pw(dv[i], p - 2, p), p);
  }
  free(dv);
  return bad;
}

/* Stage-k grouping for the device black box: hidden terms sharing their
 * exponents on x_1..x_{k-1} (contiguous, the polynomial is lex-sorted) form one
 * group l with monomial value Y_l = prod_{v<k} y_v^e_v and weights
 * W[l][jj] = sum_{h in l} c_h * xk[jj]^e_{h,k} * prod_{v>k} anchor_v^e_{h,v}.
 * den != 0 selects the denominator of a rational box.
 * Y and W need capacity nterms and nterms*nj; returns the number of groups. */
uint64_t zs_group_stage(const void *ctx, int den, uint32_t k, const uint64_t *y, const uint64_t *anchor, uint64_t nj,
                        const uint64_t *xk, uint64_t *Y, uint64_t *W) {
  const zs_box *B = (const zs_box *)ctx;
  const zs_poly *P = den ? &B->den : &B->num;
  const uint64_t p = P->p;
  const uint32_t n = P->nvars, T = P->nterms;
  uint64_t ng = 0;
  uint64_t *start = (uint64_t *)malloc(sizeof(uint64_t) * (T + 1));
  for (uint32_t h = 0; h < T; ++h) {
    int same = h > 0;
    for (uint32_t v = 0; same && v + 1 < k && v < n; ++v) same = P->exps[(size_t)h * n + v] == P->exps[(size_t)(h - 1) * n + v];
    if (!same) start[ng++] = h;
  }
  start[ng] = T;
  /* k = nvars + 1: every variable at its Zippel power, no x_k (xk[0] unused) */
  const int has_xk = k <= n;
  uint32_t maxd = 0;
  for (uint32_t h = 0; h < T && has_xk; ++h)
    if (P->exps[(size_t)h * n + (k - 1)] > maxd) maxd = P->exps[(size_t)h * n + (k - 1)];
  uint64_t *xpow = (uint64_t *)malloc(sizeof(uint64_t) * (maxd + 1) * (nj ? nj : 1));
  for (uint64_t jj = 0; jj < nj; ++jj) {
    xpow[jj * (maxd + 1)] = 1 % p;
    for (uint32_t d = 1; d <= maxd; ++d) xpow[jj * (maxd + 1) + d] = mm(xpow[jj * (maxd + 1) + d - 1], xk[jj], p);
  }
#pragma omp parallel for schedule(dynamic, 64) num_threads(B->nthreads > 0 ? B->nthreads : omp_get_max_threads())
  for (uint64_t g = 0; g < ng; ++g) {
    const uint16_t *e0 = P->exps + (size_t)start[g] * n;
    uint64_t yv = 1 % p;
    for (uint32_t v = 0; v + 1 < k && v < n; ++v) yv = mm(yv, pw(y[v], e0[v], p), p);
    Y[g] = yv;
    for (uint64_t jj = 0; jj < nj; ++jj) W[g * nj + jj] = 0;
    for (uint64_t h = start[g]; h < start[g + 1]; ++h) {
      const uint16_t *e = P->exps + (size_t)h * n;
      uint64_t a = P->coefs[h] % p;
      for (uint32_t v = k; v < n; ++v) a = mm(a, pw(anchor[v], e[v], p), p);
      const uint32_t ek = has_xk ? e[k - 1] : 0;
      for (uint64_t jj = 0; jj < nj; ++jj) {
        uint64_t w = mm(a, xpow[jj * (maxd + 1) + ek], p);
        uint64_t s = W[g * nj + jj] + w;
        W[g * nj + jj] = s >= p ? s - p : s;
      }
    }
  }
  free(start);
  free(xpow);
  return ng;
}
