/* ORACLE — test infrastructure only.
 *
 * A plain, slow CPU implementation of sparse Zippel reconstruction over F_p
 * (polynomial and balanced rational variants), written from the paper
 * "GPU Implementation of Zippel Method for Feynman Integral Reconstruction"
 * (Smirnov, Rozhnov, Voevodin, 2025).  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product library never
 * does.  It shares no source with the HIP path.
 *
 * Arithmetic: every product is an unsigned __int128 reduced with the C %
 * operator (the textbook reduction, the paper's first mulmod variant in §2.1);
 * inverses by the extended Euclidean algorithm.  No lazy or deferred
 * reductions, no blocking: each routine is the definition written out.
 *
 * Readings of the paper that this file fixes (where it is silent):
 *  - Zippel powers are i = 1..t (§1), so sum_l a_l m_l^i = v_i and
 *    a_l = s_l / (m_l * q_l(m_l)).
 *  - One set of bases y_v for all stages; stage k uses y_1..y_{k-1}.
 *  - Node 0 of each variable is its anchor c_v; further nodes come from the
 *    schedule.  The polynomial path uses exactly D_k+1 nodes for x_k.
 *  - Thiele (eq. 2) stops at the first m for which the continued fraction
 *    b_0..b_m reproduces the sample at node m+1.
 *  - Balanced Zippel (§2.2, balancing equation): slice normalisation makes
 *    the lowest nonzero denominator coefficient 1; the slice scale
 *    beta_i = N_{k-1}(y^i)/A_i(c_k), falling back to the denominator.
 *  - Final rational normalisation: the denominator's constant term is 1.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef unsigned __int128 u128;

enum {
  OR_OK = 0, OR_EINVAL = -1, OR_ENOTPRIME = -2, OR_ESINGULAR = -3, OR_EDEGEN = -4,
  OR_EPROBE = -5, OR_ENORM = -6, OR_ENOMEM = -7, OR_EBLACKBOX = -9
};

/* Black box: values at the nj*ni points (jj, ii) with x_v = y_v^(i_first+ii) for
 * v < k, x_k = xk[jj], x_v = anchor_v for v > k (k 1-based); vals[jj*ni+ii]. */
typedef int (*or_blackbox)(void *ctx, uint32_t nvars, uint32_t k, uint64_t i_first, uint64_t ni,
                           const uint64_t *y, const uint64_t *anchor, uint64_t nj, const uint64_t *xk,
                           uint64_t *vals);

typedef struct {
  uint32_t nvars;
  uint64_t nterms;
  uint16_t *exps;  /* [nterms][nvars] */
  uint64_t *coefs; /* [nterms] */
} or_poly;

static int nthreads_of(int n) { return n > 0 ? n : omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* F_p                                                                      */

uint64_t or_mul(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)(((u128)a * b) % p); }
uint64_t or_add(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)(((u128)a + b) % p); }
uint64_t or_sub(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)(((u128)a + p - b % p) % p); }

uint64_t or_pow(uint64_t a, uint64_t e, uint64_t p) {
  uint64_t r = 1 % p;
  a %= p;
  while (e) {
    if (e & 1) r = or_mul(r, a, p);
    a = or_mul(a, a, p);
    e >>= 1;
  }
  return r;
}

/* a^{-1} mod p by the extended Euclidean algorithm; 0 if a = 0 mod p. */
uint64_t or_inv(uint64_t a, uint64_t p) {
  int64_t t0 = 0, t1 = 1;  /* signed 64-bit suffices: |t| <= p < 2^63 */
  uint64_t r0 = p, r1 = a % p;
  if (r1 == 0) return 0;
  while (r1 != 0) {
    uint64_t q = r0 / r1;
    uint64_t r2 = r0 - q * r1;
    __int128 t2 = (__int128)t0 - (__int128)q * t1;
    r0 = r1; r1 = r2;
    t0 = t1; t1 = (int64_t)t2;
  }
  if (r0 != 1) return 0;
  return t0 < 0 ? (uint64_t)(t0 + (int64_t)p) : (uint64_t)t0;
}

/* Deterministic Miller-Rabin: the first twelve prime bases decide every n < 2^64. */
int or_is_prime(uint64_t n) {
  static const uint64_t B[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i)
    if (n % B[i] == 0) return n == B[i];
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = or_pow(B[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int r = 1; r < s; ++r) {
      x = or_mul(x, x, n);
      if (x == n - 1) { comp = 0; break; }
    }
    if (comp) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Dense linear algebra: Gauss-Jordan elimination mod p (the O(t^3) solve of §1) */

/* Solves A X = Bm for X; A [n][n] row-major, Bm and X [n][nrhs] row-major.
 * Returns OR_ESINGULAR if A is singular.  A and Bm are not modified. */
int or_gauss_solve(uint64_t p, size_t n, const uint64_t *A, size_t nrhs, const uint64_t *Bm, uint64_t *X) {
  size_t w = n + nrhs;
  uint64_t *T = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1) * (w ? w : 1));
  if (!T) return OR_ENOMEM;
  for (size_t i = 0; i < n; ++i) {
    for (size_t j = 0; j < n; ++j) T[i * w + j] = A[i * n + j] % p;
    for (size_t j = 0; j < nrhs; ++j) T[i * w + n + j] = Bm[i * nrhs + j] % p;
  }
  for (size_t c = 0; c < n; ++c) {
    size_t piv = n;
    for (size_t r = c; r < n; ++r)
      if (T[r * w + c] != 0) { piv = r; break; }
    if (piv == n) { free(T); return OR_ESINGULAR; }
    if (piv != c)
      for (size_t j = 0; j < w; ++j) { uint64_t tmp = T[c * w + j]; T[c * w + j] = T[piv * w + j]; T[piv * w + j] = tmp; }
    uint64_t iv = or_inv(T[c * w + c], p);
    for (size_t j = 0; j < w; ++j) T[c * w + j] = or_mul(T[c * w + j], iv, p);
    for (size_t r = 0; r < n; ++r) {
      if (r == c || T[r * w + c] == 0) continue;
      uint64_t f = T[r * w + c];
      for (size_t j = 0; j < w; ++j) T[r * w + j] = or_sub(T[r * w + j], or_mul(f, T[c * w + j], p), p);
    }
  }
  for (size_t i = 0; i < n; ++i)
    for (size_t j = 0; j < nrhs; ++j) X[i * nrhs + j] = T[i * w + n + j];
  free(T);
  return OR_OK;
}

/* The Zippel system of §1 solved by Gauss-Jordan: sum_l a_l m_l^i = v_i for
 * i = 1..t, rhs/out laid out [R][t]. */
int or_gauss_vandermonde(uint64_t p, size_t t, const uint64_t *m, size_t R, const uint64_t *rhs, uint64_t *out) {
  uint64_t *A = (uint64_t *)malloc(sizeof(uint64_t) * (t * t + 1));
  uint64_t *B = (uint64_t *)malloc(sizeof(uint64_t) * (t * R + 1));
  uint64_t *X = (uint64_t *)malloc(sizeof(uint64_t) * (t * R + 1));
  if (!A || !B || !X) { free(A); free(B); free(X); return OR_ENOMEM; }
  for (size_t i = 0; i < t; ++i)
    for (size_t l = 0; l < t; ++l) A[i * t + l] = or_pow(m[l], i + 1, p);
  for (size_t i = 0; i < t; ++i)
    for (size_t j = 0; j < R; ++j) B[i * R + j] = rhs[j * t + i];
  int st = or_gauss_solve(p, t, A, R, B, X);
  if (st == OR_OK)
    for (size_t l = 0; l < t; ++l)
      for (size_t j = 0; j < R; ++j) out[j * t + l] = X[l * R + j];
  free(A); free(B); free(X);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Transposed Vandermonde solve in O(t^2) through the master polynomial and
 * the Lagrange basis (§1 and the step list of §2.2)                        */

/* M(z) = prod_l (z - m_l) = sum_{r=0}^t M[r] z^r, built one factor at a time. */
void or_master(uint64_t p, size_t t, const uint64_t *m, uint64_t *M) {
  M[0] = 1 % p;
  for (size_t l = 0; l < t; ++l) {
    /* multiply the degree-l polynomial M[0..l] by (z - m_l) */
    M[l + 1] = M[l];
    for (size_t r = l; r >= 1; --r) M[r] = or_sub(M[r - 1], or_mul(m[l], M[r], p), p);
    M[0] = or_sub(0, or_mul(m[l], M[0], p), p);
  }
}

/* One row l of the solve.  q_l(z) = M(z)/(z - m_l) by synthetic division
 * (q_{t-1} = 1, q_{r-1} = M_r + m_l q_r), s^(j) = sum_r q_{l,r} v^(j)_{r+1},
 * delta = q_l(m_l) by Horner, a^(j) = s^(j) / (m_l delta). */
static int solve_row(uint64_t p, size_t t, const uint64_t *m, const uint64_t *M, size_t R, const uint64_t *rhs,
                     size_t l, uint64_t *a /* [R] */) {
  const uint64_t ml = m[l] % p;
  uint64_t *s = (uint64_t *)calloc(R ? R : 1, sizeof(uint64_t));
  uint64_t q = 1 % p, h = 0;
  for (size_t rr = t; rr-- > 0;) {
    /* q holds q_{l,rr} */
    for (size_t j = 0; j < R; ++j) s[j] = or_add(s[j], or_mul(q, rhs[j * t + rr], p), p);
    h = or_add(or_mul(h, ml, p), q, p);
    q = or_add(M[rr], or_mul(ml, q, p), p);
  }
  /* q now holds the remainder M(m_l), which is zero by construction */
  uint64_t w = or_mul(ml, h, p);
  int st = OR_OK;
  if (w == 0 || q != 0) {
    st = OR_ESINGULAR;
    for (size_t j = 0; j < R; ++j) a[j] = 0;
  } else {
    uint64_t wi = or_inv(w, p);
    for (size_t j = 0; j < R; ++j) a[j] = or_mul(s[j], wi, p);
  }
  free(s);
  return st;
}

/* sum_l a_l m_l^i = v_i, i = 1..t; rhs and out [R][t].  ESINGULAR if two m_l
 * coincide or one is zero. */
int or_vandermonde_solve(uint64_t p, size_t t, const uint64_t *m, size_t R, const uint64_t *rhs, uint64_t *out,
                         int nthreads) {
  if (t == 0) return OR_OK;
  uint64_t *M = (uint64_t *)malloc(sizeof(uint64_t) * (t + 1));
  if (!M) return OR_ENOMEM;
  or_master(p, t, m, M);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads_of(nthreads)) reduction(| : bad)
  for (size_t l = 0; l < t; ++l) {
    uint64_t *a = (uint64_t *)malloc(sizeof(uint64_t) * (R ? R : 1));
    if (solve_row(p, t, m, M, R, rhs, l, a) != OR_OK) bad = 1;
    for (size_t j = 0; j < R; ++j) out[j * t + l] = a[j];
    free(a);
  }
  free(M);
  return bad ? OR_ESINGULAR : OR_OK;
}

/* The same solve restricted to rows[0..nrows): out [R][nrows]. */
int or_vandermonde_solve_rows(uint64_t p, size_t t, const uint64_t *m, size_t R, const uint64_t *rhs, size_t nrows,
                              const uint64_t *rows, uint64_t *out, int nthreads) {
  uint64_t *M = (uint64_t *)malloc(sizeof(uint64_t) * (t + 1));
  if (!M) return OR_ENOMEM;
  or_master(p, t, m, M);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads_of(nthreads)) reduction(| : bad)
  for (size_t k = 0; k < nrows; ++k) {
    uint64_t *a = (uint64_t *)malloc(sizeof(uint64_t) * (R ? R : 1));
    if (solve_row(p, t, m, M, R, rhs, (size_t)rows[k], a) != OR_OK) bad = 1;
    for (size_t j = 0; j < R; ++j) out[j * nrows + k] = a[j];
    free(a);
  }
  free(M);
  return bad ? OR_ESINGULAR : OR_OK;
}

/* Multiply-back: out[ii] = sum_l a_l m_l^(i_first+ii). */
void or_vandermonde_apply(uint64_t p, size_t t, const uint64_t *m, const uint64_t *a, uint64_t i_first, size_t ni,
                          uint64_t *out) {
  for (size_t ii = 0; ii < ni; ++ii) out[ii] = 0;
  for (size_t l = 0; l < t; ++l) {
    uint64_t z = or_pow(m[l], i_first, p);
    for (size_t ii = 0; ii < ni; ++ii) {
      out[ii] = or_add(out[ii], or_mul(a[l], z, p), p);
      z = or_mul(z, m[l], p);
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Univariate Newton interpolation (eq. 1)                                  */

/* Values f(x_0..x_d) at distinct nodes -> monomial coefficients c[0..d]. */
int or_newton(uint64_t p, size_t d1 /* = d+1 */, const uint64_t *x, const uint64_t *f, uint64_t *c) {
  uint64_t *dd = (uint64_t *)malloc(sizeof(uint64_t) * (d1 ? d1 : 1));
  for (size_t i = 0; i < d1; ++i) dd[i] = f[i] % p;
  /* divided differences: dd[i] becomes f[x_0..x_i] */
  for (size_t j = 1; j < d1; ++j)
    for (size_t i = d1 - 1; i >= j; --i) {
      uint64_t den = or_sub(x[i], x[i - j], p);
      if (den == 0) { free(dd); return OR_EINVAL; }
      dd[i] = or_mul(or_sub(dd[i], dd[i - 1], p), or_inv(den, p), p);
    }
  /* nested form a_1 + (x-x_1)[a_2 + (x-x_2)[...]] expanded from the inside */
  for (size_t i = 0; i < d1; ++i) c[i] = 0;
  if (d1 == 0) { free(dd); return OR_OK; }
  c[0] = dd[d1 - 1];
  for (size_t i = d1 - 1; i-- > 0;) {
    /* c <- c * (x - x_i) + dd[i]; c currently has degree d1-2-i */
    size_t deg = d1 - 2 - i;
    c[deg + 1] = c[deg];
    for (size_t r = deg; r >= 1; --r) c[r] = or_sub(c[r - 1], or_mul(x[i], c[r], p), p);
    c[0] = or_add(or_sub(0, or_mul(x[i], c[0], p), p), dd[i], p);
  }
  free(dd);
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Univariate Thiele reconstruction (eq. 2)                                 */

/* Continued fraction b_0 + (x-x_0)/(b_1 + (x-x_1)/(... + (x-x_{m-1})/b_m)) at
 * x; returns 0 on a zero divisor (then *ok = 0). */
static uint64_t cf_eval(uint64_t p, const uint64_t *b, const uint64_t *xs, size_t m, uint64_t x, int *ok) {
  uint64_t v = b[m];
  *ok = 1;
  for (size_t s = m; s-- > 0;) {
    if (v == 0) { *ok = 0; return 0; }
    v = or_add(b[s], or_mul(or_sub(x, xs[s], p), or_inv(v, p), p), p);
  }
  return v;
}

/* From samples f at nodes x[0..n), find the shortest continued fraction
 * b_0..b_m whose value at node m+1 matches the sample there, convert it to
 * A/B, strip leading zeros and scale so that the lowest nonzero coefficient
 * of B is 1.  A and B need capacity n.  Returns EPROBE if no m <= n-2 is
 * confirmed, EDEGEN on a vanishing inverse difference. */
int or_thiele(uint64_t p, size_t n, const uint64_t *x, const uint64_t *f, uint64_t *A, uint64_t *B, int32_t *degA,
              int32_t *degB) {
  if (n < 2) return OR_EINVAL;
  uint64_t *phi = (uint64_t *)malloc(sizeof(uint64_t) * n);
  uint64_t *b = (uint64_t *)malloc(sizeof(uint64_t) * n);
  uint64_t *PA = (uint64_t *)calloc(n + 1, sizeof(uint64_t));
  uint64_t *PB = (uint64_t *)calloc(n + 1, sizeof(uint64_t));
  uint64_t *NA = (uint64_t *)calloc(n + 1, sizeof(uint64_t));
  int st = OR_OK;
  for (size_t i = 0; i < n; ++i) phi[i] = f[i] % p;  /* phi_0 */
  b[0] = phi[0];
  size_t m = 0;
  for (;;) {
    if (m + 1 >= n) { st = OR_EPROBE; goto done; }
    int ok;
    uint64_t val = cf_eval(p, b, x, m, x[m + 1], &ok);
    if (ok && val == f[m + 1] % p) break;
    /* phi_{m+1}(x_i) = (x_i - x_m) / (phi_m(x_i) - phi_m(x_m)) for i > m */
    for (size_t i = m + 1; i < n; ++i) {
      uint64_t den = or_sub(phi[i], phi[m], p);
      if (den == 0) { st = OR_EDEGEN; goto done; }
      phi[i] = or_mul(or_sub(x[i], x[m], p), or_inv(den, p), p);
    }
    b[m + 1] = phi[m + 1];
    ++m;
  }
  /* (A, B) <- (b_m, 1); then (A, B) <- (b_s A + (x - x_s) B, A) for s = m-1..0 */
  PA[0] = b[m];
  PB[0] = 1 % p;
  for (size_t s = m; s-- > 0;) {
    for (size_t r = 0; r <= n; ++r) {
      uint64_t v = or_mul(b[s], PA[r], p);
      v = or_sub(v, or_mul(x[s], PB[r], p), p);
      if (r > 0) v = or_add(v, PB[r - 1], p);
      NA[r] = v;
    }
    memcpy(PB, PA, sizeof(uint64_t) * (n + 1));
    memcpy(PA, NA, sizeof(uint64_t) * (n + 1));
  }
  {
    int32_t da = -1, db = -1;
    for (size_t r = 0; r <= n; ++r) {
      if (PA[r]) da = (int32_t)r;
      if (PB[r]) db = (int32_t)r;
    }
    if (db < 0) { st = OR_EDEGEN; goto done; }
    size_t low = 0;
    while (PB[low] == 0) ++low;
    uint64_t sc = or_inv(PB[low], p);
    for (int32_t r = 0; r <= (da > 0 ? da : 0); ++r) A[r] = or_mul(PA[r], sc, p);
    for (int32_t r = 0; r <= db; ++r) B[r] = or_mul(PB[r], sc, p);
    if (da < 0) { A[0] = 0; da = 0; }
    *degA = da;
    *degB = db;
  }
done:
  free(phi); free(b); free(PA); free(PB); free(NA);
  return st;
}

static uint64_t horner(uint64_t p, const uint64_t *c, int32_t deg, uint64_t x) {
  uint64_t v = 0;
  for (int32_t r = deg; r >= 0; --r) v = or_add(or_mul(v, x, p), c[r], p);
  return v;
}

/* ------------------------------------------------------------------------ */
/* Sparse polynomials                                                       */

static or_poly *poly_new(uint32_t nvars, uint64_t nterms) {
  or_poly *P = (or_poly *)calloc(1, sizeof(or_poly));
  P->nvars = nvars;
  P->nterms = nterms;
  P->exps = (uint16_t *)calloc((nterms ? nterms : 1) * (nvars ? nvars : 1), sizeof(uint16_t));
  P->coefs = (uint64_t *)calloc(nterms ? nterms : 1, sizeof(uint64_t));
  return P;
}

void or_poly_free(or_poly *P) {
  if (!P) return;
  free(P->exps);
  free(P->coefs);
  free(P);
}

uint64_t or_poly_nterms(const or_poly *P) { return P->nterms; }
const uint16_t *or_poly_exps(const or_poly *P) { return P->exps; }
const uint64_t *or_poly_coefs(const or_poly *P) { return P->coefs; }

/* Value at one point, directly from the definition. */
uint64_t or_poly_eval(uint64_t p, uint32_t nvars, uint64_t nterms, const uint16_t *exps, const uint64_t *coefs,
                      const uint64_t *pt) {
  uint64_t s = 0;
  for (uint64_t h = 0; h < nterms; ++h) {
    uint64_t v = coefs[h] % p;
    for (uint32_t j = 0; j < nvars; ++j) v = or_mul(v, or_pow(pt[j], exps[h * nvars + j], p), p);
    s = or_add(s, v, p);
  }
  return s;
}

/* Monomial values m_l = prod_{v<k-1} y_v^{e_{l,v}} (0-based v; stage k is 1-based). */
static void monomials(uint64_t p, const or_poly *S, uint32_t k, const uint64_t *y, uint64_t *m) {
  for (uint64_t l = 0; l < S->nterms; ++l) {
    uint64_t v = 1 % p;
    for (uint32_t j = 0; j + 1 < k; ++j) v = or_mul(v, or_pow(y[j], S->exps[l * S->nvars + j], p), p);
    m[l] = v;
  }
}

/* Lift a skeleton over x_k: values vals[j][l] of each term's coefficient at
 * nodes X[0..R] (j = 0 is the skeleton itself) -> Newton in x_k -> expanded
 * skeleton with terms (e_l, d), lexicographic order preserved. */
static int lift(uint64_t p, const or_poly *S, uint32_t k, size_t R1, const uint64_t *X, const uint64_t *vals,
                or_poly **out, int nthreads) {
  const uint64_t t = S->nterms;
  uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * (t * R1 + 1));
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads_of(nthreads)) reduction(| : bad)
  for (uint64_t l = 0; l < t; ++l) {
    uint64_t *f = (uint64_t *)malloc(sizeof(uint64_t) * R1);
    for (size_t j = 0; j < R1; ++j) f[j] = vals[j * t + l];
    if (or_newton(p, R1, X, f, g + l * R1) != OR_OK) bad = 1;
    free(f);
  }
  if (bad) { free(g); return OR_EINVAL; }
  uint64_t cnt = 0;
  for (uint64_t i = 0; i < t * R1; ++i) cnt += g[i] != 0;
  or_poly *N = poly_new(S->nvars, cnt);
  uint64_t pos = 0;
  for (uint64_t l = 0; l < t; ++l)
    for (size_t d = 0; d < R1; ++d) {
      if (g[l * R1 + d] == 0) continue;
      memcpy(N->exps + pos * S->nvars, S->exps + l * S->nvars, sizeof(uint16_t) * S->nvars);
      N->exps[pos * S->nvars + (k - 1)] = (uint16_t)d;
      N->coefs[pos] = g[l * R1 + d];
      ++pos;
    }
  free(g);
  *out = N;
  return OR_OK;
}

/* Node list of variable v (0-based): anchor, then its schedule nodes. */
static void node_list(const uint64_t *anchor, const uint64_t *nodes, const uint32_t *nnodes, uint32_t v, size_t cnt,
                      uint64_t *X) {
  size_t off = 0;
  for (uint32_t u = 0; u < v; ++u) off += nnodes[u];
  X[0] = anchor[v];
  for (size_t j = 1; j < cnt; ++j) X[j] = nodes[off + j - 1];
}

static int check_probes(uint64_t p, uint32_t n, const or_poly *N, const or_poly *D, uint32_t nprobes,
                        const uint64_t *probes, const uint64_t *anchor, or_blackbox bb, void *ctx) {
  for (uint32_t q = 0; q < nprobes; ++q) {
    const uint64_t *pt = probes + (size_t)q * n;
    uint64_t val;
    uint64_t one = 1;
    if (bb(ctx, n, n, 1, 1, pt, anchor, 1, pt + (n - 1), &val) != 0) return OR_EBLACKBOX;
    (void)one;
    uint64_t nv = or_poly_eval(p, n, N->nterms, N->exps, N->coefs, pt);
    if (D) {
      uint64_t dv = or_poly_eval(p, n, D->nterms, D->exps, D->coefs, pt);
      if (nv != or_mul(val, dv, p)) return OR_EPROBE;
    } else if (nv != val) {
      return OR_EPROBE;
    }
  }
  return OR_OK;
}

static int check_common(uint64_t p, uint32_t nvars, const uint32_t *deg, const uint64_t *y, const uint64_t *anchor) {
  if (p < 3 || p >= ((uint64_t)1 << 63) || nvars == 0 || nvars > 64 || !deg || !y || !anchor) return OR_EINVAL;
  if (!or_is_prime(p)) return OR_ENOTPRIME;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Polynomial Zippel (§1): stage 1 is Newton in x_1; stage k >= 2 solves one
 * transposed Vandermonde system of size t = |S_{k-1}| with D_k right-hand
 * sides (values at x_k = node 1..D_k) and lifts each term by Newton in x_k.
 * last_stage (1..n) stops early and returns f(x_1..x_L, anchors).          */
int or_zippel(uint64_t p, uint32_t nvars, const uint32_t *deg, const uint64_t *y, const uint64_t *anchor,
              const uint64_t *nodes, const uint32_t *nnodes, uint32_t nprobes, const uint64_t *probes,
              uint32_t last_stage, or_blackbox bb, void *ctx, int nthreads, or_poly **out) {
  int st = check_common(p, nvars, deg, y, anchor);
  if (st) return st;
  for (uint32_t v = 0; v < nvars; ++v)
    if (nnodes[v] < deg[v]) return OR_EINVAL;
  const uint32_t L = (last_stage == 0 || last_stage > nvars) ? nvars : last_stage;
  /* stage 1 */
  size_t R1 = (size_t)deg[0] + 1;
  uint64_t *X = (uint64_t *)malloc(sizeof(uint64_t) * (R1 + 1));
  node_list(anchor, nodes, nnodes, 0, R1, X);
  uint64_t *f = (uint64_t *)malloc(sizeof(uint64_t) * R1);
  if (bb(ctx, nvars, 1, 1, 1, y, anchor, R1, X, f) != 0) { free(X); free(f); return OR_EBLACKBOX; }
  or_poly *root = poly_new(nvars, 1);
  root->coefs[0] = 1 % p; /* the empty monomial; its single value list is f */
  or_poly *S = NULL;
  st = lift(p, root, 1, R1, X, f, &S, nthreads);
  or_poly_free(root);
  free(X); free(f);
  if (st) return st;
  for (uint32_t k = 2; k <= L && st == OR_OK; ++k) {
    const uint64_t t = S->nterms;
    const size_t R = deg[k - 1];
    R1 = R + 1;
    X = (uint64_t *)malloc(sizeof(uint64_t) * (R1 + 1));
    node_list(anchor, nodes, nnodes, k - 1, R1, X);
    uint64_t *m = (uint64_t *)malloc(sizeof(uint64_t) * (t + 1));
    uint64_t *vals = (uint64_t *)malloc(sizeof(uint64_t) * (t * R1 + 1));
    monomials(p, S, k, y, m);
    /* values at node 0 are the skeleton's coefficients */
    for (uint64_t l = 0; l < t; ++l) vals[l] = S->coefs[l];
    if (R > 0 && t > 0) {
      uint64_t *rhs = (uint64_t *)malloc(sizeof(uint64_t) * (t * R + 1));
      if (bb(ctx, nvars, k, 1, t, y, anchor, R, X + 1, rhs) != 0) st = OR_EBLACKBOX;
      if (st == OR_OK) st = or_vandermonde_solve(p, t, m, R, rhs, vals + t, nthreads);
      free(rhs);
    }
    or_poly *Sn = NULL;
    if (st == OR_OK) st = lift(p, S, k, R1, X, vals, &Sn, nthreads);
    free(X); free(m); free(vals);
    if (st == OR_OK) { or_poly_free(S); S = Sn; }
  }
  if (st == OR_OK && L == nvars && nprobes > 0) st = check_probes(p, nvars, S, NULL, nprobes, probes, anchor, bb, ctx);
  if (st != OR_OK) { or_poly_free(S); return st; }
  *out = S;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Balanced Zippel for f = P/Q (§1, §2.2 balancing equation).  Stage 1:
 * Thiele in x_1 gives N_1/D_1.  Stage k: per slice i = 1..T Thiele in x_k at
 * x_{<k} = y^i gives A_i/B_i; beta_i = N_{k-1}(y^i)/A_i(c_k) removes the
 * slice's unknown scale so beta_i A_i(node j) and beta_i B_i(node j) are the
 * values of one common multiple C*P and C*Q; numerator and denominator are
 * then each lifted by the polynomial step.  At the end D(0) is scaled to 1.  */

static int thiele_slice(uint64_t p, size_t n, const uint64_t *X, const uint64_t *fv, uint64_t *A, uint64_t *B,
                        int32_t *da, int32_t *db) {
  return or_thiele(p, n, X, fv, A, B, da, db);
}

int or_balanced_zippel(uint64_t p, uint32_t nvars, const uint32_t *degN, const uint32_t *degD, const uint64_t *y,
                       const uint64_t *anchor, const uint64_t *nodes, const uint32_t *nnodes, uint32_t nprobes,
                       const uint64_t *probes, uint32_t last_stage, or_blackbox bb, void *ctx, int nthreads,
                       or_poly **num, or_poly **den) {
  int st = check_common(p, nvars, degN, y, anchor);
  if (st) return st;
  if (!degD) return OR_EINVAL;
  for (uint32_t v = 0; v < nvars; ++v) {
    uint32_t m = 2 * degN[v] > 0 ? 2 * degN[v] - 1 : 0;
    if (2 * degD[v] > m) m = 2 * degD[v];
    if (nnodes[v] < m + 1) return OR_EINVAL;
  }
  const uint32_t L = (last_stage == 0 || last_stage > nvars) ? nvars : last_stage;
  or_poly *SN = NULL, *SD = NULL;
  /* stage 1 */
  {
    size_t n1 = (size_t)nnodes[0] + 1;
    uint64_t *X = (uint64_t *)malloc(sizeof(uint64_t) * n1);
    uint64_t *fv = (uint64_t *)malloc(sizeof(uint64_t) * n1);
    uint64_t *A = (uint64_t *)calloc(n1 + 1, sizeof(uint64_t));
    uint64_t *B = (uint64_t *)calloc(n1 + 1, sizeof(uint64_t));
    node_list(anchor, nodes, nnodes, 0, n1, X);
    int32_t da, db;
    if (bb(ctx, nvars, 1, 1, 1, y, anchor, n1, X, fv) != 0) st = OR_EBLACKBOX;
    if (st == OR_OK) st = thiele_slice(p, n1, X, fv, A, B, &da, &db);
    if (st == OR_OK && (da > (int32_t)degN[0] || db > (int32_t)degD[0])) st = OR_EDEGEN;
    if (st == OR_OK) {
      uint64_t cn = 0, cd = 0;
      for (int32_t r = 0; r <= da; ++r) cn += A[r] != 0;
      for (int32_t r = 0; r <= db; ++r) cd += B[r] != 0;
      SN = poly_new(nvars, cn);
      SD = poly_new(nvars, cd);
      uint64_t a = 0, b = 0;
      for (int32_t r = 0; r <= da; ++r)
        if (A[r]) { SN->exps[a * nvars] = (uint16_t)r; SN->coefs[a++] = A[r]; }
      for (int32_t r = 0; r <= db; ++r)
        if (B[r]) { SD->exps[b * nvars] = (uint16_t)r; SD->coefs[b++] = B[r]; }
    }
    free(X); free(fv); free(A); free(B);
  }
  for (uint32_t k = 2; k <= L && st == OR_OK; ++k) {
    const uint64_t tN = SN->nterms, tD = SD->nterms, T = tN > tD ? tN : tD;
    const size_t nk = (size_t)nnodes[k - 1] + 1;
    uint64_t *X = (uint64_t *)malloc(sizeof(uint64_t) * nk);
    node_list(anchor, nodes, nnodes, k - 1, nk, X);
    uint64_t *F = (uint64_t *)malloc(sizeof(uint64_t) * (T * nk + 1));
    uint64_t *mN = (uint64_t *)malloc(sizeof(uint64_t) * (tN + 1));
    uint64_t *mD = (uint64_t *)malloc(sizeof(uint64_t) * (tD + 1));
    uint64_t *Ai = (uint64_t *)calloc(T * (nk + 1) + 1, sizeof(uint64_t));
    uint64_t *Bi = (uint64_t *)calloc(T * (nk + 1) + 1, sizeof(uint64_t));
    int32_t *dA = (int32_t *)malloc(sizeof(int32_t) * (T + 1));
    int32_t *dB = (int32_t *)malloc(sizeof(int32_t) * (T + 1));
    uint64_t *nprev = (uint64_t *)malloc(sizeof(uint64_t) * (T + 1));
    uint64_t *dprev = (uint64_t *)malloc(sizeof(uint64_t) * (T + 1));
    uint64_t *beta = (uint64_t *)malloc(sizeof(uint64_t) * (T + 1));
    monomials(p, SN, k, y, mN);
    monomials(p, SD, k, y, mD);
    if (bb(ctx, nvars, k, 1, T, y, anchor, nk, X, F) != 0) st = OR_EBLACKBOX;
    int bad = 0;
    if (st == OR_OK) {
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads_of(nthreads)) reduction(min : bad)
      for (uint64_t i = 0; i < T; ++i) {
        uint64_t *fv = (uint64_t *)malloc(sizeof(uint64_t) * nk);
        for (size_t j = 0; j < nk; ++j) fv[j] = F[j * T + i];
        int s2 = thiele_slice(p, nk, X, fv, Ai + i * (nk + 1), Bi + i * (nk + 1), &dA[i], &dB[i]);
        if (s2 < bad) bad = s2;
        free(fv);
      }
      st = bad;
    }
    int32_t rhoN = 0, rhoD = 0;
    if (st == OR_OK && T > 0) {
      rhoN = dA[0]; rhoD = dB[0];
      for (uint64_t i = 0; i < T; ++i)
        if (dA[i] != rhoN || dB[i] != rhoD) st = OR_EDEGEN;
      if (rhoN > (int32_t)degN[k - 1] || rhoD > (int32_t)degD[k - 1]) st = OR_EDEGEN;
    }
    if (st == OR_OK) {
      /* N_{k-1}(y^i), D_{k-1}(y^i) for i = 1..T: transposed Vandermonde apply */
      or_vandermonde_apply(p, tN, mN, SN->coefs, 1, T, nprev);
      or_vandermonde_apply(p, tD, mD, SD->coefs, 1, T, dprev);
      for (uint64_t i = 0; i < T && st == OR_OK; ++i) {
        uint64_t a0 = horner(p, Ai + i * (nk + 1), dA[i], X[0]);
        uint64_t b0 = horner(p, Bi + i * (nk + 1), dB[i], X[0]);
        if (nprev[i] != 0 && a0 != 0) beta[i] = or_mul(nprev[i], or_inv(a0, p), p);
        else if (dprev[i] != 0 && b0 != 0) beta[i] = or_mul(dprev[i], or_inv(b0, p), p);
        else st = OR_EDEGEN;
      }
    }
    or_poly *newN = NULL, *newD = NULL;
    for (int side = 0; side < 2 && st == OR_OK; ++side) {
      const or_poly *S = side == 0 ? SN : SD;
      const uint64_t *mm = side == 0 ? mN : mD;
      const int32_t rho = side == 0 ? rhoN : rhoD;
      const uint64_t *C = side == 0 ? Ai : Bi;
      const int32_t *dc = side == 0 ? dA : dB;
      const uint64_t t = S->nterms;
      const size_t R1 = (size_t)rho + 1;
      uint64_t *vals = (uint64_t *)malloc(sizeof(uint64_t) * (t * R1 + 1));
      for (uint64_t l = 0; l < t; ++l) vals[l] = S->coefs[l];
      if (rho > 0 && t > 0) {
        uint64_t *rhs = (uint64_t *)malloc(sizeof(uint64_t) * (t * rho + 1));
        for (int32_t j = 1; j <= rho; ++j)
          for (uint64_t i = 0; i < t; ++i)
            rhs[(size_t)(j - 1) * t + i] = or_mul(beta[i], horner(p, C + i * (nk + 1), dc[i], X[j]), p);
        st = or_vandermonde_solve(p, t, mm, (size_t)rho, rhs, vals + t, nthreads);
        free(rhs);
      }
      if (st == OR_OK) st = lift(p, S, k, R1, X, vals, side == 0 ? &newN : &newD, nthreads);
      free(vals);
    }
    free(X); free(F); free(mN); free(mD); free(Ai); free(Bi); free(dA); free(dB);
    free(nprev); free(dprev); free(beta);
    if (st == OR_OK) {
      or_poly_free(SN); or_poly_free(SD);
      SN = newN; SD = newD;
    } else {
      or_poly_free(newN); or_poly_free(newD);
    }
  }
  if (st == OR_OK && L == nvars) {
    /* normalise: the denominator's constant term becomes 1 */
    uint64_t c0 = 0;
    for (uint64_t h = 0; h < SD->nterms; ++h) {
      int zero = 1;
      for (uint32_t v = 0; v < nvars; ++v) zero &= SD->exps[h * nvars + v] == 0;
      if (zero) { c0 = SD->coefs[h]; break; }
    }
    if (c0 == 0) st = OR_ENORM;
    else {
      uint64_t ci = or_inv(c0, p);
      for (uint64_t h = 0; h < SN->nterms; ++h) SN->coefs[h] = or_mul(SN->coefs[h], ci, p);
      for (uint64_t h = 0; h < SD->nterms; ++h) SD->coefs[h] = or_mul(SD->coefs[h], ci, p);
    }
    if (st == OR_OK && nprobes > 0) st = check_probes(p, nvars, SN, SD, nprobes, probes, anchor, bb, ctx);
  }
  if (st != OR_OK) { or_poly_free(SN); or_poly_free(SD); return st; }
  *num = SN;
  *den = SD;
  return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Dense variable-by-variable Newton (the Introduction's multivariate scheme):
 * the full tensor of coefficients from the black box on the grid of nodes
 * X_v[0..D_v].  Brute force for tiny cases; coef [prod (D_v+1)] row-major
 * with the last variable fastest.                                           */
int or_dense_newton(uint64_t p, uint32_t nvars, const uint32_t *deg, const uint64_t *anchor, const uint64_t *nodes,
                    const uint32_t *nnodes, or_blackbox bb, void *ctx, uint64_t *coef) {
  size_t total = 1;
  for (uint32_t v = 0; v < nvars; ++v) total *= (size_t)deg[v] + 1;
  uint64_t **X = (uint64_t **)malloc(sizeof(uint64_t *) * nvars);
  for (uint32_t v = 0; v < nvars; ++v) {
    X[v] = (uint64_t *)malloc(sizeof(uint64_t) * (deg[v] + 1));
    node_list(anchor, nodes, nnodes, v, deg[v] + 1, X[v]);
  }
  /* grid values: for each prefix (x_1..x_{n-1}) one black-box call over x_n */
  const size_t last = (size_t)deg[nvars - 1] + 1;
  const size_t npre = total / last;
  uint64_t *pt = (uint64_t *)malloc(sizeof(uint64_t) * (nvars + 1));
  int st = OR_OK;
  for (size_t a = 0; a < npre && st == OR_OK; ++a) {
    size_t rem = a;
    for (uint32_t v = nvars - 1; v-- > 0;) {
      pt[v] = X[v][rem % (deg[v] + 1)];
      rem /= deg[v] + 1;
    }
    if (bb(ctx, nvars, nvars, 1, 1, pt, anchor, last, X[nvars - 1], coef + a * last) != 0) st = OR_EBLACKBOX;
  }
  /* interpolate along each axis in turn */
  size_t inner = 1;
  for (uint32_t v = nvars; v-- > 0 && st == OR_OK;) {
    const size_t d1 = (size_t)deg[v] + 1;
    const size_t outer = total / (inner * d1);
    uint64_t *f = (uint64_t *)malloc(sizeof(uint64_t) * d1);
    uint64_t *c = (uint64_t *)malloc(sizeof(uint64_t) * d1);
    for (size_t o = 0; o < outer; ++o)
      for (size_t in = 0; in < inner; ++in) {
        for (size_t j = 0; j < d1; ++j) f[j] = coef[(o * d1 + j) * inner + in];
        or_newton(p, d1, X[v], f, c);
        for (size_t j = 0; j < d1; ++j) coef[(o * d1 + j) * inner + in] = c[j];
      }
    free(f); free(c);
    inner *= d1;
  }
  for (uint32_t v = 0; v < nvars; ++v) free(X[v]);
  free(X); free(pt);
  return st;
}

int or_max_threads(void) { return omp_get_max_threads(); }
