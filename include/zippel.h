/* zippel.h — C ABI of the MI355X (gfx950) sparse Zippel reconstruction library.
 *
 * What is computed (Smirnov, Rozhnov, Voevodin, "GPU Implementation of Zippel
 * Method for Feynman Integral Reconstruction", 2025):
 *   - The unknown is a black-box function over F_p, p a prime below 2^63, that
 *     the caller evaluates at points the library chooses (Introduction: modular
 *     black-box reconstruction; a result is accepted when further probes match).
 *   - Polynomials are reconstructed variable by variable (Introduction, eq. 1):
 *     stage k assumes the skeleton of stage k-1, samples at the Zippel points
 *     (y_1^i, ..., y_{k-1}^i), i = 1..t, solves one transposed Vandermonde
 *     system of size t per stage for D_k right-hand sides in O(t^2) (§1, §2.2),
 *     and lifts every term by univariate Newton interpolation in x_k (eq. 1).
 *   - Rational functions P/Q use the balanced Zippel variant (§1, §2.2 and its
 *     balancing equation): per-slice Thiele reconstruction (eq. 2) in x_k, a
 *     per-slice factor that makes all slices share one normalisation, then the
 *     polynomial step on numerator and denominator separately.
 *
 * Conventions for every entry point:
 *   - Return a zr_status; nothing throws across the ABI.  On error no output
 *     is produced (zr_poly outputs are left empty).
 *   - Device pointers ("d_") are caller-owned HIP device memory; host pointers
 *     ("h_" or plain const arrays in structs) are caller-owned host memory.
 *   - All device work is ordered on the caller's stream.  zippel_* calls return
 *     after their host results are ready; vandermonde_solve_batch is
 *     asynchronous and reports per-system status in device memory.
 *   - Values handed in must lie in [0, p), otherwise ZR_EINVAL (host inputs are
 *     checked; device inputs are the caller's responsibility).
 *   - Calls on different streams may run concurrently; calls are otherwise
 *     not synchronised with each other.
 */
#ifndef ZIPPEL_H
#define ZIPPEL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ZR_OK = 0,
  ZR_EINVAL = -1,     /* bad argument (sizes, p out of range, value >= p) */
  ZR_ENOTPRIME = -2,  /* p fails deterministic Miller-Rabin */
  ZR_ESINGULAR = -3,  /* two monomial values coincide or one is zero: the Zippel system is singular */
  ZR_EDEGEN = -4,     /* degenerate interpolation (vanishing inverse difference, slice degrees differ) */
  ZR_EPROBE = -5,     /* the result does not reproduce the black box at a probe point, or samples ran out */
  ZR_ENORM = -6,      /* rational result: the denominator has no constant term */
  ZR_ENOMEM = -7,     /* device or host allocation failed */
  ZR_EDEVICE = -8,    /* a HIP runtime call failed */
  ZR_EBLACKBOX = -9   /* the black box returned nonzero */
} zr_status;

const char* zr_strerror(int status);
/* Details of the last failure of a library call on this thread (the HIP call
 * and its error, or the failed allocation); "" when none was recorded. */
const char* zr_last_error(void);

/* Result polynomial.  Library-owned host memory; release with zr_poly_free. */
typedef struct {
  uint32_t nvars;
  uint64_t nterms;
  uint16_t* exps;   /* [nterms][nvars] row-major, lexicographically ascending on (e_1..e_n) */
  uint64_t* coeffs; /* [nterms], each in [1, p) */
} zr_poly;
void zr_poly_free(zr_poly* poly);

/* Points the black box must evaluate.  Point (ii, jj), ii in [0, ni), jj in [0, nj):
 *   x_v = y[v]^(i_first + ii)   for v < k-1   (0-based v; the Zippel powers of §1)
 *   x_v = xk[jj]                for v = k-1   (values of the variable being added)
 *   x_v = anchor[v]             for v > k-1   (variables not yet reached)
 * and its value goes to d_vals[jj * ni + ii].  All three arrays are host memory.
 * A single explicit point x is expressed as k = nvars, ni = 1, i_first = 1,
 * y = x[0..n-2], xk = {x[n-1]}.
 * k = nvars + 1 (the further primes of zippel_reconstruct_rational): every
 * variable at its Zippel power, x_v = y[v]^(i_first + ii) for all v, nj = 1,
 * anchor and xk unused.  The values are always wanted modulo p below. */
typedef struct {
  uint32_t nvars;
  uint32_t k;          /* stage, 1-based */
  uint64_t i_first;
  uint64_t ni;
  uint64_t nj;
  const uint64_t* y;
  const uint64_t* anchor;
  const uint64_t* xk;
  uint64_t p;
  uint32_t nexpr;      /* expressions wanted per point: value of expression e at
                          point (ii, jj) goes to d_vals[(e * nj + jj) * ni + ii]
                          (zippel_reconstruct_multi); 1 for every other call */
} zr_points;

/* Black box: fill d_vals[nj*ni] (device memory) with values in [0, p), ordered
 * before later work on `stream` (enqueue on it, or finish before returning).
 * Nonzero return -> ZR_EBLACKBOX. */
typedef int (*zr_blackbox_fn)(void* ctx, const zr_points* pts, uint64_t* d_vals, hipStream_t stream);

/* Reconstruction parameters.
 * Sampling schedule (the random choices of the method): either explicit
 * (y, anchor, nodes non-NULL) or derived from `seed` by zr_schedule().
 *   y[v]      Zippel base of variable v, 2 <= y < p-1
 *   anchor[v] value c_v of x_v while it is not yet reconstructed, 1 <= c < p
 *   nodes     per variable v, nnodes[v] further distinct values of x_v (not equal
 *             to anchor[v]), concatenated in variable order.  Polynomial path:
 *             nnodes[v] >= deg[v].  Balanced path: nnodes[v] >= zr_thiele_nodes(...).
 * Degree bounds: deg[v] bounds deg_{x_v} of the polynomial (of the numerator for
 * the balanced path); deg_den[v] bounds the denominator (balanced only). */
typedef struct {
  uint64_t p;                /* prime, 3 <= p < 2^63 */
  uint32_t nvars;            /* 1..64 */
  const uint32_t* deg;       /* [nvars] */
  const uint32_t* deg_den;   /* [nvars] or NULL */
  uint64_t seed;             /* used when y/anchor/nodes are NULL */
  const uint64_t* y;         /* [nvars] or NULL */
  const uint64_t* anchor;    /* [nvars] or NULL */
  const uint64_t* nodes;     /* concatenated, or NULL */
  const uint32_t* nnodes;    /* [nvars] counts of `nodes`, or NULL with seed-derived nodes */
  uint32_t nprobes;          /* random-point checks of the final result (0 = off) */
  const uint64_t* probes;    /* [nprobes][nvars] or NULL (then derived from seed) */
  uint32_t last_stage;       /* 0 = all; L stops after stage L and returns f(x_1..x_L, anchors) */
  uint32_t first_stage;      /* 0 or 1: start at stage 1.  k >= 2 (polynomial path only): resume at
                                stage k from `start`, the result of stage k-1 of the same schedule */
  const zr_poly* start;      /* first_stage = k >= 2: f(x_1..x_{k-1}, anchors) as zippel_reconstruct
                                returns it with last_stage = k-1 (host; exponents of x_k..x_n zero,
                                e_v <= deg[v], terms distinct and lexicographically ascending,
                                coefficients < p); otherwise ignored.  Copied before the call returns. */
} zr_params;

/* Result with rational coefficients (zippel_reconstruct_rational).
 * Library-owned host memory; release with zr_qpoly_free. */
typedef struct {
  uint32_t nvars;
  uint64_t nterms;
  uint32_t nwords;  /* 64-bit words per magnitude */
  uint32_t nprimes; /* primes used, the confirming one included */
  uint16_t* exps;   /* [nterms][nvars], lexicographically ascending */
  uint64_t* num;    /* [nterms][nwords] |numerator|, least significant word first */
  uint8_t* neg;     /* [nterms] 1 when the numerator is negative */
  uint64_t* den;    /* [nterms][nwords] denominator > 0, coprime to the numerator */
} zr_qpoly;
void zr_qpoly_free(zr_qpoly* q);

/* Number of nodes beyond the anchor that the balanced path needs for a variable
 * with numerator/denominator degree bounds (a, b): a continued fraction with
 * coefficients b_0..b_m has type (ceil(m/2), floor(m/2)), so m = max(2a-1, 2b),
 * plus one confirming sample (eq. 2). */
uint32_t zr_thiele_nodes(uint32_t deg_num, uint32_t deg_den);

/* Seeded sampling schedule (SplitMix64, Steele-Lea-Flood 2014; uniform draws in
 * [lo, hi) by rejection of u >= floor(2^64/n)*n).  Draw order: y_1..y_n in
 * [2, p-1); anchors in [1, p); for each variable its nnodes[v] nodes in [1, p),
 * redrawing repeats of the anchor or of earlier nodes; then nprobes points.
 * Outputs are host arrays sized nvars, sum(nnodes), nprobes*nvars. */
zr_status zr_schedule(uint64_t p, uint32_t nvars, const uint32_t* nnodes, uint64_t seed, uint32_t nprobes,
                      uint64_t* y, uint64_t* anchor, uint64_t* nodes, uint64_t* probes);

/* Deterministic Miller-Rabin (first twelve prime bases; exact for all 64-bit n). */
int zr_is_prime(uint64_t n);

/* Polynomial Zippel reconstruction (§1): returns f with deg_{x_v} f <= deg[v],
 * terms with nonzero coefficients in lexicographic order. */
zr_status zippel_reconstruct(const zr_params* params, zr_blackbox_fn bb, void* ctx, hipStream_t stream,
                             zr_poly* out);

/* Balanced Zippel for a rational function (§1, §2.2): returns num/den in
 * lowest terms with den(0,...,0) = 1 (ZR_ENORM if den has no constant term). */
zr_status zippel_balanced_reconstruct(const zr_params* params, zr_blackbox_fn bb, void* ctx, hipStream_t stream,
                                      zr_poly* num, zr_poly* den);

/* Polynomial Zippel without known degree bounds (Introduction: a result is
 * accepted when further probes reproduce it).  Stage k samples x_k at its
 * anchor and then at the schedule's nodes in batches (the first as wide as
 * the previous stage's degree plus `confirm`, at most 63, then 16 at a time;
 * the batches change how many samples are drawn, not the result); after
 * each node m it forms, for every term, the divided difference of order m of
 * the term's values at x_0..x_m, and stops at the first m whose last
 * `confirm` orders vanish for all terms.  The stage's degree is
 * D = m - confirm; the terms are lifted over x_0..x_D as in
 * zippel_reconstruct.
 *   params     as for zippel_reconstruct, with deg[v] read as a cap: at most
 *              deg[v] + confirm nodes of x_v are sampled, and an explicit
 *              schedule must hold that many; last_stage 0 or nvars,
 *              first_stage 0 or 1, deg[v] + confirm <= 127
 *   confirm    1..8 vanishing orders that end a stage
 *   deg_found  host [nvars] or NULL: the degree found for each variable
 * Errors as zippel_reconstruct; ZR_EPROBE also when a stage reaches its cap
 * without `confirm` vanishing orders. */
zr_status zippel_reconstruct_adaptive(const zr_params* params, uint32_t confirm, zr_blackbox_fn bb, void* ctx,
                                      hipStream_t stream, zr_poly* out, uint32_t* deg_found);

/* Several polynomials reconstructed together (§2.2: one solve serves several
 * expressions of various degrees).  The black box returns all nexpr values
 * at each point (zr_points.nexpr = nexpr).  Stage k solves ONE transposed
 * Vandermonde system on the union of the expressions' stage-(k-1) skeletons
 * with sum_e deg[e][k-1] right-hand sides; each expression is lifted by its
 * own Newton interpolation over the first deg[e][k-1] + 1 nodes of x_k.
 *   params   prime, schedule, probes as for zippel_reconstruct; params->deg is
 *            ignored (the schedule needs, per variable, the largest bound);
 *            last_stage 0 or nvars, first_stage 0 or 1, deg_den NULL
 *   nexpr    1..64 expressions
 *   deg      host [nexpr][nvars] degree bounds of each expression
 *   out      [nexpr] results (zr_poly_free each); probes compare every
 *            expression with the black box
 * Errors as zippel_reconstruct; on error every out[e] is left empty. */
zr_status zippel_reconstruct_multi(const zr_params* params, uint32_t nexpr, const uint32_t* deg, zr_blackbox_fn bb,
                                   void* ctx, hipStream_t stream, zr_poly* out);

/* Polynomial with rational coefficients from its values modulo several
 * primes: the modular reconstruction is finished by the recovery of rational
 * numbers (§1; the multi-prime Zippel routine of §2.2).
 *   params     the first prime and its reconstruction (params->p, schedule,
 *              degree bounds, probes) exactly as for zippel_reconstruct, which
 *              runs first and fixes the term set; last_stage must be 0 or
 *              nvars and first_stage 0 or 1
 *   primes     nprimes further primes, used in order (1 + nprimes <= 8); every
 *              prime, the first included, lies in (2^62, 2^63) and all differ
 *   bb, ctx    the black box; each call names its prime in zr_points.p.  For
 *              further prime j (1-based) it is asked once for the t points
 *              k = nvars + 1 (every x_v = y_v^i, i = 1..t, bases y drawn by
 *              zr_schedule from seed params->seed + j)
 * Each further prime gives every term's coefficient modulo it by one
 * transposed Vandermonde system with a single right-hand side; after each,
 * the fractions reconstructed from the primes so far (Chinese remainder
 * theorem, then Wang's rational reconstruction with |num|, den < 2^e,
 * e = floor((bits(P) - 2) / 2) for the product P of those primes) are tested
 * against the next prime's residues, and the call returns when all agree.
 * Errors: as zippel_reconstruct for the first prime; ZR_EPROBE when the
 * primes run out before such a confirmation; ZR_ESINGULAR when two monomial
 * values coincide modulo a further prime. */
zr_status zippel_reconstruct_rational(const zr_params* params, const uint64_t* primes, uint32_t nprimes,
                                      zr_blackbox_fn bb, void* ctx, hipStream_t stream, zr_qpoly* out);

/* Coefficients of a known term set modulo p (the further-prime step of
 * zippel_reconstruct_rational): solves sum_l a_l m_l^i = v_i, i = 1..t, with
 * m_l = prod_v y[v]^e_{l,v} over all nvars variables, as W(m_l) / (m_l M'(m_l))
 * with W's coefficients w_d = sum_r M_{r+d+1} v_{r+1} (M the master polynomial).
 *   h_exps    host [t][nvars] exponents of distinct monomials
 *   y         host [nvars] bases, each < p
 *   d_vals    device [t]: v_i at [i-1]
 *   d_out     device [t]: a_l at [l]
 *   d_status  device int32: ZR_OK or ZR_ESINGULAR (two m_l equal, or one 0)
 * Asynchronous on `stream` after the exponent upload; argument errors return at once. */
zr_status zr_skeleton_solve(uint64_t p, uint32_t nvars, uint32_t t, const uint16_t* h_exps, const uint64_t* y,
                            const uint64_t* d_vals, uint64_t* d_out, int32_t* d_status, hipStream_t stream);

/* Per-slice Thiele reconstruction (eq. 2), the univariate step of balanced
 * Zippel (§2.2).  For each of T slices: the shortest continued fraction
 * b_0 + (x - x_0)/(b_1 + (x - x_1)/(... + (x - x_{m-1})/b_m)) through the
 * samples at X[0..m] whose value at X[m+1] equals the sample there, written
 * as A(x)/B(x) and scaled so that the lowest nonzero coefficient of B is 1.
 *   d_X       device [nk], distinct nodes in [0, p)
 *   d_F       device [nk][T], each < p: the sample of slice i at X[j] is at [j][i]
 *   d_A, d_B  device [nk+1][T] outputs: coefficient r of slice i at [r][i]
 *             (zero above the degree); not written for a failed slice
 *   d_degA, d_degB, d_status  device [T] int32: the degrees, and ZR_OK,
 *             ZR_EDEGEN (a vanishing inverse difference before confirmation,
 *             or B = 0) or ZR_EPROBE (nothing confirmed within the nk samples);
 *             degrees -1 for a failed slice
 * nk <= 511 runs one wavefront per slice; longer node lists one lane per
 * slice with library-allocated scratch.  Asynchronous on `stream`; argument
 * errors return at once (ZR_EINVAL, ZR_ENOTPRIME). */
zr_status zr_thiele_slices(uint64_t p, uint32_t T, uint32_t nk, const uint64_t* d_X, const uint64_t* d_F,
                           uint64_t* d_A, uint64_t* d_B, int32_t* d_degA, int32_t* d_degB, int32_t* d_status,
                           hipStream_t stream);

/* One transposed Vandermonde system (§1, §2.2) through the one-system solve
 * of the plain reconstruction: master polynomial, synthetic-division dot
 * products (the pass chosen by zr_solve_variant), Horner and scaling.  Solves
 *      sum_l a_l * m_l^i = v_i,   i = 1..t
 * for each of R right-hand sides.
 *   d_mono   device [t], distinct nonzero values < p
 *   d_rhs    device [R][t]: v_i of right-hand side j at [j][i-1]
 *   d_out    device [R][t]: a_l of right-hand side j at [j][l]; may equal d_rhs
 *   d_status device int32: ZR_OK, or ZR_ESINGULAR when two m_l coincide or
 *            one is 0 (d_out then unspecified)
 * Asynchronous on `stream`; argument errors return at once. */
zr_status zr_vandermonde_solve(uint64_t p, uint32_t t, uint32_t R, const uint64_t* d_mono, const uint64_t* d_rhs,
                               uint64_t* d_out, int32_t* d_status, hipStream_t stream);

/* zr_vandermonde_solve for callers that cannot allocate device memory (code
 * under stream capture, serving loops that forbid hipMalloc): same arguments,
 * same results, same kernels, but the master polynomial and the solve's
 * workspace live in one fixed 64 MiB device array inside the library (one per
 * GPU, held until the process ends) instead of memory from the allocator.  The
 * call allocates nothing and launches no memset: its status word is cleared by
 * a kernel, and every workspace word is written before it is read, so nothing
 * left by an earlier call is used.
 *   Size limit: a system whose workspace does not fit the array (at R = 40,
 *   t above about 45 000; before that the chunks share fewer partial-sum
 *   slots, then the dot-product pass runs in fewer chunks) returns ZR_EINVAL
 *   before any device work, with the reason in zr_last_error().
 *   Every call on one GPU uses that GPU's one array: calls that overlap on the
 *   same GPU (other streams, other threads) race and must be serialised by the
 *   caller.  The first call on a device looks the array's address up once. */
zr_status zr_vandermonde_solve_noalloc(uint64_t p, uint32_t t, uint32_t R, const uint64_t* d_mono,
                                       const uint64_t* d_rhs, uint64_t* d_out, int32_t* d_status,
                                       hipStream_t stream);

/* Batched transposed Vandermonde solve (the O(t^2) step of §1 and §2.2, many
 * systems and right-hand sides at once).  System s has t_s unknowns and R_s
 * right-hand sides; for each right-hand side j it solves
 *      sum_l a_l * m_l^i = v_i,   i = 1..t_s
 * (Zippel powers start at 1).
 *   d_sys_off [nsys+1] device, prefix sums of t_s; m for system s at d_mono[d_sys_off[s] ..]
 *   d_mono    device, monomial values, distinct and nonzero within a system
 *   h_nrhs    [nsys] host, R_s
 *   h_sys_off [nsys+1] host copy of d_sys_off (sizes drive the launch)
 *   d_rhs_off [nsys+1] device, prefix sums of R_s * t_s; h_rhs_off the host copy
 *   d_rhs     device, system s at d_rhs + rhs_off[s], laid out [R_s][t_s]: v_i at [j][i-1]
 *   d_out     device, same layout as d_rhs: a_l at [j][l]  (may not alias d_rhs)
 *   d_status  [nsys] device int32: ZR_OK or ZR_ESINGULAR (outputs of that system unspecified)
 * Asynchronous on `stream`; host-side argument errors return immediately. */
zr_status vandermonde_solve_batch(size_t nsys, uint64_t p, const uint64_t* d_sys_off, const uint64_t* h_sys_off,
                                  const uint64_t* d_mono, const uint32_t* h_nrhs, const uint64_t* d_rhs_off,
                                  const uint64_t* h_rhs_off, const uint64_t* d_rhs, uint64_t* d_out,
                                  int32_t* d_status, hipStream_t stream);

/* Batched polynomial Zippel (§1): n independent reconstructions advanced stage
 * by stage together, so that each stage's master polynomials, transposed
 * Vandermonde solves (one persistent work-queue pass over all systems),
 * Newton lifts and expansions run as one launch sequence for the whole batch.
 *   params[n]  one parameter set per instance; every valid instance must use
 *              the same prime (ZR_EINVAL for the whole call otherwise)
 *   bb, ctx[n] the black box, called with ctx[i] for instance i (ctx may be
 *              NULL: then every call gets NULL)
 *   out[n]     results (library-owned, zr_poly_free each); empty for failed instances
 *   status[n]  per-instance ZR_OK or that instance's error; one instance's
 *              failure does not stop the others
 * Returns ZR_OK when the batch ran, whatever the per-instance statuses. */
zr_status zippel_reconstruct_batch(uint32_t n, const zr_params* params, zr_blackbox_fn bb, void* const* ctx,
                                   hipStream_t stream, zr_poly* out, int32_t* status);

/* Dot-product pass of the one-system solve (§2.2, the O(t^2 R) sums), both on
 * the integer vector ALU: 0 one wave per tile of right-hand sides, each
 * running the synthetic division chain with carry-free 64-bit
 * multiply-accumulates; 1 (default) a producer wave runs the chain once per
 * row block and publishes it through LDS to one consumer wave per tile
 * (systems with at most 10 right-hand sides run as 0).  Same results for
 * both.  Any other value returns ZR_EINVAL and leaves the choice unchanged. */
zr_status zr_solve_variant(int variant);

/* Graph mode of the batched paths (zippel_reconstruct_batch, the server,
 * vandermonde_solve_batch): with on != 0 each stage's device-side solve
 * sequence (master polynomials, packing, chunk chains, the persistent dot-product
 * pass, scaling) is captured into one hipGraph and launched as a unit.  Off by
 * default; results are identical either way. */
void zr_batch_graphs(int on);

/* Size bands of the batched solve, by system size t: [1,64), [64,256),
 * [256,1024), [1024,4096), [4096,inf).  Per band: whether small systems share
 * wavefronts (lane = (system, row)), and the shortest chunk of the synthetic
 * division range when a system is split across wavefronts. */
typedef struct {
  uint32_t packed;
  uint32_t min_chunk;
} zr_band_choice;
#define ZR_NBANDS 5

/* Measure the candidates of every band on the current device (synthetic
 * systems mod p, about a second) and keep the fastest for later batched calls
 * of this process.  table[ZR_NBANDS] receives the choices (may be NULL). */
zr_status zr_autotune(uint64_t p, hipStream_t stream, zr_band_choice* table);
/* Current choices (defaults until zr_autotune ran); returns 1 if tuned. */
int zr_tuning_get(zr_band_choice* table);
/* Override the choices (tests and experiments). */
zr_status zr_tuning_set(const zr_band_choice* table);

/* Served form.  Reconstruction requests arrive over time (the coefficients of a
 * modular reduction stream out one by one, Introduction); the server admits
 * them first come, first served while a slot is free and the sum of the
 * active requests' estimated device footprints stays within hbm_budget bytes
 * (a request above the budget still runs when nothing else is active).  A
 * request's estimate covers its next stage and is recomputed after every step
 * from the sizes of the skeletons it has reached, so requests are admitted by
 * what they hold now, not by a guess of their final size.  Each
 * zr_server_step advances every active request by one stage, batching the
 * stage's Vandermonde solves, Newton matrices and lifts of all of them into one
 * launch sequence, so requests admitted at a step boundary share the device
 * with those already running (continuous batching).  Skeletons stay on the
 * device between steps.  A result is bit-identical to the same request run
 * alone through zippel_reconstruct / zippel_balanced_reconstruct.
 * One server is driven from one host thread; all its device work is on `stream`. */
typedef struct zr_server zr_server;

typedef struct {
  uint64_t submitted, admitted, completed, failed, steps;
  uint64_t footprint, peak_footprint;  /* bytes of the active requests' next stages (estimates) */
  uint64_t active, pending, peak_active;
} zr_server_stats;

zr_status zr_server_create(zr_server** srv, uint64_t p, uint64_t hbm_budget, uint32_t max_active,
                           hipStream_t stream);
void zr_server_destroy(zr_server* srv);
/* Queue a request: polynomial (balanced = 0) or rational (balanced = 1) with
 * the parameters of zippel_reconstruct / zippel_balanced_reconstruct (copied;
 * params may be released on return).  expected_terms caps the skeleton size
 * that a footprint estimate assumes for the stage ahead (0: the degree bounds'
 * monomial count).  The black box is called with ctx from zr_server_step.
 * *id receives the request's handle.  Resumption (first_stage >= 2) is not
 * served: ZR_EINVAL. */
zr_status zr_server_submit(zr_server* srv, const zr_params* params, int balanced, uint64_t expected_terms,
                           zr_blackbox_fn bb, void* ctx, uint64_t* id);
/* Admit what fits, advance every active request by one stage, retire the
 * finished ones.  Outputs (may be NULL): requests active after the step,
 * still pending, and finished in this step. */
zr_status zr_server_step(zr_server* srv, uint32_t* n_active, uint32_t* n_pending, uint32_t* n_finished);
/* Result of a request: returns 1 while it is pending or active, 0 once finished
 * (then *status, *num and *den (den empty for polynomials) are filled, the
 * caller owns the polynomials and the id is forgotten), ZR_EINVAL for an
 * unknown id.  num or den NULL discards that output. */
int zr_server_poll(zr_server* srv, uint64_t id, int32_t* status, zr_poly* num, zr_poly* den);
/* Ids of the requests that finished since the previous call, in the order they
 * finished, leaving out those already collected with zr_server_poll: up to cap
 * of them are written to ids and their count returned (the rest are kept for
 * the next call; 0 for a NULL server, or NULL ids with cap above 0).  A serving
 * loop then collects exactly those results with zr_server_poll instead of
 * polling every request still in flight. */
uint32_t zr_server_finished(zr_server* srv, uint64_t* ids, uint32_t cap);
zr_status zr_server_get_stats(zr_server* srv, zr_server_stats* stats);

/* ---- helpers for callers and black boxes ---------------------------------- */

/* Synchronous copies between host and device memory on `stream`. */
zr_status zr_copy_h2d(void* d_dst, const void* h_src, size_t bytes, hipStream_t stream);
zr_status zr_copy_d2h(void* h_dst, const void* d_src, size_t bytes, hipStream_t stream);
zr_status zr_copy_d2d(void* d_dst, const void* d_src, size_t bytes, hipStream_t stream);

/* Record/replay black box: wraps another black box, records every call's device
 * output; later replays them in the same order (descriptor sizes must match,
 * else the replay call returns nonzero).  For benchmarks that exclude the
 * black box's own cost. */
typedef struct zr_recorder zr_recorder;
zr_status zr_recorder_create(zr_recorder** rec, zr_blackbox_fn inner, void* inner_ctx);
void zr_recorder_destroy(zr_recorder* rec);
void zr_recorder_rewind(zr_recorder* rec);          /* next call replays record 0 */
void zr_recorder_set_replay(zr_recorder* rec, int replay);
int zr_recorder_blackbox(void* rec, const zr_points* pts, uint64_t* d_vals, hipStream_t stream);

/* Kernel timing: when enabled, the library brackets each launch of its named
 * kernels with HIP events on the launch stream and accumulates durations.
 * on = 1 times every named launch; on = 2 only the solve's dot-product pass
 * ("vs_dots"), which keeps the event overhead out of the other launches;
 * 0 turns timing off. */
void zr_timing_enable(int on);
void zr_timing_reset(void);
/* Returns the number of timed launches of `kernel` and their total in ms. */
uint64_t zr_timing_get(const char* kernel, double* total_ms);

/* Algorithmic work counters of the last zippel_* call on this thread. */
typedef struct {
  uint64_t mulmods;       /* algorithmic modular products (each multiply-accumulate counts 1) */
  uint64_t solve_mulmods; /* of which in the Vandermonde solves: R t^2 + 2 t(t-1) per system */
  uint64_t vsolve_terms;  /* sum of t*R over all solved systems */
  uint32_t stages;
  uint64_t max_t;
  uint64_t dot_products;  /* of which the dot products of the solves: R t^2 per system */
  uint64_t chain_steps;   /* steps of the synthetic-division chains q_{l,r}: t(t-1) per system */
} zr_counters;
void zr_last_counters(zr_counters* out);

#ifdef __cplusplus
}
#endif
#endif /* ZIPPEL_H */
