// Internal launchers of the gfx950 kernels.  All take device pointers and a
// stream, enqueue asynchronously and return the hipError_t of the launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.hpp"

namespace zr {

// ---- transposed Vandermonde solve (§1, §2.2) --------------------------------
// One system: t unknowns, R right-hand sides.  The row range of the
// synthetic-division recurrence q_{r-1} = M_r + m_l q_r is cut into S chunks
// of length L (chunk c covers r in [max(t-(c+1)L,0), t-cL)); a chunk's start
// value is an affine function of the previous chunk's, so chunks run in
// parallel after a first chain-only pass and a per-row scan.
struct VsolvePlan {
  uint32_t t, R;
  uint32_t L, S;       // chunk length and count
  uint32_t RT, ntile;  // right-hand sides per tile (even), number of tiles
  uint32_t ldv;        // row stride (32-bit words) of one packed row of a tile
  uint32_t pc;         // 1: producer/consumer pass (chain once per row block, one wave per tile)
  uint32_t Sd;         // partial-sum slots per row and right-hand side (the chunks take them in turn)
  uint32_t ng, Rg;     // right-hand-side groups (one dot-product pass each) and the largest group's size
  uint32_t dchain;     // 1: delta_l from the chain pass (sum r M_r m^r), no Horner sum in the producer
  uint32_t tw[8];      // producer/consumer pass: right-hand sides of each consumer's tile
  size_t vt32;         // 32-bit words of the packed right-hand sides
};
VsolvePlan vsolve_plan(uint32_t t, uint32_t R, uint32_t num_cus);
// true when the producer/consumer pass is selected (solve variant 1, the default)
bool vsolve_uses_pc();

// Workspace (device, uint64 elements) needed by vsolve for a plan.
size_t vsolve_workspace_words(const VsolvePlan& P);

// Solve using the master polynomial lower coefficients Mc[0..t) (monic, degree t).
//   mono [t], rhs [R][ld_rhs] with v^(j)_{r+1} at rhs[j*ld_rhs + r],
//   out  [R][ld_out] receives a^(j)_l at out[j*ld_out + l]; out may equal rhs.
//   status: set to ZR_ESINGULAR (-3) when a row is singular (m_l delta_l = 0).
hipError_t vsolve(const zr_mod& M, const VsolvePlan& P, const uint64_t* mono, const uint64_t* Mc,
                  const uint64_t* rhs, size_t ld_rhs, uint64_t* out, size_t ld_out, uint64_t* work,
                  int32_t* status, hipStream_t s);

// Master polynomial M(z) = prod_l (z - m_l): lower coefficients into Mc[t];
// tmp is a scratch array of master_tmp_words(t).  Product tree, ceil(log2 t) levels.
size_t master_tmp_words(uint32_t t);
hipError_t master_poly(const zr_mod& M, uint32_t t, const uint64_t* mono, uint64_t* Mc, uint64_t* tmp,
                       hipStream_t s);

// ---- Newton lift (eq. 1) and skeleton expansion ------------------------------
// g[d][l] = sum_i W[d][i] vals[i][l] with W the inverse Vandermonde matrix of
// the stage's nodes; Wl holds W as 22-bit limbs laid out [i][d][3].  cnt[l]
// receives the number of nonzero g[.][l].
hipError_t newton_lift(const zr_mod& M, uint32_t t, uint32_t D1, const uint64_t* vals, const uint32_t* Wl,
                       uint64_t* g, uint32_t* cnt, hipStream_t s);

// Exclusive scan of cnt[n] into off[n+1] (off[n] = total); tmp needs scan_tmp_words(n).
size_t scan_tmp_words(uint32_t n);
hipError_t exclusive_scan(uint32_t n, const uint32_t* cnt, uint32_t* off, uint32_t* tmp, hipStream_t s);

// New skeleton terms (e_l, d) for g[d][l] != 0, lexicographic order.
//   exps_old/new: SoA [nvars][ld] uint16 with ld_old = t, ld_new = cap_new.
//   ypow: y_k^d (d < D1) and Shoup constants ypowp.
hipError_t expand(const zr_mod& M, uint32_t t, uint32_t D1, uint32_t kvar, uint32_t nvars,
                  const uint16_t* exps_old, const uint64_t* mono_old, const uint64_t* g, const uint32_t* off,
                  const uint64_t* ypow, const uint64_t* ypowp, uint16_t* exps_new, uint64_t* coef_new,
                  uint64_t* mono_new, uint32_t ld_new, hipStream_t s);

// Value of the sparse polynomial at one point: sum_l coef_l prod_v tab[v][e_{l,v}].
//   tab: [nvars][ldtab] powers of the point's coordinates; partial: scratch of
//   kPolyEvalBlocks words.
constexpr uint32_t kPolyEvalBlocks = 64;
hipError_t poly_eval_point(const zr_mod& M, uint32_t t, uint32_t nvars, const uint16_t* exps, uint32_t ld,
                           const uint64_t* coef, const uint64_t* tab, uint32_t ldtab, uint64_t* result,
                           uint64_t* partial, hipStream_t s);

// Monomial values m_l = prod_{v < nv} y_v^{e_{l,v}} of a skeleton: exps SoA
// [..][ld] uint16; the powers y_v^d of variable v at tabs[off[v] + d].
struct MonoTables {
  uint32_t off[64];
};
hipError_t mono_values(const zr_mod& M, uint32_t t, uint32_t nv, const uint16_t* exps, uint32_t ld,
                       const uint64_t* tabs, const MonoTables& T, uint64_t* mono, hipStream_t s);

// ---- small helpers -----------------------------------------------------------
hipError_t fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);
hipError_t fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s);
hipError_t copy_u64(uint64_t* dst, const uint64_t* src, size_t n, hipStream_t s);

// ---- balanced path ------------------------------------------------------------
// Per-slice Thiele reconstruction (eq. 2).  F [nk][T] samples at nodes X[0..nk),
// outputs per slice i: A[(nk+1)][T], B[(nk+1)][T] column i, degA/degB[T], status[T].
// scratch: thiele_scratch_words(T, nk) words (none for nk <= 511).
size_t thiele_scratch_words(uint32_t T, uint32_t nk);
hipError_t thiele_slices(const zr_mod& M, uint32_t T, uint32_t nk, const uint64_t* X, const uint64_t* F,
                         uint64_t* A, uint64_t* B, int32_t* degA, int32_t* degB, int32_t* st, uint64_t* scratch,
                         hipStream_t s);

// Thiele for the slices of several reconstructions in one launch:
// thiele_slices_per_block(max nk) slices per block, d_prefix[n+1] the prefix
// sums of cdiv(T_j, that count); job scratch as for thiele_slices.
struct ThieleJob {
  uint32_t T, nk;
  const uint64_t* X;
  const uint64_t* F;
  uint64_t* A;
  uint64_t* B;
  int32_t* degA;
  int32_t* degB;
  int32_t* st;
  uint64_t* scratch;
};
uint32_t thiele_slices_per_block(uint32_t max_nk);
hipError_t thiele_slices_batch(const zr_mod& M, uint32_t n, const uint32_t* d_prefix, uint32_t total_blocks,
                               uint32_t max_nk, const ThieleJob* d_jobs, hipStream_t s);

// Transposed Vandermonde apply: out[i] = sum_l a_l m_l^(i+1), i = 0..T-1.
hipError_t vapply(const zr_mod& M, uint32_t t, const uint64_t* mono, const uint64_t* a, uint32_t T, uint64_t* out,
                  uint64_t* work, size_t work_words, hipStream_t s);
size_t vapply_work_words(uint32_t t, uint32_t T);

// Many applies in two launches: d_prefix[n+1] prefix sums of
// vapply_batch_blocks(t_q, T_q), d_sum_prefix[n+1] of cdiv(T_q, 256); each
// job's work holds vapply_work_words(t, T) words.
struct VapplyJob {
  uint32_t t, T;
  const uint64_t* mono;
  const uint64_t* a;
  uint64_t* out;
  uint64_t* work;
};
uint32_t vapply_batch_blocks(uint32_t t, uint32_t T);
hipError_t vapply_batch(const zr_mod& M, uint32_t n, const uint32_t* d_prefix, uint32_t total,
                        const uint32_t* d_sum_prefix, uint32_t sum_total, const VapplyJob* d_jobs, hipStream_t s);

// The balancing of many reconstructions in two launches (as balance_rhs per
// job, with beta[T] per job; a slice without a factor sets *status = ZR_EDEGEN):
// d_beta_prefix of balance_beta_blocks(T), d_rhs_prefix of balance_rhs_blocks(...).
struct BalanceJob {
  uint32_t T, tN, tD;
  int32_t rhoN, rhoD;
  const uint64_t* X;
  const uint64_t* A;
  const uint64_t* B;
  const int32_t* degA;
  const int32_t* degB;
  const uint64_t* nprev;
  const uint64_t* dprev;
  uint64_t* beta;
  uint64_t* vN;
  size_t ldN;
  uint64_t* vD;
  size_t ldD;
  int32_t* status;
};
uint32_t balance_beta_blocks(uint32_t T);
uint32_t balance_rhs_blocks(uint32_t tN, uint32_t tD, int32_t rhoN, int32_t rhoD);
hipError_t balance_batch(const zr_mod& M, uint32_t n, const uint32_t* d_beta_prefix, uint32_t beta_total,
                         const uint32_t* d_rhs_prefix, uint32_t rhs_total, const BalanceJob* d_jobs, hipStream_t s);

// Balanced right-hand sides: beta_i from N_{k-1}(y^i)/A_i(x_0) (fallback
// D_{k-1}(y^i)/B_i(x_0)) into beta[T], then vN[j][i] = beta_i A_i(x_{j+1})
// (j < rhoN, i < tN) and vD[j][i] = beta_i B_i(x_{j+1}) (j < rhoD, i < tD).
// st[i] = -4 if no beta exists.  tN, tD <= T.
hipError_t balance_rhs(const zr_mod& M, uint32_t T, uint32_t nk, const uint64_t* X, const uint64_t* A,
                       const uint64_t* B, const int32_t* degA, const int32_t* degB, const uint64_t* nprev,
                       const uint64_t* dprev, uint32_t tN, int32_t rhoN, uint64_t* vN, size_t ldN, uint32_t tD,
                       int32_t rhoD, uint64_t* vD, size_t ldD, int32_t* st, uint64_t* beta, hipStream_t s);

// *out = code when any of st[0..T) is nonzero (out left alone otherwise).
hipError_t fold_status(const int32_t* st, uint32_t T, int32_t* out, int32_t code, hipStream_t s);

// Scale every coefficient by c (in place).
hipError_t scale_u64(const zr_mod& M, uint64_t* v, size_t n, uint64_t c, hipStream_t s);

// ---- batched solve -------------------------------------------------------------
struct BatchItem {  // one (system, row tile, chunk, rhs tile) work item
  uint32_t sys;
  uint32_t row0;
  uint32_t chunk;
  uint32_t tile;
};

// ---- kernel timing ---------------------------------------------------------------
struct TimedLaunch {
  const char* name;
  hipStream_t s;
  hipEvent_t e0, e1;
  bool on;
  TimedLaunch(const char* n, hipStream_t st);
  ~TimedLaunch();
};

}  // namespace zr
