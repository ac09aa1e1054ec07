// Batched launches: many independent transposed Vandermonde systems, Newton
// lifts and probe evaluations in one sequence of kernel launches.  Every
// batched kernel maps its block index to (system, local block) through a
// prefix array of per-system block counts; the solve's dominant pass runs as a
// persistent kernel over a work queue of (system, row block, chunk, tile)
// items, largest first.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#include "driver.hpp"
#include "field.hpp"
#include "kernels.hpp"

namespace zr {

// Per-band choices of the batched solve.  Bands by system size t:
// [1,64), [64,256), [256,1024), [1024,4096), [4096,inf).
constexpr int kBands = 5;
uint32_t band_of(uint32_t t);

struct BandTuning {
  uint32_t packed;     // 1: systems of this band share wavefronts (lane = (system, row))
  uint32_t min_chunk;  // shortest chunk of the synthetic-division range when a system is split
};
struct Tuning {
  BandTuning band[kBands];
  uint32_t tuned;  // 1 once measured on this device
};

// Current per-band table (defaults until autotune() has run on this device).
Tuning& tuning();
// Measure the candidates of every band on the current device and keep the
// fastest; cost: a few hundred milliseconds, once per process.
void autotune(const zr_mod& M, hipStream_t s);

// Graph mode of batched_solve: its device-side launch sequence is captured
// into one hipGraph and launched as a unit.  Graphs launched on a stream are
// destroyed at that stream's next synchronisation by batched_lift
// (release_graphs).
bool graphs_enabled();
hipStream_t capture_stream();
void set_graphs(bool on);
void retire_graph(hipStream_t s, hipGraph_t g, hipGraphExec_t ge);
void release_graphs(hipStream_t s);

// One system: t unknowns, R right-hand sides in rhs[R][t] (unknowns written
// back in place), monomial values mono[t].  status: 0 or ZR_ESINGULAR.
struct SolveJob {
  uint32_t t, R;
  const uint64_t* mono;
  uint64_t* rhs;
  int32_t* status;
};

// Master polynomials and solves of all jobs (enqueued on s, no host sync),
// all systems through the persistent work-queue pass.
void batched_solve(const zr_mod& M, const std::vector<SolveJob>& jobs, hipStream_t s);

// Newton matrices and powers of y_k for many (nodes, y_k) sets at once:
// for job j, Wl (D1*D1*3 + 24 words, limbs [i][d][3] of the inverse
// Vandermonde matrix of the D1 nodes) and ypow (2*D1 words: y_k^d and their
// Shoup constants).
struct ConstsJob {
  uint32_t D1;
  const uint64_t* h_nodes;  // host, D1 nodes
  uint64_t yk;
  uint32_t* Wl;             // device outputs
  uint64_t* ypow;
};
size_t newton_W_words(uint32_t D1);
void batched_consts(const zr_mod& M, const std::vector<ConstsJob>& jobs, hipStream_t s);

// Newton lift + expansion of many skeletons: vals[D1][t] (row 0 = values at
// the anchor node) -> new skeletons allocated from `keep`.  One host
// synchronisation; returns the statuses read back at that point (d_status
// entries of the jobs, may be null).
struct LiftJob {
  uint32_t kvar, D1;
  const Skeleton* old;
  const uint64_t* vals;
  const uint32_t* Wl;
  const uint64_t* ypow;
  const int32_t* d_status;
  Skeleton* out;  // filled
};
std::vector<int32_t> batched_lift(const zr_mod& M, const std::vector<LiftJob>& jobs, DevArena& keep, hipStream_t s);

// Values of sparse polynomials at points: result[j] = sum_l coef_l prod_v
// tab[v][e_{l,v}], tab [nvars][ldtab] (device).
struct EvalJob {
  const Skeleton* poly;
  const uint64_t* tab;
  uint32_t ldtab;
  uint64_t* result;
};
void batched_eval(const zr_mod& M, const std::vector<EvalJob>& jobs, hipStream_t s);

// The constant 1 as a stage-0 skeleton for each entry of out (one upload).
void constant_skeletons(DevArena& A, const std::vector<uint32_t>& nvars, const std::vector<Skeleton*>& out,
                        uint64_t p, hipStream_t s);

// Many device-to-device copies (even byte counts) in one launch.
struct CopyJob {
  const void* src;
  void* dst;
  size_t bytes;
};
void batched_copy(const std::vector<CopyJob>& jobs, hipStream_t s);

// Exponent arrays from the skeletons' SoA layout [nvars][t] to the results'
// term-major layout [t][nvars], many in one launch.
struct TransposeJob {
  const uint16_t* src;
  uint16_t* dst;
  uint32_t t, nvars;
};
void batched_exps_to_terms(const std::vector<TransposeJob>& jobs, hipStream_t s);

// Power tables of points: tab[v][d] = pt[v]^d for v < nv, d < ld (device).
struct PowJob {
  const uint64_t* pt;
  uint64_t* tab;
  uint32_t nv, ld;
};
void batched_power_tables(const zr_mod& M, const std::vector<PowJob>& jobs, hipStream_t s);

// Host-to-device upload of many small host arrays in one copy (pinned staging).
class Blob {
 public:
  template <class T>
  size_t add(const T* p, size_t n) {
    const size_t off = (bytes_.size() + 255) & ~(size_t)255;
    bytes_.resize(off + n * sizeof(T));
    if (n) memcpy(bytes_.data() + off, p, n * sizeof(T));
    return off;
  }
  template <class T>
  size_t add(const std::vector<T>& v) {
    return add(v.data(), v.size());
  }
  // upload; returns the device base (valid while A lives)
  char* upload(DevArena& A, hipStream_t s);

 private:
  std::vector<char> bytes_;
};

}  // namespace zr
