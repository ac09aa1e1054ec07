// Host-side pieces of the reconstruction driver shared by the polynomial,
// balanced and batched paths.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <mutex>
#include <map>
#include <vector>

#include "../../include/zippel.h"
#include "field.hpp"

namespace zr {

struct Error {
  int code;
  explicit Error(int c) : code(c) {}
};

// Throw Error(ZR_ENOMEM / ZR_EDEVICE) for a failed HIP call, recording the
// call's text and location for zr_last_error().
void check_at(hipError_t e, const char* what, const char* file, int line);
#define check(e) ::zr::check_at((e), #e, __FILE__, __LINE__)
void note_error(const char* fmt, ...);
void h2d(void* d, const void* h, size_t bytes, hipStream_t s);
void d2h_sync(void* h, const void* d, size_t bytes, hipStream_t s);

// Device workspace from the library's stream-ordered block cache; released to
// the cache (for later work on the same stream) on destruction.
struct DevArena {
  hipStream_t s;
  int dev = 0;
  std::multimap<size_t, void*>* free_list = nullptr;  // the block cache's free list of (dev, s)
  std::vector<std::pair<void*, size_t>> blocks;
  explicit DevArena(hipStream_t st);
  ~DevArena();
  DevArena(const DevArena&) = delete;
  DevArena& operator=(const DevArena&) = delete;
  void* raw(size_t bytes);
  template <class T>
  T* alloc(size_t n) {
    return (T*)raw(n * sizeof(T));
  }
};

// Validated parameters and the materialised sampling schedule.
struct Params {
  uint64_t p;
  zr_mod M;
  uint32_t nvars, last, nprobes;
  uint32_t first;            // first stage to run (1, or k >= 2 with the stage-(k-1) skeleton in `start`)
  const zr_poly* start = nullptr;
  std::vector<uint32_t> deg, deg_den, need, nnodes;
  std::vector<uint64_t> y, anchor, nodes, probes;
  std::vector<size_t> node_off;
  Params(const zr_params* P, bool balanced);
  // anchor of variable v followed by its first count-1 nodes
  std::vector<uint64_t> node_list(uint32_t v, uint32_t count) const;
};

// Device-resident skeleton: exponents SoA [nvars][t], coefficients, monomial
// values m_l = prod_{v<k} y_v^{e_{l,v}} for the next stage.
struct Skeleton {
  uint32_t nvars = 0, t = 0;
  uint16_t* exps = nullptr;
  uint64_t* coef = nullptr;
  uint64_t* mono = nullptr;
  void alloc(DevArena& A, uint32_t nv, uint32_t n);
};

bool is_prime_u64(uint64_t n);
void make_schedule(uint64_t p, uint32_t nvars, const uint32_t* nnodes, uint64_t seed, uint32_t nprobes,
                   uint64_t* y, uint64_t* anchor, uint64_t* nodes, uint64_t* probes);
std::vector<uint32_t> newton_matrix_limbs(const zr_mod& M, const std::vector<uint64_t>& X);
uint32_t device_cus();
zr_counters& counters();
void count_solve(uint64_t t, uint64_t R);
void count_newton(uint64_t t, uint64_t D1);

void call_bb(zr_blackbox_fn bb, void* ctx, const Params& P, uint32_t k, uint64_t ni, const uint64_t* y,
             const uint64_t* xk, uint64_t nj, uint64_t* d_vals, hipStream_t s);
// Per-variable device constants (Newton matrix limbs, powers of y_v).
struct StageConsts {
  uint32_t* base = nullptr;
  std::vector<size_t> woff, yoff;  // offsets in 32-bit words
  StageConsts(const Params& P, DevArena& A, const std::vector<uint32_t>& D1s, hipStream_t s);
  const uint32_t* W(uint32_t v) const { return base + woff[v]; }
  const uint64_t* ypow(uint32_t v) const { return (const uint64_t*)(base + yoff[v]); }
};

int32_t* host_scratch();
// Pinned host words (at least n), thread-local, reused across calls.
int32_t* host_words(size_t n);
uint32_t lift_stage(const Params& P, uint32_t kvar, const Skeleton& S, const uint64_t* d_vals, uint32_t D1,
                    const uint32_t* d_W, const uint64_t* d_ypow, DevArena& keep, Skeleton& out, hipStream_t s,
                    int32_t* d_status);
void check_probes(const Params& P, zr_blackbox_fn bb, void* ctx, const Skeleton& N, const Skeleton* D,
                  hipStream_t s);
void solve_stage(const Params& P, const Skeleton& S, uint64_t* vals, uint32_t R, hipStream_t s, int32_t* d_status);
void download(const Skeleton& S, hipStream_t s, zr_poly* out);
// Upload the caller's stage-(P.first - 1) skeleton (P.start) and compute its
// monomial values from the power tables of K.
void upload_start(const Params& P, const StageConsts& K, DevArena& keep, Skeleton& S, hipStream_t s);

// balanced path pieces shared with the server
void check_slices(const std::vector<int32_t>& st, const std::vector<int32_t>& dA, const std::vector<int32_t>& dB,
                  uint32_t bn, uint32_t bd, int32_t& rhoN, int32_t& rhoD);
void host_skeleton(const Params& P, const std::vector<uint64_t>& c, DevArena& keep, Skeleton& S, hipStream_t s);
uint32_t stage1_skeleton_host(const Params& P, const std::vector<uint64_t>& c, std::vector<uint16_t>& exps,
                              std::vector<uint64_t>& coef, std::vector<uint64_t>& mono);
void balanced_stage1(const Params& P, zr_blackbox_fn bb, void* ctx, DevArena& keep, Skeleton& SN, Skeleton& SD,
                     hipStream_t s);
void balanced_finish(const Params& P, zr_blackbox_fn bb, void* ctx, Skeleton& SN, Skeleton& SD, hipStream_t s,
                     zr_poly* num, zr_poly* den);

}  // namespace zr
