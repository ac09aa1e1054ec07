// Device-side evaluation for the synthetic black box (input generation only;
// no code shared with the reconstruction library).
//
// At stage k the requested points are x_v = y_v^i (v < k), x_k = xk[jj],
// anchors beyond.  Grouping hidden terms by their exponents on x_1..x_{k-1}
// (done on the host) gives values
//     out[jj][ii] = sum_l W[l][jj] * Y_l^(i_first + ii)
// with Y_l the group's monomial value and W the group's weights.  A workgroup
// owns 64 consecutive powers; for each tile of 64 groups it first builds the
// table Y_l^i in LDS (power chains in Montgomery form), then every lane sums
// W[l][jj] * Y_l^i for its power in exact 192-bit arithmetic.  Montgomery form
// is removed once per output by a final reduction.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 u128;

namespace {

struct Mont {
  uint64_t p, ninv, r1, r2;  // ninv = -p^{-1} mod 2^64, r1 = 2^64 mod p, r2 = 2^128 mod p
};

__device__ __forceinline__ uint64_t redc(const Mont& M, u128 T) {
  const uint64_t m = (uint64_t)T * M.ninv;
  const u128 s = T + (u128)m * M.p;  // < 2 p 2^64 < 2^128 for p < 2^63
  uint64_t r = (uint64_t)(s >> 64);
  return r >= M.p ? r - M.p : r;
}

__device__ __forceinline__ uint64_t mmul(const Mont& M, uint64_t a, uint64_t b) { return redc(M, (u128)a * b); }

__device__ uint64_t mpow(const Mont& M, uint64_t a, uint64_t e) {
  uint64_t r = M.r1;
  while (e) {
    if (e & 1) r = mmul(M, r, a);
    a = mmul(M, a, a);
    e >>= 1;
  }
  return r;
}

constexpr int TI = 64;    // powers per workgroup
constexpr int TH = 64;    // groups per tile
constexpr int NW = 4;     // waves per workgroup
constexpr int JMAX = 16;  // outputs per wave (nj <= NW * JMAX)

__global__ void __launch_bounds__(256) k_apply(Mont M, uint32_t T, const uint64_t* __restrict__ Y,
                                               const uint64_t* __restrict__ W, uint32_t nj, uint64_t i_first,
                                               uint64_t ni, uint64_t* __restrict__ out) {
  __shared__ uint64_t Z[TH][TI + 1];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t i0 = (uint64_t)blockIdx.x * TI;
  u128 acc[JMAX];
  uint64_t top[JMAX];
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    acc[j] = 0;
    top[j] = 0;
  }
  for (uint32_t h0 = 0; h0 < T; h0 += TH) {
    // table of Y_l^i: wave w fills powers [16w, 16w+16) for the 64 groups of the tile
    {
      const uint32_t h = h0 + lane;
      uint64_t z = 0, y = 0;
      if (h < T) {
        y = mmul(M, Y[h], M.r2);  // to Montgomery form
        z = mpow(M, y, i_first + i0 + 16 * wave);
      }
      for (int s = 0; s < 16; ++s) {
        Z[lane][16 * wave + s] = z;
        z = mmul(M, z, y);
      }
    }
    __syncthreads();
    const uint32_t hn = (T - h0) < (uint32_t)TH ? (T - h0) : (uint32_t)TH;
    for (uint32_t hh = 0; hh < hn; ++hh) {
      const uint64_t zv = Z[hh][lane];
      const uint64_t* w = W + (size_t)(h0 + hh) * nj;
#pragma unroll
      for (int j = 0; j < JMAX; ++j) {
        const uint32_t jj = wave + NW * j;
        if (jj < nj) {
          const u128 pr = (u128)w[jj] * zv;
          const u128 s = acc[j] + pr;
          top[j] += s < pr;
          acc[j] = s;
        }
      }
    }
    __syncthreads();
  }
  const uint64_t ii = i0 + lane;
  if (ii >= ni) return;
#pragma unroll
  for (int j = 0; j < JMAX; ++j) {
    const uint32_t jj = wave + NW * j;
    if (jj < nj) {
      uint64_t x = (uint64_t)((((u128)top[j]) << 64 | (uint64_t)(acc[j] >> 64)) % M.p);
      x = (uint64_t)((((u128)x) << 64 | (uint64_t)acc[j]) % M.p);
      out[(size_t)jj * ni + ii] = redc(M, (u128)x);  // remove the Montgomery factor
    }
  }
}

}  // namespace

extern "C" int zsd_apply(uint64_t p, uint32_t T, const uint64_t* d_Y, const uint64_t* d_W, uint32_t nj,
                         uint64_t i_first, uint64_t ni, uint64_t* d_out, hipStream_t s) {
  if (nj > (uint32_t)(NW * JMAX) || p < 3 || p >= (1ull << 63)) return -1;
  if (ni == 0 || nj == 0) return 0;
  Mont M;
  M.p = p;
  uint64_t inv = 1;  // p^{-1} mod 2^64 by Newton iteration
  for (int k = 0; k < 7; ++k) inv *= 2 - p * inv;
  M.ninv = (uint64_t)0 - inv;
  M.r1 = (uint64_t)((((u128)1) << 64) % p);
  M.r2 = (uint64_t)(((u128)M.r1 * M.r1) % p);
  const uint32_t blocks = (uint32_t)((ni + TI - 1) / TI);
  hipLaunchKernelGGL(k_apply, dim3(blocks), dim3(256), 0, s, M, T, d_Y, d_W, nj, i_first, ni, d_out);
  return hipGetLastError() == hipSuccess ? 0 : -8;
}
