// Device-side evaluation for the synthetic black box (input generation only;
// no code shared with the reconstruction library).
//
// At stage k the requested points are x_v = y_v^i (v < k), x_k = xk[jj],
// anchors beyond.  Grouping hidden terms by their exponents on x_1..x_{k-1}
// (done on the host) gives values
//     out[jj][ii] = sum_l W[l][jj] * Y_l^(i_first + ii)
// with Y_l the group's monomial value and W the group's weights.
//
// A workgroup owns 64 consecutive powers (lane = power) and one chunk of the
// groups.  For each tile of 64 groups it builds the table Y_l^i in LDS (power
// chains in Montgomery form), then every wave accumulates W[l][jj] * Y_l^i for
// its share of the jj.  Products are summed exactly without carries: the power
// is split into 32-bit halves and W into 22-bit pieces, so each of the six
// partial products is below 2^54 and goes into its own 64-bit column; the
// columns are normalised every 512 groups.  With several group chunks the
// partial sums (reduced mod p) are added by a second kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned __int128 u128;

namespace {

struct Mont {
  uint64_t p, ninv, r1, r2;  // ninv = -p^{-1} mod 2^64, r1 = 2^64 mod p, r2 = 2^128 mod p
  uint64_t r76;              // 2^76 mod p
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
constexpr int JMAX = 12;  // outputs per wave (nj <= NW * JMAX)

struct Cols {
  uint64_t c0, c22, c32, c44, c54, c76;
};

// Move the bits above each low column's range into the column of matching
// weight; the top column is kept below p (its weight 2^76 is applied mod p).
__device__ __forceinline__ void cols_norm(Cols& a, uint64_t p) {
  a.c54 += (a.c0 >> 54) + (a.c22 >> 32) + (a.c32 >> 22) + (a.c44 >> 10);
  a.c0 &= (1ull << 54) - 1;
  a.c22 &= (1ull << 32) - 1;
  a.c32 &= (1ull << 22) - 1;
  a.c44 &= (1ull << 10) - 1;
  a.c76 += a.c54 >> 22;
  a.c54 &= (1ull << 22) - 1;
  a.c76 %= p;
}

// (c0 + c22 2^22 + c32 2^32 + c44 2^44 + c54 2^54 + c76 2^76) mod p
__device__ uint64_t cols_mod(const Mont& M, Cols a) {
  cols_norm(a, M.p);
  const u128 lo = (u128)a.c0 + ((u128)a.c22 << 22) + ((u128)a.c32 << 32) + ((u128)a.c44 << 44) +
                  ((u128)a.c54 << 54);
  const uint64_t r = (uint64_t)(lo % M.p);
  const uint64_t t = (uint64_t)(((u128)a.c76 * M.r76) % M.p);
  const uint64_t v = r + t;
  return v >= M.p ? v - M.p : v;
}

__global__ void __launch_bounds__(256) k_apply(Mont M, uint32_t T, uint32_t hchunk, const uint64_t* __restrict__ Y,
                                               const uint64_t* __restrict__ W, uint32_t nj, uint64_t i_first,
                                               uint64_t ni, uint64_t* __restrict__ out) {
  __shared__ uint64_t Z[TH][TI + 1];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t i0 = (uint64_t)blockIdx.x * TI;
  const uint32_t hbeg = blockIdx.y * hchunk;
  const uint32_t hend = hbeg + hchunk < T ? hbeg + hchunk : T;
  Cols acc[JMAX];
#pragma unroll
  for (int j = 0; j < JMAX; ++j) acc[j] = Cols{0, 0, 0, 0, 0, 0};
  uint32_t since = 0;
  for (uint32_t h0 = hbeg; h0 < hend; h0 += TH) {
    // table of Y_l^i: wave w fills powers [16w, 16w+16) for the 64 groups of the tile
    {
      const uint32_t h = h0 + lane;
      uint64_t z = 0, y = 0;
      if (h < hend) {
        y = mmul(M, Y[h], M.r2);  // to Montgomery form
        z = mpow(M, y, i_first + i0 + 16 * wave);
      }
      for (int s = 0; s < 16; ++s) {
        Z[lane][16 * wave + s] = z;
        z = mmul(M, z, y);
      }
    }
    __syncthreads();
    const uint32_t hn = (hend - h0) < (uint32_t)TH ? (hend - h0) : (uint32_t)TH;
    for (uint32_t hh = 0; hh < hn; ++hh) {
      const uint64_t zv = Z[hh][lane];
      const uint32_t z0 = (uint32_t)zv, z1 = (uint32_t)(zv >> 32);
      const uint64_t* w = W + (size_t)(h0 + hh) * nj;
#pragma unroll
      for (int j = 0; j < JMAX; ++j) {
        const uint32_t jj = wave + NW * j;
        if (jj < nj) {
          const uint64_t wv = w[jj];
          const uint32_t v0 = (uint32_t)(wv & 0x3FFFFF), v1 = (uint32_t)((wv >> 22) & 0x3FFFFF),
                         v2 = (uint32_t)(wv >> 44);
          acc[j].c0 += (uint64_t)z0 * v0;
          acc[j].c22 += (uint64_t)z0 * v1;
          acc[j].c44 += (uint64_t)z0 * v2;
          acc[j].c32 += (uint64_t)z1 * v0;
          acc[j].c54 += (uint64_t)z1 * v1;
          acc[j].c76 += (uint64_t)z1 * v2;
        }
      }
      if (++since == 512) {
#pragma unroll
        for (int j = 0; j < JMAX; ++j) cols_norm(acc[j], M.p);
        since = 0;
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
      const uint64_t x = cols_mod(M, acc[j]);
      // remove the Montgomery factor
      out[((size_t)blockIdx.y * nj + jj) * ni + ii] = redc(M, (u128)x);
    }
  }
}

// out[jj][ii] = sum over chunks c of part[c][jj][ii] mod p
__global__ void k_sum_chunks(uint64_t p, uint32_t nchunk, const uint64_t* __restrict__ part, size_t n,
                             uint64_t* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t s = 0;
  for (uint32_t c = 0; c < nchunk; ++c) {
    s += part[(size_t)c * n + i];
    s = s >= p ? s - p : s;
  }
  out[i] = s;
}

// out[i] = num[i] / den[i] mod p (Fermat inverse); flag set when a den[i] is 0
__global__ void k_divide(Mont M, size_t n, const uint64_t* __restrict__ num, const uint64_t* __restrict__ den,
                         uint64_t* __restrict__ out, int32_t* __restrict__ flag) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t d = den[i];
  if (d == 0) {
    *flag = 1;
    out[i] = 0;
    return;
  }
  // Montgomery: dm = d R, inv = d^(p-2) R, result = num * d^-1
  const uint64_t dm = mmul(M, d, M.r2);
  const uint64_t im = mpow(M, dm, M.p - 2);
  out[i] = mmul(M, num[i], im);  // num * d^-1 R * R^-1
}

}  // namespace

// out[i] = num[i] / den[i] mod p for i < n; *d_flag = 1 if a denominator is 0.
extern "C" int zsd_divide(uint64_t p, size_t n, const uint64_t* d_num, const uint64_t* d_den, uint64_t* d_out,
                          int32_t* d_flag, hipStream_t s) {
  if (p < 3 || p >= (1ull << 63)) return -1;
  if (n == 0) return 0;
  Mont M;
  M.p = p;
  uint64_t inv = 1;
  for (int k = 0; k < 7; ++k) inv *= 2 - p * inv;
  M.ninv = (uint64_t)0 - inv;
  M.r1 = (uint64_t)((((u128)1) << 64) % p);
  M.r2 = (uint64_t)(((u128)M.r1 * M.r1) % p);
  M.r76 = (uint64_t)((((u128)1) << 76) % p);
  hipLaunchKernelGGL(k_divide, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, M, n, d_num, d_den, d_out, d_flag);
  return hipGetLastError() == hipSuccess ? 0 : -8;
}

// Scratch needed by zsd_apply for (T, nj, ni): 64-bit words (0 if none).
extern "C" size_t zsd_apply_scratch_words(uint32_t T, uint32_t nj, uint64_t ni) {
  const uint64_t blocks = (ni + TI - 1) / TI;
  uint64_t chunks = 1;
  // enough workgroups to fill the device: split the groups when the powers alone give too few
  while (blocks * chunks < 2048 && (uint64_t)T / (chunks * 2) >= 256) chunks *= 2;
  return chunks > 1 ? (size_t)chunks * nj * ni : 0;
}

extern "C" int zsd_apply(uint64_t p, uint32_t T, const uint64_t* d_Y, const uint64_t* d_W, uint32_t nj,
                         uint64_t i_first, uint64_t ni, uint64_t* d_out, uint64_t* d_scratch, hipStream_t s) {
  if (nj > (uint32_t)(NW * JMAX) || p < 3 || p >= (1ull << 63)) return -1;
  if (ni == 0 || nj == 0) return 0;
  Mont M;
  M.p = p;
  uint64_t inv = 1;  // p^{-1} mod 2^64 by Newton iteration
  for (int k = 0; k < 7; ++k) inv *= 2 - p * inv;
  M.ninv = (uint64_t)0 - inv;
  M.r1 = (uint64_t)((((u128)1) << 64) % p);
  M.r2 = (uint64_t)(((u128)M.r1 * M.r1) % p);
  M.r76 = (uint64_t)((((u128)1) << 76) % p);
  const uint64_t blocks = (ni + TI - 1) / TI;
  const size_t sw = zsd_apply_scratch_words(T, nj, ni);
  const uint32_t chunks = sw ? (uint32_t)(sw / ((size_t)nj * ni)) : 1;
  if (chunks > 1 && !d_scratch) return -2;
  const uint32_t hchunk = (T + chunks - 1) / chunks;
  uint64_t* dst = chunks > 1 ? d_scratch : d_out;
  hipLaunchKernelGGL(k_apply, dim3((uint32_t)blocks, chunks), dim3(256), 0, s, M, T, hchunk, d_Y, d_W, nj, i_first,
                     ni, dst);
  if (chunks > 1) {
    const size_t n = (size_t)nj * ni;
    hipLaunchKernelGGL(k_sum_chunks, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, p, chunks, d_scratch, n,
                       d_out);
  }
  return hipGetLastError() == hipSuccess ? 0 : -8;
}
