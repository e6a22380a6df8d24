// Gaussian test block Omega (Alg. 5 step 1).
//
// Counter-based generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11),
// key (seed, 0); block b of four 64-bit words uses counter (b + 1, 0, 0, 0).
// Box-Muller on consecutive word pairs (w0, w1):
//   u1 = ((w0 >> 11) + 1) 2^-53 in (0, 1],  u2 = (w1 >> 11) 2^-53 in [0, 1)
//   z0 = sqrt(-2 ln u1) cos(2 pi u2),  z1 = sqrt(-2 ln u1) sin(2 pi u2)
// Element e of the row-major rows x cols block is z of pair e / 2, so one
// thread turns one Philox block into four elements; the generation is
// write-bound.
#include "common.h"

namespace dsv {

namespace {

__device__ __forceinline__ void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1, uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

__device__ __forceinline__ void box_muller(uint64_t w0, uint64_t w1, double &z0, double &z1) {
  const double two_pi = 6.283185307179586476925286766559;
  const double u1 = (double)((w0 >> 11) + 1) * 0x1.0p-53;
  const double u2 = (double)(w1 >> 11) * 0x1.0p-53;
  const double r = sqrt(-2.0 * log(u1));
  double s, c;
  sincos(two_pi * u2, &s, &c);
  z0 = r * c;
  z1 = r * s;
}

// row_to (optional): element (r, c) of the block is stored in row row_to[r]
// of out (the block drawn in one row order, stored in another).
template <typename TO>
__global__ __launch_bounds__(256) void k_gaussian(uint64_t seed, int64_t rows, int64_t cols,
                                                  TO *__restrict__ out, int64_t ld,
                                                  const int32_t *__restrict__ row_to) {
  const int64_t total = rows * cols;
  const int64_t nblk = (total + 3) / 4;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblk;
       b += (int64_t)gridDim.x * blockDim.x) {
    uint64_t w[4];
    philox4x64_10((uint64_t)b + 1, 0, 0, 0, seed, 0, w);
    double z[4];
    box_muller(w[0], w[1], z[0], z[1]);
    box_muller(w[2], w[3], z[2], z[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t e = 4 * b + i;
      if (e < total) {
        const int64_t r = e / cols, c = e - r * cols;
        const int64_t ro = row_to ? (int64_t)row_to[r] : r;
        elem<TO>::st(out + ro * ld + c, (decltype(elem<TO>::ld(out)))z[i]);
      }
    }
  }
}

// Omega of a batch in one launch: matrix i (rows off[i] .. off[i+1] of the
// stacked panel) from the Philox stream keyed (seed0 + i, 0), its blocks of
// 4 elements numbered from 0 within the matrix (boff: their prefix over the
// matrices), so each matrix gets the values a launch of k_gaussian of its
// own gives.
template <typename TO>
__global__ __launch_bounds__(256) void k_gaussian_batched(uint64_t seed0, int count,
                                                          const int64_t *__restrict__ off,
                                                          const int64_t *__restrict__ boff, int64_t cols,
                                                          TO *__restrict__ out, int64_t ld) {
  const int64_t nblk = boff[count];
  for (int64_t gb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gb < nblk;
       gb += (int64_t)gridDim.x * blockDim.x) {
    // the last matrix whose blocks start at or before gb (empty matrices
    // start where the next one does and are passed over)
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (boff[mid] <= gb) lo = mid; else hi = mid - 1;
    }
    const int64_t b = gb - boff[lo];
    const int64_t total = (off[lo + 1] - off[lo]) * cols;
    uint64_t w[4];
    philox4x64_10((uint64_t)b + 1, 0, 0, 0, seed0 + (uint64_t)lo, 0, w);
    double z[4];
    box_muller(w[0], w[1], z[0], z[1]);
    box_muller(w[2], w[3], z[2], z[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t e = 4 * b + i;
      if (e < total) {
        const int64_t r = e / cols, c = e - r * cols;
        elem<TO>::st(out + (off[lo] + r) * ld + c, (decltype(elem<TO>::ld(out)))z[i]);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_philox_raw(uint64_t seed, int64_t nwords,
                                                    uint64_t *__restrict__ out) {
  const int64_t nblk = (nwords + 3) / 4;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblk;
       b += (int64_t)gridDim.x * blockDim.x) {
    uint64_t w[4];
    philox4x64_10((uint64_t)b + 1, 0, 0, 0, seed, 0, w);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (4 * b + i < nwords) out[4 * b + i] = w[i];
  }
}

int grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (int)g;
}

}  // namespace

hipError_t launch_gaussian(uint64_t seed, int64_t rows, int64_t cols, void *out, int64_t ld,
                           int dtype, hipStream_t st, const int32_t *row_to) {
  const int64_t nblk = (rows * cols + 3) / 4;
  if (nblk == 0) return hipSuccess;
  const int g = grid_for(nblk, 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_gaussian<float>, dim3(g), dim3(256), 0, st, seed, rows, cols, (float *)out, ld, row_to);
  else if (dtype == 1)
    hipLaunchKernelGGL(k_gaussian<double>, dim3(g), dim3(256), 0, st, seed, rows, cols, (double *)out, ld, row_to);
  else
    hipLaunchKernelGGL(k_gaussian<bf16>, dim3(g), dim3(256), 0, st, seed, rows, cols, (bf16 *)out, ld, row_to);
  return hipGetLastError();
}

hipError_t launch_gaussian_batched(uint64_t seed0, int count, const int64_t *off, const int64_t *boff,
                                   int64_t nblk, int64_t cols, void *out, int64_t ld, int dtype, hipStream_t st) {
  if (nblk == 0 || count <= 0) return hipSuccess;
  const int g = grid_for(nblk, 256);
  if (dtype == 0)
    hipLaunchKernelGGL(k_gaussian_batched<float>, dim3(g), dim3(256), 0, st, seed0, count, off, boff, cols,
                       (float *)out, ld);
  else if (dtype == 1)
    hipLaunchKernelGGL(k_gaussian_batched<double>, dim3(g), dim3(256), 0, st, seed0, count, off, boff, cols,
                       (double *)out, ld);
  else
    hipLaunchKernelGGL(k_gaussian_batched<bf16>, dim3(g), dim3(256), 0, st, seed0, count, off, boff, cols,
                       (bf16 *)out, ld);
  return hipGetLastError();
}

hipError_t launch_philox_raw(uint64_t seed, int64_t nwords, uint64_t *out, hipStream_t st) {
  const int64_t nblk = (nwords + 3) / 4;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_raw, dim3(grid_for(nblk, 256)), dim3(256), 0, st, seed, nwords, out);
  return hipGetLastError();
}

}  // namespace dsv
