// Evaluation kernels for the error metrics of Sec. 4 that need more than the
// Gram of A^T U: the residual metric eps_res (columns of A^T U - V diag(S))
// and the spectral metric eps_spec, whose ||A - U diag(S) V^T||_2 comes from
// a Lanczos process on E^T E (E = A - U S V^T) run by the driver with these
// vector kernels and the library's SpMM.
//
// Vectors and the factors U, V are FP64 and column-major (one contiguous
// vector per column, leading dimension = vector length).  Every reduction
// sums fixed strips of rows per workgroup and then the strip sums in strip
// order, so results repeat bit for bit.
#include "common.h"

namespace dsv {

namespace {

constexpr int kEvalBlock = 256;

int grid_for(int64_t work, int block, int64_t cap) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kEvalBlock / kWave; ++w) s += red[w];
  return s;  // valid in thread 0
}

// partial[j * nb + b] = sum over strip b of X[j * ldx + r] * y[r]
__global__ __launch_bounds__(kEvalBlock) void k_dots_partial(int64_t n, const double *__restrict__ X, int64_t ldx,
                                                             const double *__restrict__ y,
                                                             double *__restrict__ partial, int nb, int64_t strip) {
  __shared__ double red[kEvalBlock / kWave];
  const int j = blockIdx.y, b = blockIdx.x;
  const int64_t r0 = (int64_t)b * strip;
  const int64_t r1 = r0 + strip < n ? r0 + strip : n;
  const double *x = X + (int64_t)j * ldx;
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kEvalBlock) acc = fma(x[r], y[r], acc);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)j * nb + b] = s;
}

// partial[i * nb + b] = sum over strip b of (Z[i * ld + r] - S[i] * V[i * ld + r])^2
__global__ __launch_bounds__(kEvalBlock) void k_resid_partial(int64_t n, const double *__restrict__ Z,
                                                              const double *__restrict__ V, int64_t ld,
                                                              const double *__restrict__ S,
                                                              double *__restrict__ partial, int nb, int64_t strip) {
  __shared__ double red[kEvalBlock / kWave];
  const int i = blockIdx.y, b = blockIdx.x;
  const int64_t r0 = (int64_t)b * strip;
  const int64_t r1 = r0 + strip < n ? r0 + strip : n;
  const double s_i = S[i];
  const double *z = Z + (int64_t)i * ld, *v = V + (int64_t)i * ld;
  double acc = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kEvalBlock) {
    const double d = z[r] - s_i * v[r];
    acc = fma(d, d, acc);
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partial[(int64_t)i * nb + b] = s;
}

// out[j] = sum_b partial[j * nb + b], in strip order
__global__ __launch_bounds__(kEvalBlock) void k_strip_reduce(int J, int nb, const double *__restrict__ partial,
                                                             double *__restrict__ out) {
  const int j = blockIdx.x * kEvalBlock + threadIdx.x;
  if (j >= J) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(int64_t)j * nb + b];
  out[j] = s;
}

// y[r] -= sum_j X[j * ldx + r] * c_j, c_j = c[j] (times scale[j] when given)
__global__ __launch_bounds__(kEvalBlock) void k_combo(int64_t n, int J, const double *__restrict__ X, int64_t ldx,
                                                      const double *__restrict__ c,
                                                      const double *__restrict__ scale, double *__restrict__ y) {
  const int64_t stride = (int64_t)gridDim.x * kEvalBlock;
  for (int64_t r = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; r < n; r += stride) {
    double s = 0.0;
    for (int j = 0; j < J; ++j) s = fma(X[(int64_t)j * ldx + r], scale ? scale[j] * c[j] : c[j], s);
    y[r] -= s;
  }
}

// out[r] = w[r] / sqrt(*nrm2)
__global__ __launch_bounds__(kEvalBlock) void k_scale_by_norm(int64_t n, const double *__restrict__ w,
                                                              const double *__restrict__ nrm2,
                                                              double *__restrict__ out) {
  const double inv = 1.0 / sqrt(*nrm2);
  const int64_t stride = (int64_t)gridDim.x * kEvalBlock;
  for (int64_t r = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; r < n; r += stride) out[r] = w[r] * inv;
}

// out[j * ldo + row_to(r)] = in[r * ldi + j]: a row-major block (F32 or F64)
// to FP64 column-major, rows optionally renumbered
template <typename T>
__global__ __launch_bounds__(kEvalBlock) void k_to_colmajor(int64_t rows, int cols, const T *__restrict__ in,
                                                            int64_t ldi, double *__restrict__ out, int64_t ldo,
                                                            const int32_t *__restrict__ row_to) {
  const int64_t total = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * kEvalBlock;
  for (int64_t e = (int64_t)blockIdx.x * kEvalBlock + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / cols;
    const int j = (int)(e - r * cols);
    const int64_t ro = row_to ? (int64_t)row_to[r] : r;
    out[(int64_t)j * ldo + ro] = (double)in[r * ldi + j];
  }
}

int strips_for(int64_t n, int64_t *strip) {
  int nb = (int)((n + 4095) / 4096);
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  *strip = (n + nb - 1) / nb;
  return nb;
}

}  // namespace

size_t eval_partial_elems(int J) { return (size_t)J * 256; }

hipError_t launch_dots(int64_t n, int J, const double *X, int64_t ldx, const double *y, double *partial,
                       double *out, hipStream_t st) {
  if (J < 1 || n < 1) return hipErrorInvalidValue;
  int64_t strip = 0;
  const int nb = strips_for(n, &strip);
  hipLaunchKernelGGL(k_dots_partial, dim3((unsigned)nb, (unsigned)J), dim3(kEvalBlock), 0, st, n, X, ldx, y, partial,
                     nb, strip);
  hipLaunchKernelGGL(k_strip_reduce, dim3((unsigned)((J + kEvalBlock - 1) / kEvalBlock)), dim3(kEvalBlock), 0, st, J,
                     nb, (const double *)partial, out);
  return hipGetLastError();
}

hipError_t launch_resid_norms(int64_t n, int k, const double *Z, const double *V, int64_t ld, const double *S,
                              double *partial, double *out, hipStream_t st) {
  if (k < 1 || n < 1) return hipErrorInvalidValue;
  int64_t strip = 0;
  const int nb = strips_for(n, &strip);
  hipLaunchKernelGGL(k_resid_partial, dim3((unsigned)nb, (unsigned)k), dim3(kEvalBlock), 0, st, n, Z, V, ld, S,
                     partial, nb, strip);
  hipLaunchKernelGGL(k_strip_reduce, dim3((unsigned)((k + kEvalBlock - 1) / kEvalBlock)), dim3(kEvalBlock), 0, st, k,
                     nb, (const double *)partial, out);
  return hipGetLastError();
}

hipError_t launch_combo(int64_t n, int J, const double *X, int64_t ldx, const double *c, const double *scale,
                        double *y, hipStream_t st) {
  if (J < 1 || n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_combo, dim3(grid_for(n, kEvalBlock, 8192)), dim3(kEvalBlock), 0, st, n, J, X, ldx, c, scale,
                     y);
  return hipGetLastError();
}

hipError_t launch_scale_by_norm(int64_t n, const double *w, const double *nrm2, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_by_norm, dim3(grid_for(n, kEvalBlock, 8192)), dim3(kEvalBlock), 0, st, n, w, nrm2, out);
  return hipGetLastError();
}

hipError_t launch_to_colmajor(int64_t rows, int cols, const void *in, int64_t ldi, int idtype, double *out,
                              int64_t ldo, const int32_t *row_to, hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  const int g = grid_for(rows * cols, kEvalBlock, 16384);
  if (idtype == 0)
    hipLaunchKernelGGL(k_to_colmajor<float>, dim3(g), dim3(kEvalBlock), 0, st, rows, cols, (const float *)in, ldi,
                       out, ldo, row_to);
  else if (idtype == 1)
    hipLaunchKernelGGL(k_to_colmajor<double>, dim3(g), dim3(kEvalBlock), 0, st, rows, cols, (const double *)in, ldi,
                       out, ldo, row_to);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dsv
