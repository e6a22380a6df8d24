// Sparse-structure kernels: CSR validation, the explicit CSR of A^T used by
// the transposed products of Alg. 5 (steps 2 and 4), and the row-split plan
// of the SpMM.  All integer work; results are independent of scheduling.
//
// CSR(A^T) build (a stable sort by column):
//   1. validation: one thread per nonzero finds its row by binary search in
//      the row pointer, checks the column (range, strictly increasing in the
//      row) and the value (finite), and records its row;
//   2. a stable LSD radix sort of the column indices (only the bits that
//      column numbers below n use) carrying the nonzero index: every column
//      of A then lists its nonzeros in their CSR order, i.e. by increasing
//      row, with no per-column sort and no atomics on the columns (a Zipf
//      matrix sends a tenth of its nonzeros to its first column);
//   3. one thread per entry gathers its row and value, one thread per
//      column finds where the column starts in the sorted keys.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "common.h"

namespace dsv {

namespace {

int grid_for(int64_t work, int block, int64_t cap = 65536) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// ------------------------------------------------------------------ scan
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the exclusive
// prefix and the block total.
__device__ int64_t block_excl_scan(int64_t v, int64_t *sh, int64_t &total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t inc = wave_incl_scan(v);
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    int64_t s = lane < nw ? sh[lane] : 0;
    int64_t si = wave_incl_scan(s);
    if (lane < nw) sh[lane] = si - s;
    if (lane == nw - 1) sh[32] = si;
  }
  __syncthreads();
  int64_t r = inc - v + sh[wave];
  total = sh[32];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const int64_t *__restrict__ in, int64_t n,
                                                          int64_t *__restrict__ sums) {
  __shared__ int64_t sh[40];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    if (idx < n) s += in[idx];
  }
  int64_t tot;
  block_excl_scan(s, sh, tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_sums(int64_t *__restrict__ sums, int64_t nb) {
  __shared__ int64_t sh[40];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += blockDim.x) {
    int64_t idx = base + threadIdx.x;
    int64_t v = idx < nb ? sums[idx] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan(v, sh, tot);
    if (idx < nb) sums[idx] = ex + carry;
    carry += tot;
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const int64_t *__restrict__ in, int64_t n,
                                                         const int64_t *__restrict__ sums,
                                                         int64_t *__restrict__ out, int64_t nb) {
  __shared__ int64_t sh[40];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    v[i] = idx < n ? in[idx] : 0;
    s += v[i];
  }
  int64_t tot;
  int64_t ex = block_excl_scan(s, sh, tot) + sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t idx = base + (int64_t)threadIdx.x * kScanItems + i;
    if (idx < n) out[idx] = ex;
    ex += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

__device__ __forceinline__ int64_t row_of(const int64_t *__restrict__ rp, int64_t m, int64_t e) {
  int64_t lo = 0, hi = m - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (rp[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ validation
template <typename TV>
__global__ __launch_bounds__(256) void k_validate(int64_t m, int64_t n, int64_t nnz,
                                                  const int64_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col,
                                                  const TV *__restrict__ val,
                                                  int32_t *__restrict__ rowidx,
                                                  int32_t *__restrict__ flags) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int bad = 0, nonfinite = 0;
  // row pointer: starts at 0, nondecreasing, ends at nnz
  for (int64_t r = t0; r < m; r += stride) bad |= rp[r] > rp[r + 1];
  if (t0 == 0 && (rp[0] != 0 || rp[m] != nnz)) bad = 1;
  if (m > 0) {
    for (int64_t e = t0; e < nnz; e += stride) {
      const int64_t r = row_of(rp, m, e);
      const int32_t c = col[e];
      rowidx[e] = (int32_t)r;
      if (c < 0 || (int64_t)c >= n)
        bad = 1;
      else if (e > 0 && e > rp[r] && col[e - 1] >= c)
        bad = 1;
      const double v = (double)val[e];
      if (!(v - v == 0.0)) nonfinite = 1;
    }
  }
  // one atomic per wavefront and flag
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, 1);
  if (__ballot(nonfinite) && (threadIdx.x & 63) == 0) atomicOr(flags, 2);
}

// ------------------------------------------------------------------ transpose
// Entry p of CSR(A^T): the nonzero src[p] of A sorted to position p.
template <typename TV>
__global__ __launch_bounds__(256) void k_tgather(int64_t nnz, const int32_t *__restrict__ src,
                                                 const int32_t *__restrict__ rowidx,
                                                 const TV *__restrict__ val, int32_t *__restrict__ colT,
                                                 TV *__restrict__ valT) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
    const int32_t s = src[p];
    colT[p] = rowidx[s];
    valT[p] = val[s];
  }
}

// Row pointer of A^T: rowT[c] = first position whose sorted column key is
// >= c (c = 0..n; rowT[n] = nnz).
__global__ __launch_bounds__(256) void k_tbounds(int64_t n, int64_t nnz, const uint32_t *__restrict__ keys,
                                                 int64_t *__restrict__ rowT) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n; c += stride) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)keys[mid] < c) lo = mid + 1; else hi = mid;
    }
    rowT[c] = lo;
  }
}

unsigned key_bits(int64_t n) {
  unsigned b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

// ------------------------------------------------------------------ SpMM plan
__global__ __launch_bounds__(256) void k_plan_count(int64_t R, const int64_t *__restrict__ rp,
                                                    int32_t long_row, int64_t *__restrict__ nch) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
    const int64_t len = rp[r + 1] - rp[r];
    nch[r] = len > long_row ? (len + long_row - 1) / long_row : 0;
  }
}

__global__ __launch_bounds__(256) void k_plan_fill(int64_t R, const int64_t *__restrict__ rp,
                                                   int32_t long_row, const int64_t *__restrict__ off,
                                                   ChunkTask *__restrict__ tasks,
                                                   LongRow *__restrict__ longs,
                                                   int32_t *__restrict__ nlong) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
    const int64_t b = rp[r], e = rp[r + 1];
    const int64_t nc = off[r + 1] - off[r];
    if (nc == 0) continue;
    const int32_t slot = atomicAdd(nlong, 1);
    LongRow lr;
    lr.row = r;
    lr.first = off[r];
    lr.nch = nc;
    longs[slot] = lr;
    for (int64_t c = 0; c < nc; ++c) {
      ChunkTask t;
      t.begin = b + c * long_row;
      t.end = t.begin + long_row < e ? t.begin + long_row : e;
      tasks[off[r] + c] = t;
    }
  }
}

__global__ void k_fill_zero_i32(int32_t *p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

}  // namespace

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile + 2); }

hipError_t launch_scan_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *tmp, hipStream_t st) {
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  if (n == 0) {
    return hipMemsetAsync(out, 0, sizeof(int64_t), st);
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, st, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanBlock), 0, st, in, n, tmp, out, nb);
  return hipGetLastError();
}

hipError_t launch_validate(int64_t m, int64_t n, int64_t nnz, const int64_t *rp, const int32_t *col,
                           const void *val, int dtype, int32_t *rowidx, int32_t *flags, hipStream_t st) {
  const int64_t work = nnz > m ? nnz : m;
  const int g = grid_for(work, 256, 16384);
  if (dtype == 1)
    hipLaunchKernelGGL(k_validate<double>, dim3(g), dim3(256), 0, st, m, n, nnz, rp, col,
                       (const double *)val, rowidx, flags);
  else
    hipLaunchKernelGGL(k_validate<float>, dim3(g), dim3(256), 0, st, m, n, nnz, rp, col,
                       (const float *)val, rowidx, flags);
  return hipGetLastError();
}

size_t transpose_ws_bytes(int64_t n, int64_t nnz) {
  size_t sort_bytes = 0;
  const size_t cnt = nnz > 0 ? (size_t)nnz : 1;
  (void)rocprim::radix_sort_pairs(nullptr, sort_bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                  rocprim::counting_iterator<int32_t>(0), (int32_t *)nullptr, cnt, 0u,
                                  key_bits(n));
  return 2 * 4 * (cnt + 64) + sort_bytes + 256;
}

hipError_t launch_transpose(int64_t n, int64_t nnz, const int32_t *col, const int32_t *rowidx, const void *val,
                            int dtype, int64_t *rowT, int32_t *colT, void *valT, void *ws, size_t ws_bytes,
                            hipStream_t st) {
  const size_t cnt = nnz > 0 ? (size_t)nnz : 1;
  uint32_t *keys = (uint32_t *)ws;
  int32_t *src = (int32_t *)(keys + cnt + 64);
  void *tmp = (void *)(src + cnt + 64);
  size_t tmp_bytes = ws_bytes - 2 * 4 * (cnt + 64);
  if (nnz > 0) {
    // validated columns are in [0, n): sort on their low bits only
    const hipError_t e = rocprim::radix_sort_pairs(tmp, tmp_bytes, (const uint32_t *)col, keys,
                                                   rocprim::counting_iterator<int32_t>(0), src, (size_t)nnz, 0u,
                                                   key_bits(n), st);
    if (e != hipSuccess) return e;
    const int g = grid_for(nnz, 256, 16384);
    if (dtype == 1)
      hipLaunchKernelGGL(k_tgather<double>, dim3(g), dim3(256), 0, st, nnz, src, rowidx, (const double *)val,
                         colT, (double *)valT);
    else
      hipLaunchKernelGGL(k_tgather<float>, dim3(g), dim3(256), 0, st, nnz, src, rowidx, (const float *)val,
                         colT, (float *)valT);
  }
  hipLaunchKernelGGL(k_tbounds, dim3(grid_for(n + 1, 256, 16384)), dim3(256), 0, st, n, nnz, keys, rowT);
  return hipGetLastError();
}

hipError_t launch_plan_count(int64_t R, const int64_t *rp, int32_t long_row, int64_t *nch,
                             hipStream_t st) {
  if (R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_count, dim3(grid_for(R, 256, 16384)), dim3(256), 0, st, R, rp, long_row, nch);
  return hipGetLastError();
}

hipError_t launch_plan_fill(int64_t R, const int64_t *rp, int32_t long_row, const int64_t *off,
                            ChunkTask *tasks, LongRow *longs, int32_t *nlong, hipStream_t st) {
  if (R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_fill, dim3(grid_for(R, 256, 16384)), dim3(256), 0, st, R, rp, long_row, off,
                     tasks, longs, nlong);
  return hipGetLastError();
}

hipError_t launch_fill_zero_i32(int32_t *p, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace dsv
