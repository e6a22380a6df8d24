// Dense head of a degree-ordered sparse operand, for the products with M and
// M^T of the power pass (Alg. 5 steps 2, 4 and 9).
//
// With the rows in non-increasing nonzero count, the first rows of a
// power-law matrix are nearly dense: on a 200000 x 100000 Zipf(1.1) matrix
// the first 128 rows hold 41 % of the 10M nonzeros, with 9 to 100 % of the
// columns each.  The row-split SpMM gathers one full panel row per nonzero,
// so those rows read the panel over and over (and they cost more per nonzero
// than the rest: leaving the first 128 rows out made the product of that
// matrix 2.1x faster).  As a dense product on the matrix cores, the panel is
// read once for all of them.  The SpMM plan leaves the head rows out of its
// chunks, and these kernels fill them:
//   - k_head_count: H, the leading rows with at least max(long_row + 1,
//     ncols / 16) nonzeros, at most kHeadMax; none if fewer than
//     kHeadMinRows qualify or if they hold fewer than kHeadNnzPerCol x ncols
//     nonzeros (the dense product reads the whole panel once, about what
//     that many gathers of the row-split kernel cost);
//   - k_head_clear, k_head_scatter: Dt = M[0:H, :]^T as a dense
//     ncols x kHeadMax array (its columns H..Hp-1 zero, Hp = H rounded up
//     to 16; the columns past Hp are never read);
//   - k_head_partial: kHeadSplits row ranges of the panel X; block s forms
//     the H x ldc product Dt[range]^T X[range] on v_mfma_f32_16x16x4 (FP32
//     and BF16 panels, FP32 accumulation as in the SpMM) or
//     v_mfma_f64_16x16x4 (FP64), with the operands loaded straight from
//     memory a few k-steps ahead (the layout of the Gram kernel: lane L holds
//     A[L%16][L/16] and B[L/16][L%16]);
//   - k_head_reduce: sums the partial products in split order (the result
//     does not depend on scheduling), subtracts alpha Q for the shifted
//     product, and writes rows 0..H-1 of Y.
#include <algorithm>

#include "common.h"

namespace dsv {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// Partial products: 8 x 10 tiles of 16 x 16 per split (H <= 128 rows,
// ldc <= 160 columns), in the accumulator layout (tile, lane, register).
constexpr int kHeadTiles = kHeadMax / 16;
constexpr int kHeadTilesJ = kHeadMaxCols / 16;
constexpr int64_t kHeadSplitElems = (int64_t)kHeadTiles * kHeadTilesJ * 256;

template <typename TA> struct head_mfma;
template <> struct head_mfma<float> {
  typedef f4 acc;
  __device__ static __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register q of lane L holds D[4 (L / 16) + q][L % 16]
  __device__ static __forceinline__ int row(int L, int q) { return 4 * (L >> 4) + q; }
};
template <> struct head_mfma<double> {
  typedef d4 acc;
  __device__ static __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator register q of lane L holds D[L / 16 + 4 q][L % 16]
  __device__ static __forceinline__ int row(int L, int q) { return (L >> 4) + 4 * q; }
};

// Raw buffer loads: an offset at or past the end of the range reads zero.
constexpr int kHeadBufWord3 = 0x00020000;
__device__ __forceinline__ float hb_ld(__amdgpu_buffer_rsrc_t r, int off, const float *) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double hb_ld(__amdgpu_buffer_rsrc_t r, int off, const double *) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float hb_ld(__amdgpu_buffer_rsrc_t r, int off, const bf16 *) {
  return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0) << 16);
}

__device__ __forceinline__ bool head_done(const int32_t *done) {
  return done && __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kHeadMax) void k_head_count(int64_t R, const int64_t *__restrict__ rp, int64_t thr,
                                                         int64_t min_nnz, int32_t *__restrict__ out) {
  __shared__ int first;
  const int lim = (int)(R < kHeadMax ? R : kHeadMax);
  if (threadIdx.x == 0) first = lim;
  __syncthreads();
  const int i = threadIdx.x;
  if (i < lim && rp[i + 1] - rp[i] < thr) atomicMin(&first, i);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int h = first;
    *out = h >= kHeadMinRows && rp[h] - rp[0] >= min_nnz ? h : 0;
  }
}

// Dt: the first Hp = 16 ceil(H / 16) entries of each of its ncols rows are
// cleared, then every nonzero of the head rows of M (entries [rp[0], rp[H]),
// its row found by a search over rp[0..H]) is stored at Dt[column][row].
// Each (column, row) pair occurs once, so the scattered stores never meet.
template <typename TA>
__global__ __launch_bounds__(256) void k_head_clear(int64_t ncols, int Hp, TA *__restrict__ Dt) {
  // 16 lanes a row
  const int64_t g0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int64_t gs = ((int64_t)gridDim.x * blockDim.x) >> 4;
  const int q = threadIdx.x & 15;
  for (int64_t c = g0; c < ncols; c += gs)
    for (int i = q; i < Hp; i += 16) Dt[c * kHeadMax + i] = (TA)0;
}

template <typename TV, typename TA>
__global__ __launch_bounds__(256) void k_head_scatter(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                      const TV *__restrict__ val, int H, TA *__restrict__ Dt) {
  __shared__ int64_t rps[kHeadMax + 1];
  for (int i = threadIdx.x; i <= H; i += blockDim.x) rps[i] = rp[i];
  __syncthreads();
  const int64_t b = rps[0], e = rps[H];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < e; j += stride) {
    // the row r with rps[r] <= j < rps[r + 1]
    int lo = 0, hi = H - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rps[mid] <= j) lo = mid; else hi = mid - 1;
    }
    Dt[(int64_t)col[j] * kHeadMax + lo] = (TA)val[j];
  }
}

// Block s: rows [s K / S, (s + 1) K / S) of X and Dt.  Wavefront w owns the
// tile row w (and w + 4 when TWO) of the H x ldc product and its first NJ
// tile columns (NJ >= ceil(ldc / 16)); its lanes load their A operands (Dt)
// and B operands (X) P k-steps ahead.  Every MFMA is unconditional (the
// operands past H and ldc are zero), so the accumulators stay in place.
template <typename TX, typename TA, int P, int NJ, bool TWO>
__global__ __launch_bounds__(256) void k_head_partial(int64_t K, const TX *__restrict__ X, int64_t ldx, int ldc,
                                                      int H, const TA *__restrict__ Dt,
                                                      const int32_t *__restrict__ done, TA *__restrict__ part) {
  if (head_done(done)) return;
  using M = head_mfma<TA>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kr = lane >> 4, kc = lane & 15;
  const int TI = (H + 15) >> 4;
  const int ti0 = wave, ti1 = wave + 4;
  if (ti0 >= TI) return;
  const bool two = TWO && ti1 < TI;
  const int64_t s = blockIdx.x;
  const int64_t k0 = s * K / kHeadSplits, k1 = (s + 1) * K / kHeadSplits;
  typename M::acc acc0[NJ], acc1[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    acc0[j] = typename M::acc{0, 0, 0, 0};
    acc1[j] = typename M::acc{0, 0, 0, 0};
  }
  const int64_t rows = k1 - k0;
  if (rows > 0) {
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(X + k0 * ldx), 0, (int)(rows * ldx * (int64_t)sizeof(TX)), kHeadBufWord3);
    const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(Dt + k0 * kHeadMax), 0, (int)(rows * kHeadMax * (int64_t)sizeof(TA)), kHeadBufWord3);
    bool colok[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) colok[j] = 16 * j + kc < ldc;
    const int xstep = (int)(4 * ldx * (int64_t)sizeof(TX));
    constexpr int dstep = 4 * kHeadMax * (int)sizeof(TA);
    int xo = (int)((kr * ldx + kc) * (int64_t)sizeof(TX));
    int dof = (kr * kHeadMax + kc) * (int)sizeof(TA);
    // tile row ti1 of a wave without one reads past the range (zero)
    const int d1 = two ? 16 * ti1 * (int)sizeof(TA) : (int)(rows * kHeadMax * (int64_t)sizeof(TA));
    TA xa[P][NJ], da[P][2];
#pragma unroll
    for (int p = 0; p < P; ++p) {
#pragma unroll
      for (int j = 0; j < NJ; ++j) xa[p][j] = (TA)hb_ld(rx, xo + 16 * j * (int)sizeof(TX), X);
      da[p][0] = hb_ld(rd, dof + 16 * ti0 * (int)sizeof(TA), Dt);
      if constexpr (TWO) da[p][1] = hb_ld(rd, dof + d1, Dt);
      xo += xstep;
      dof += dstep;
    }
    for (int64_t kb = 0; kb < rows; kb += 4 * P) {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        TA bv[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) bv[j] = colok[j] ? xa[p][j] : (TA)0;
        const TA a0 = da[p][0];
        const TA a1 = TWO ? da[p][1] : (TA)0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) xa[p][j] = (TA)hb_ld(rx, xo + 16 * j * (int)sizeof(TX), X);
        da[p][0] = hb_ld(rd, dof + 16 * ti0 * (int)sizeof(TA), Dt);
        if constexpr (TWO) da[p][1] = hb_ld(rd, dof + d1, Dt);
        xo += xstep;
        dof += dstep;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          acc0[j] = M::step(a0, bv[j], acc0[j]);
          if constexpr (TWO) acc1[j] = M::step(a1, bv[j], acc1[j]);
        }
      }
    }
  }
  TA *out = part + s * kHeadSplitElems;
  const int TJ = (ldc + 15) >> 4;
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    if (j >= TJ) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // through a VGPR before the store (as in the Gram kernel, whose FP64
      // accumulators stored directly read back stale rows)
      TA x0 = acc0[j][q];
      asm volatile("" : "+v"(x0));
      out[(int64_t)(ti0 * kHeadTilesJ + j) * 256 + lane * 4 + q] = x0;
      if (two) {
        TA x1 = acc1[j][q];
        asm volatile("" : "+v"(x1));
        out[(int64_t)(ti1 * kHeadTilesJ + j) * 256 + lane * 4 + q] = x1;
      }
    }
  }
}

// Block b: 64 elements of tile b / 4 of the product; wavefront w sums splits
// [w S / 4, (w + 1) S / 4) in order, and the four sums are added in
// wavefront order.
template <typename TX, typename TA, typename TY, bool SHIFT>
__global__ __launch_bounds__(256) void k_head_reduce(int H, int ldc, const TA *__restrict__ part,
                                                     TY *__restrict__ Y, int64_t ldy, const TX *__restrict__ Q,
                                                     int64_t ldq, const double *__restrict__ alpha,
                                                     const int32_t *__restrict__ done) {
  if (head_done(done)) return;
  __shared__ TA red[4][64];
  const int TJ = (ldc + 15) >> 4;
  const int tile = blockIdx.x >> 2;
  const int ti = tile / TJ, tj = tile - ti * TJ;
  const int wave = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int e = (blockIdx.x & 3) * 64 + t;
  const TA *p = part + (int64_t)(ti * kHeadTilesJ + tj) * 256 + e;
  constexpr int SQ = kHeadSplits / 4;
  const int s0 = wave * SQ;
  TA sum = (TA)0;
  for (int s = s0; s < s0 + SQ; s += 8) {
    TA v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(int64_t)(s + u) * kHeadSplitElems];
#pragma unroll
    for (int u = 0; u < 8; ++u) sum += v[u];
  }
  red[wave][t] = sum;
  __syncthreads();
  if (wave != 0) return;
  TA y = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
  const int L = e >> 2, q = e & 3;
  const int i = 16 * ti + head_mfma<TA>::row(L, q), j = 16 * tj + (L & 15);
  if (i >= H || j >= ldc) return;
  if constexpr (SHIFT) y = y - (TA)(*alpha) * (TA)elem<TX>::ld(Q + (int64_t)i * ldq + j);
  elem<TY>::st(Y + (int64_t)i * ldy + j, y);
}

template <typename TX, typename TA, typename TY>
hipError_t run_head(int H, int64_t K, const void *X, int64_t ldx, int ldc, const void *Dt, void *part, void *Y,
                    int64_t ldy, const void *Q, int64_t ldq, const double *alpha, const int32_t *done,
                    hipStream_t st) {
  constexpr int P = sizeof(TA) == 8 ? 6 : 12;
  const int TI = (H + 15) / 16, TJ = (ldc + 15) / 16;
  const bool two = TI > 4;
#define DSV_HEAD_PARTIAL(NJ, TWO)                                                                                 \
  hipLaunchKernelGGL((k_head_partial<TX, TA, P, NJ, TWO>), dim3(kHeadSplits), dim3(256), 0, st, K, (const TX *)X, \
                     ldx, ldc, H, (const TA *)Dt, done, (TA *)part)
  if (TJ <= 2) {
    if (two) DSV_HEAD_PARTIAL(2, true); else DSV_HEAD_PARTIAL(2, false);
  } else if (TJ <= 4) {
    if (two) DSV_HEAD_PARTIAL(4, true); else DSV_HEAD_PARTIAL(4, false);
  } else if (TJ <= 8) {
    if (two) DSV_HEAD_PARTIAL(8, true); else DSV_HEAD_PARTIAL(8, false);
  } else {
    if (two) DSV_HEAD_PARTIAL(kHeadTilesJ, true); else DSV_HEAD_PARTIAL(kHeadTilesJ, false);
  }
#undef DSV_HEAD_PARTIAL
  if (alpha)
    hipLaunchKernelGGL((k_head_reduce<TX, TA, TY, true>), dim3(TI * TJ * 4), dim3(256), 0, st, H, ldc,
                       (const TA *)part, (TY *)Y, ldy, (const TX *)Q, ldq, alpha, done);
  else
    hipLaunchKernelGGL((k_head_reduce<TX, TA, TY, false>), dim3(TI * TJ * 4), dim3(256), 0, st, H, ldc,
                       (const TA *)part, (TY *)Y, ldy, (const TX *)Q, ldq, alpha, done);
  return hipGetLastError();
}

}  // namespace

size_t head_dt_bytes(int64_t ncols, int tdtype) {
  return (size_t)ncols * kHeadMax * (tdtype == 1 ? 8 : 4);
}

size_t head_part_bytes(int tdtype) { return (size_t)kHeadSplits * kHeadSplitElems * (tdtype == 1 ? 8 : 4); }

bool head_fits(int64_t K, int64_t ldx, int xdtype, int ldc) {
  const int64_t xs = xdtype == 1 ? 8 : xdtype == 2 ? 2 : 4;
  const int64_t rows = K / kHeadSplits + 1 + 4 * 6;
  const int64_t wmax = (ldx * xs > kHeadMax * 8 ? ldx * xs : kHeadMax * 8);
  return ldc <= kHeadMaxCols && rows * wmax < ((int64_t)1 << 31) - 4096;
}

hipError_t launch_head_count(int64_t R, const int64_t *rp, int64_t thr, int64_t min_nnz, int32_t *out,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_head_count, dim3(1), dim3(kHeadMax), 0, st, R, rp, thr, min_nnz, out);
  return hipGetLastError();
}

hipError_t launch_head_build(int64_t ncols, const int64_t *rp, const int32_t *col, const void *val, int vdtype,
                             int H, void *Dt, int tdtype, hipStream_t st) {
  if (H <= 0 || H > kHeadMax || ncols <= 0) return hipErrorInvalidValue;
  const int Hp = (H + 15) & ~15;
  const unsigned cgrid = (unsigned)std::min<int64_t>((ncols * 16 + 255) / 256, 16384);
  if (vdtype == 0 && tdtype == 0) {
    hipLaunchKernelGGL((k_head_clear<float>), dim3(cgrid), dim3(256), 0, st, ncols, Hp, (float *)Dt);
    hipLaunchKernelGGL((k_head_scatter<float, float>), dim3(4096), dim3(256), 0, st, rp, col, (const float *)val, H,
                       (float *)Dt);
  } else if (vdtype == 1 && tdtype == 1) {
    hipLaunchKernelGGL((k_head_clear<double>), dim3(cgrid), dim3(256), 0, st, ncols, Hp, (double *)Dt);
    hipLaunchKernelGGL((k_head_scatter<double, double>), dim3(4096), dim3(256), 0, st, rp, col, (const double *)val,
                       H, (double *)Dt);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_head_product(int H, int64_t K, const void *X, int64_t ldx, int xdtype, int ldc, const void *Dt,
                               int tdtype, void *part, void *Y, int64_t ldy, int ydtype, const void *Q,
                               int64_t ldq, const double *alpha, const int32_t *done, hipStream_t st) {
  if (H <= 0 || H > kHeadMax || K <= 0 || !head_fits(K, ldx, xdtype, ldc)) return hipErrorInvalidValue;
  // the accumulation type of the SpMM: FP64 for FP64 panels, else FP32
  if (tdtype != (xdtype == 1 ? 1 : 0)) return hipErrorInvalidValue;
  if (xdtype == 0 && ydtype == 0)
    return run_head<float, float, float>(H, K, X, ldx, ldc, Dt, part, Y, ldy, Q, ldq, alpha, done, st);
  if (xdtype == 1 && ydtype == 1)
    return run_head<double, double, double>(H, K, X, ldx, ldc, Dt, part, Y, ldy, Q, ldq, alpha, done, st);
  if (xdtype == 2 && ydtype == 2)
    return run_head<bf16, float, bf16>(H, K, X, ldx, ldc, Dt, part, Y, ldy, Q, ldq, alpha, done, st);
  if (xdtype == 2 && ydtype == 0)
    return run_head<bf16, float, float>(H, K, X, ldx, ldc, Dt, part, Y, ldy, Q, ldq, alpha, done, st);
  return hipErrorInvalidValue;
}

}  // namespace dsv
