// Batched form: many independent matrices advance pass-synchronously through
// Alg. 5, every step one launch over all of them.
//
// The B operators M_b are stacked into one block-diagonal CSR (rows and
// columns offset per matrix), so the library's transpose and SpMM kernels
// serve all of them at once; a row-to-matrix map lets the SpMM read each
// matrix's shift and stop flag.  The dense steps of eigSVD (Alg. 3) work on
// per-matrix blocks of the stacked panels:
//   - Gram: work items (matrix, strip of rows) each write a partial of the
//     upper triangle of C_b^T C_b in FP64; a second kernel sums the items of
//     each matrix in item order (deterministic);
//   - rescale: Out_b = (C_b - alpha_b R_b) W_b per strip, W_b staged in LDS;
//   - sign normalisation: one workgroup per matrix;
//   - eig: the Jacobi kernel, one workgroup per matrix.
// Work items of a matrix whose pass-start snapshot says stopped are skipped.
#include "common.h"

namespace dsv {

namespace {

constexpr int kBThreads = 256;

// Block-diagonal assembly.  Each matrix b is validated against its own
// sizes (row_ptr[0] = 0, row_ptr[m_b] = nnz_b, columns in [0, n_b)); the
// stacked CSR is then checked as a whole for order, uniqueness and finite
// values by the usual validation kernel.  in_place: the arrays were already
// copied to their stacked positions and only need the offsets.
template <typename TV>
__global__ __launch_bounds__(kBThreads) void k_bassemble(const BMatDesc *__restrict__ d, int64_t *__restrict__ rp,
                                                         int32_t *__restrict__ col, TV *__restrict__ val,
                                                         int in_place, int32_t *__restrict__ flags) {
  const BMatDesc m = d[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < m.m; i += stride) {
    const int64_t v = in_place ? rp[m.row_off + i] : m.rp[i];
    if (i == 0 && v != 0) atomicOr(flags, 1);
    rp[m.row_off + i] = v + m.nnz_off;
  }
  if (t0 == 0) {
    const int64_t last = in_place ? m.nnz : m.rp[m.m];
    if (last != m.nnz) atomicOr(flags, 1);
  }
  for (int64_t j = t0; j < m.nnz; j += stride) {
    const int32_t c = in_place ? col[m.nnz_off + j] : m.col[j];
    if (c < 0 || c >= m.n) atomicOr(flags, 1);
    col[m.nnz_off + j] = c + (int32_t)m.col_off;
    if (!in_place) val[m.nnz_off + j] = ((const TV *)m.val)[j];
  }
}

__global__ void k_bassemble_tail(int64_t *__restrict__ rp, int64_t total_rows, int64_t total_nnz) {
  if (threadIdx.x == 0 && blockIdx.x == 0) rp[total_rows] = total_nnz;
}

// row -> matrix map of one side of the stacked operator
__global__ __launch_bounds__(kBThreads) void k_browmat(const int64_t *__restrict__ off, int count,
                                                       int32_t *__restrict__ rowmat) {
  const int b = blockIdx.y;
  if (b >= count) return;
  const int64_t r0 = off[b], r1 = off[b + 1];
  for (int64_t r = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < r1;
       r += (int64_t)gridDim.x * blockDim.x)
    rowmat[r] = b;
}

// pass-start snapshot of the stop flags (or clearing them, snap = 0)
__global__ __launch_bounds__(kBThreads) void k_bsnap(SolverState *__restrict__ st, int count, int snap) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < count) st[b].pass_skip = snap ? st[b].done : 0;
}

// Gram partials: item it covers rows [r0, r1) of matrix b; entry (i, j),
// i <= j, packed row by row.  Rows are staged in LDS as FP64.
template <typename TC>
__global__ __launch_bounds__(kBThreads) void k_bgram_partial(const BItem *__restrict__ items, int l,
                                                             const TC *__restrict__ C, int64_t ldc,
                                                             double *__restrict__ partial,
                                                             const SolverState *__restrict__ st, int gate) {
  extern __shared__ double strip[];  // kBStrip x l
  const BItem it = items[blockIdx.x];
  const int ne = l * (l + 1) / 2;
  double *out = partial + (int64_t)blockIdx.x * ne;
  if (gate && st[it.mat].pass_skip) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int ei[4], ej[4];
  // entries of this thread: e = tid + 256 s (s < 4 covers l <= 44; larger l
  // loop over entry groups below)
  for (int e0 = 0; e0 < ne; e0 += 4 * kBThreads) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      acc[s] = 0.0;
      int e = e0 + threadIdx.x + s * kBThreads;
      ei[s] = -1;
      ej[s] = 0;
      if (e < ne) {
        int i = 0;
        while (e >= l - i) {
          e -= l - i;
          ++i;
        }
        ei[s] = i;
        ej[s] = i + e;
      }
    }
    for (int64_t rb = it.r0; rb < it.r1; rb += kBStrip) {
      const int nr = (int)((it.r1 - rb) < kBStrip ? (it.r1 - rb) : kBStrip);
      __syncthreads();
      for (int x = threadIdx.x; x < nr * l; x += kBThreads) {
        const int rr = x / l, cc = x - rr * l;
        strip[rr * l + cc] = to_d(C[(rb + rr) * ldc + cc]);
      }
      __syncthreads();
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if (ei[s] < 0) continue;
        double a = acc[s];
        for (int rr = 0; rr < nr; ++rr) a = fma(strip[rr * l + ei[s]], strip[rr * l + ej[s]], a);
        acc[s] = a;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int e = e0 + threadIdx.x + s * kBThreads;
      if (e < ne) out[e] = acc[s];
    }
  }
}

// G_b = sum of the partials of matrix b's items, in item order; full
// symmetric l x l output
__global__ __launch_bounds__(kBThreads) void k_bgram_reduce(const int64_t *__restrict__ item_off, int l,
                                                            const double *__restrict__ partial,
                                                            double *__restrict__ G, int64_t g_stride,
                                                            const SolverState *__restrict__ st, int gate) {
  const int b = blockIdx.y;
  if (gate && st[b].pass_skip) return;
  const int ne = l * (l + 1) / 2;
  const int64_t i0 = item_off[b], i1 = item_off[b + 1];
  double *Gb = G + (int64_t)b * g_stride;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t it = i0; it < i1; ++it) s += partial[it * ne + e];
    int i = 0, r = e;
    while (r >= l - i) {
      r -= l - i;
      ++i;
    }
    const int j = i + r;
    Gb[(int64_t)i * l + j] = s;
    Gb[(int64_t)j * l + i] = s;
  }
}

// Out rows [r0, r1) of matrix b = (C - alpha_b R) W_b (W_b: l x c of a
// row-major l x ldw block), columns c..ldo-1 zero.  FP64 accumulation.
template <typename TC, typename TO>
__global__ __launch_bounds__(kBThreads) void k_brescale(const BItem *__restrict__ items, int l,
                                                        const TC *__restrict__ C, const TC *__restrict__ R,
                                                        int64_t ldc, const double *__restrict__ W,
                                                        int64_t w_stride, int64_t ldw, int c,
                                                        TO *__restrict__ Out, int64_t ldo,
                                                        const SolverState *__restrict__ st, int gate) {
  extern __shared__ double lds[];
  const BItem it = items[blockIdx.x];
  if (gate && st[it.mat].pass_skip) return;
  double *Ws = lds;              // l x c
  double *Cs = lds + l * c;      // kBStrip x l
  const double *Wb = W + (int64_t)it.mat * w_stride;
  for (int x = threadIdx.x; x < l * c; x += kBThreads) {
    const int k = x / c, j = x - k * c;
    Ws[x] = Wb[(int64_t)k * ldw + j];
  }
  const double a = R ? st[it.mat].alpha : 0.0;
  for (int64_t rb = it.r0; rb < it.r1; rb += kBStrip) {
    const int nr = (int)((it.r1 - rb) < kBStrip ? (it.r1 - rb) : kBStrip);
    __syncthreads();
    for (int x = threadIdx.x; x < nr * l; x += kBThreads) {
      const int rr = x / l, kk = x - rr * l;
      double v = to_d(C[(rb + rr) * ldc + kk]);
      if (R) v = fma(-a, to_d(R[(rb + rr) * ldc + kk]), v);
      Cs[rr * l + kk] = v;
    }
    __syncthreads();
    for (int x = threadIdx.x; x < nr * (int)ldo; x += kBThreads) {
      const int rr = x / (int)ldo, j = x - rr * (int)ldo;
      double s = 0.0;
      if (j < c)
        for (int k = 0; k < l; ++k) s = fma(Cs[rr * l + k], Ws[k * c + j], s);
      elem<TO>::st(Out + (rb + rr) * ldo + j, (decltype(elem<TO>::ld(Out)))s);
    }
  }
}

// Sign normalisation of matrix b (one workgroup): for each column the entry
// of largest magnitude of V_b (lowest row on ties) becomes positive, and U_b
// is flipped alike.  Columns go kBSignCols at a time: each thread reads
// whole row segments and keeps the largest entry of every column of the
// group, the wavefronts reduce them lane to lane, wavefront 0 combines the
// wavefronts and picks the signs, then one pass flips the rows of V_b and
// U_b.
constexpr int kBSignCols = 16;
template <typename T>
__global__ __launch_bounds__(kBThreads) void k_bsign(const int64_t *__restrict__ voff, const int64_t *__restrict__ uoff,
                                                     int k, T *__restrict__ V, T *__restrict__ U, int64_t ld) {
  constexpr int NW = kBThreads / kWave;
  __shared__ double smax[NW][kBSignCols];
  __shared__ int64_t sidx[NW][kBSignCols];
  __shared__ double sgn[kBSignCols];
  const int b = blockIdx.x, lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t v0 = voff[b], v1 = voff[b + 1], u0 = uoff[b], u1 = uoff[b + 1];
  for (int i0 = 0; i0 < k; i0 += kBSignCols) {
    const int nc = k - i0 < kBSignCols ? k - i0 : kBSignCols;
    double best[kBSignCols];
    int64_t bi[kBSignCols];
#pragma unroll
    for (int j = 0; j < kBSignCols; ++j) {
      best[j] = -1.0;
      bi[j] = INT64_MAX;
    }
    for (int64_t r = v0 + threadIdx.x; r < v1; r += kBThreads) {
#pragma unroll
      for (int j = 0; j < kBSignCols; ++j) {
        if (j < nc) {
          const double a = fabs(to_d(V[r * ld + i0 + j]));
          if (a > best[j]) {  // rows rise within a thread: the first of equals stays
            best[j] = a;
            bi[j] = r;
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kBSignCols; ++j) {
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const double a = __shfl_xor(best[j], o, kWave);
        const int64_t ii = __shfl_xor(bi[j], o, kWave);
        if (a > best[j] || (a == best[j] && ii < bi[j])) {
          best[j] = a;
          bi[j] = ii;
        }
      }
      if (lane == 0) {
        smax[wave][j] = best[j];
        sidx[wave][j] = bi[j];
      }
    }
    __syncthreads();
    if (threadIdx.x < nc) {
      const int j = threadIdx.x;
      double a = smax[0][j];
      int64_t ii = sidx[0][j];
      for (int w = 1; w < NW; ++w)
        if (smax[w][j] > a || (smax[w][j] == a && sidx[w][j] < ii)) {
          a = smax[w][j];
          ii = sidx[w][j];
        }
      sgn[j] = (ii < v1 && to_d(V[ii * ld + i0 + j]) < 0.0) ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int64_t r = v0 + threadIdx.x; r < v1; r += kBThreads)
      for (int j = 0; j < nc; ++j)
        if (sgn[j] < 0.0) elem<T>::st(V + r * ld + i0 + j, (decltype(elem<T>::ld(V)))(-to_d(V[r * ld + i0 + j])));
    for (int64_t r = u0 + threadIdx.x; r < u1; r += kBThreads)
      for (int j = 0; j < nc; ++j)
        if (sgn[j] < 0.0) elem<T>::st(U + r * ld + i0 + j, (decltype(elem<T>::ld(U)))(-to_d(U[r * ld + i0 + j])));
    __syncthreads();
  }
}

int blocks_for(int64_t work) {
  int64_t g = (work + kBThreads - 1) / kBThreads;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

}  // namespace

hipError_t launch_bassemble(const BMatDesc *d, int count, int64_t max_rows_nnz, int64_t total_rows,
                            int64_t total_nnz, int64_t *rp, int32_t *col, void *val, int vdtype, int in_place,
                            int32_t *flags, hipStream_t st) {
  if (count < 1) return hipSuccess;
  dim3 grid((unsigned)blocks_for(max_rows_nnz), (unsigned)count);
  if (vdtype == 1)
    hipLaunchKernelGGL(k_bassemble<double>, grid, dim3(kBThreads), 0, st, d, rp, col, (double *)val, in_place, flags);
  else
    hipLaunchKernelGGL(k_bassemble<float>, grid, dim3(kBThreads), 0, st, d, rp, col, (float *)val, in_place, flags);
  hipLaunchKernelGGL(k_bassemble_tail, dim3(1), dim3(64), 0, st, rp, total_rows, total_nnz);
  return hipGetLastError();
}

hipError_t launch_browmat(const int64_t *off, int count, int64_t max_rows, int32_t *rowmat, hipStream_t st) {
  if (count < 1) return hipSuccess;
  dim3 grid((unsigned)blocks_for(max_rows), (unsigned)count);
  hipLaunchKernelGGL(k_browmat, grid, dim3(kBThreads), 0, st, off, count, rowmat);
  return hipGetLastError();
}

hipError_t launch_bsnap(SolverState *state, int count, int snap, hipStream_t st) {
  if (count < 1) return hipSuccess;
  hipLaunchKernelGGL(k_bsnap, dim3((count + kBThreads - 1) / kBThreads), dim3(kBThreads), 0, st, state, count,
                     snap);
  return hipGetLastError();
}

size_t bgram_partial_elems(int64_t n_items, int l) { return (size_t)n_items * (size_t)(l * (l + 1) / 2); }

hipError_t launch_bgram(const BItem *items, int64_t n_items, const int64_t *item_off, int count, int l,
                        const void *C, int64_t ldc, int cdtype, double *partial, double *G, int64_t g_stride,
                        const SolverState *state, int gate, hipStream_t st) {
  if (n_items < 1) return hipSuccess;
  if (l < 1 || l > kMaxL || n_items > INT32_MAX) return hipErrorInvalidValue;
  const size_t shm = sizeof(double) * (size_t)kBStrip * l;
  if (cdtype == 0)
    hipLaunchKernelGGL(k_bgram_partial<float>, dim3((unsigned)n_items), dim3(kBThreads), shm, st, items, l,
                       (const float *)C, ldc, partial, state, gate);
  else if (cdtype == 1)
    hipLaunchKernelGGL(k_bgram_partial<double>, dim3((unsigned)n_items), dim3(kBThreads), shm, st, items, l,
                       (const double *)C, ldc, partial, state, gate);
  else
    return hipErrorInvalidValue;
  const int ne = l * (l + 1) / 2;
  dim3 grid((unsigned)((ne + kBThreads - 1) / kBThreads), (unsigned)count);
  hipLaunchKernelGGL(k_bgram_reduce, grid, dim3(kBThreads), 0, st, item_off, l, partial, G, g_stride, state, gate);
  return hipGetLastError();
}

hipError_t launch_brescale(const BItem *items, int64_t n_items, int l, const void *C, const void *R, int64_t ldc,
                           int cdtype, const double *W, int64_t w_stride, int64_t ldw, int c, void *Out,
                           int64_t ldo, int odtype, const SolverState *state, int gate, hipStream_t st) {
  if (n_items < 1) return hipSuccess;
  if (l < 1 || l > kMaxL || c < 1 || c > l || ldo < c || n_items > INT32_MAX) return hipErrorInvalidValue;
  const size_t shm = sizeof(double) * ((size_t)l * c + (size_t)kBStrip * l);
  if (shm > 64 * 1024) return hipErrorInvalidValue;
  const dim3 g((unsigned)n_items), bl(kBThreads);
#define DSV_BR(TC, TO)                                                                                     \
  hipLaunchKernelGGL((k_brescale<TC, TO>), g, bl, shm, st, items, l, (const TC *)C, (const TC *)R, ldc, W, \
                     w_stride, ldw, c, (TO *)Out, ldo, state, gate)
  if (cdtype == 0 && odtype == 0)
    DSV_BR(float, float);
  else if (cdtype == 0 && odtype == 2)
    DSV_BR(float, bf16);
  else if (cdtype == 2 && odtype == 0)
    DSV_BR(bf16, float);
  else if (cdtype == 1 && odtype == 1)
    DSV_BR(double, double);
  else
    return hipErrorInvalidValue;
#undef DSV_BR
  return hipGetLastError();
}

hipError_t launch_bsign(const int64_t *voff, const int64_t *uoff, int count, int k, void *V, void *U, int64_t ld,
                        int dtype, hipStream_t st) {
  if (count < 1) return hipSuccess;
  if (dtype == 0)
    hipLaunchKernelGGL(k_bsign<float>, dim3((unsigned)count), dim3(kBThreads), 0, st, voff, uoff, k, (float *)V,
                       (float *)U, ld);
  else if (dtype == 1)
    hipLaunchKernelGGL(k_bsign<double>, dim3((unsigned)count), dim3(kBThreads), 0, st, voff, uoff, k,
                       (double *)V, (double *)U, ld);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dsv
