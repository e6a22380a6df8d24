// Dense tall-skinny kernels of eigSVD (Alg. 3) and of the final step of
// Alg. 5, plus small utilities.
//
// Gram G = C^T C (Alg. 3 step 1), FP64 accumulation on the FP64 matrix
// cores: the l columns are cut into T = ceil(l/16) tiles and only the
// T(T+1)/2 upper tiles are computed.  A 256-thread block stages 32 rows of C
// in LDS as FP64 (FP32 inputs convert exactly), and each wavefront owns a
// fixed set of upper tiles, issuing v_mfma_f64_16x16x4 per tile per 4 rows.
// Every block writes its partial tiles; a second kernel sums the partials in
// block order (deterministic) and mirrors the upper triangle.
//
// Rescale Out = C W (Alg. 3 step 3, and U = B W_B, V = Q V_B of Alg. 5
// step 11).  FP32 / BF16 path: W (l x c) is converted to FP32 once per block
// into LDS; each wavefront walks 16-row tiles of C, loading its A operand
// straight from memory, and computes all output tiles of its rows with
// v_mfma_f32_16x16x4.  FP64 path: plain FP64 FMAs (used for the FP64 form).
//
// MFMA operand layout (16x16x4, one block): lane L holds A[L%16][L/16] and
// B[L/16][L%16].  Accumulators: FP32 register q of lane L is D[4*(L/16)+q][L%16];
// FP64 register q of lane L is D[L/16+4q][L%16].
#include "common.h"

namespace dsv {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));


// ------------------------------------------------------------------ Gram
constexpr int kGramRows = 32;

template <typename TC, int LT>
__global__ __launch_bounds__(256) void k_gram_partial(int64_t r, int l, const TC *__restrict__ C,
                                                      int64_t ldc, double *__restrict__ partial,
                                                      int64_t rows_per_block,
                                                      const int32_t *__restrict__ done,
                                                      int32_t *__restrict__ snap) {
  if (done) {
    const int32_t d = *done;
    if (snap && blockIdx.x == 0 && threadIdx.x == 0) *snap = d;
    if (d) return;
  }
  constexpr int NT = LT * (LT + 1) / 2;
  constexpr int TPW = (NT + 3) / 4;
  constexpr int W = LT * 16;
  constexpr int S = W + 1;  // LDS row stride (doubles), odd to spread banks
  __shared__ double tile[kGramRows * S];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int tI[TPW], tJ[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    int t = wave + 4 * i, I = 0;
    if (t >= NT) t = NT - 1;  // duplicate work is discarded below
    while (t >= LT - I) {
      t -= LT - I;
      ++I;
    }
    tI[i] = I;
    tJ[i] = I + t;
  }
  d4 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t row0 = (int64_t)blockIdx.x * rows_per_block;
  int64_t row1 = row0 + rows_per_block;
  if (row1 > r) row1 = r;
  const int kr = lane >> 4, kc = lane & 15;
  for (int64_t rb = row0; rb < row1; rb += kGramRows) {
    for (int idx = threadIdx.x; idx < kGramRows * W; idx += 256) {
      const int rr = idx / W, cc = idx - rr * W;
      const int64_t row = rb + rr;
      tile[rr * S + cc] = (row < row1 && cc < l) ? to_d(C[row * ldc + cc]) : 0.0;
    }
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < kGramRows / 4; ++s) {
      const double *trow = tile + (s * 4 + kr) * S + kc;
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        if (wave + 4 * i < NT) {
          // The B column offset is made opaque to the compiler so that a
          // diagonal tile loads A and B into different registers: an FP64
          // MFMA fed the same VGPR pair as both operands returned wrong rows
          // 8-15 of the tile on gfx950.
          int jo = tJ[i] * 16;
          asm volatile("" : "+v"(jo));
          const double a = trow[tI[i] * 16];
          const double b = trow[jo];
          acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  double *out = partial + (int64_t)blockIdx.x * NT * 256;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = wave + 4 * i;
    if (t < NT) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // Move the accumulator through a VGPR before storing: a store that
        // read the FP64 MFMA accumulator registers directly returned stale
        // values for the last rows written by the final MFMA on gfx950.
        double v = acc[i][q];
        asm volatile("" : "+v"(v));
        out[(int64_t)t * 256 + lane * 4 + q] = v;
      }
    }
  }
}

// Sum the block partials; write the full symmetric G.  Eight threads share
// an element: thread s sums blocks s, s+8, s+16, ... in order, then the eight
// partial sums are added in order s = 0..7 (deterministic).
template <int LT>
__global__ __launch_bounds__(256) void k_gram_reduce(int l, int nblocks, const double *__restrict__ partial,
                                                     double *__restrict__ G,
                                                     const int32_t *__restrict__ done) {
  if (done && *done) return;
  constexpr int NT = LT * (LT + 1) / 2;
  __shared__ double part[256];
  const int sub = threadIdx.x & 7;
  const int64_t e = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
  double s = 0.0;
  if (e < (int64_t)NT * 256) {
    const int64_t stride = (int64_t)NT * 256;
    const double *p = partial + e;
    int b = sub;
    for (; b + 24 < nblocks; b += 32) {
      const double x0 = p[(int64_t)b * stride], x1 = p[(int64_t)(b + 8) * stride];
      const double x2 = p[(int64_t)(b + 16) * stride], x3 = p[(int64_t)(b + 24) * stride];
      s += x0;
      s += x1;
      s += x2;
      s += x3;
    }
    for (; b < nblocks; b += 8) s += p[(int64_t)b * stride];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (sub != 0 || e >= (int64_t)NT * 256) return;
  double tot = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) tot += part[threadIdx.x + i];
  int t = (int)(e >> 8);
  const int within = (int)(e & 255);
  const int lane = within >> 2, q = within & 3;
  int I = 0;
  while (t >= LT - I) {
    t -= LT - I;
    ++I;
  }
  const int J = I + t;
  // FP64 16x16x4 accumulator: register q of lane L holds D[L/16 + 4q][L%16]
  const int row = I * 16 + (lane >> 4) + 4 * q;
  const int col = J * 16 + (lane & 15);
  if (row >= l || col >= l) return;
  if (I == J && row > col) return;
  G[(int64_t)row * l + col] = tot;
  G[(int64_t)col * l + row] = tot;
}

// ------------------------------------------------------------------ rescale
// Four consecutive elements of an FP32 or BF16 row (one 16- or 8-byte load).
__device__ __forceinline__ float4 load4f(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ float4 load4f(const bf16 *p) {
  const uint2 u = *reinterpret_cast<const uint2 *>(p);
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u), __uint_as_float(u.y << 16),
                     __uint_as_float(u.y & 0xffff0000u));
}

// FP32 MFMA rescale.  W (LK x WC, FP32) is staged once per block in LDS;
// each wavefront then walks 16-row tiles of C on its own (no block
// barriers after the staging).  For a k-slab of 16, lane L loads the four
// consecutive elements k0 + 4(L/16) .. +3 of row L%16 with one vector load
// and feeds them to four MFMA steps; step s uses k = k0 + 4(L/16) + s in
// both operands (a permutation of the k order inside the slab), so the A
// operand never goes through LDS.  The next slab's loads are issued before
// the current slab's MFMAs.  Columns k >= l of C are masked to zero (pad
// columns may hold anything); with R, the input is C - alpha R, formed in
// FP64 and rounded once.
template <typename TC, typename TO, int LTO>
__global__ __launch_bounds__(256) void k_rescale_mfma(int64_t r, int l, const TC *__restrict__ C,
                                                      int64_t ldc, const double *__restrict__ W,
                                                      int64_t ldw, int c, TO *__restrict__ Out,
                                                      int64_t ldo, const int32_t *__restrict__ done,
                                                      const TC *__restrict__ R,
                                                      const double *__restrict__ alpha) {
  if (done && *done) return;
  const double a_sh = R ? *alpha : 0.0;
  constexpr int WC = LTO * 16;
  constexpr int SW = WC + 4;
  extern __shared__ float lds[];
  const int LK = (l + 15) & ~15;  // k-slabs of 16
  float *Ws = lds;                // LK x SW
  for (int idx = threadIdx.x; idx < LK * WC; idx += 256) {
    const int kk = idx / WC, cc = idx - kk * WC;
    Ws[kk * SW + cc] = (kk < l && cc < c) ? (float)W[(int64_t)kk * ldw + cc] : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, kq = lane >> 4;  // A row, k quad
  const int64_t ntiles = (r + 15) / 16;
  const int nslab = LK / 16;
  auto load_slab = [&](int64_t row, int k0) -> float4 {
    const int kb = k0 + 4 * kq;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row < r && kb < l) {
      // ld is a multiple of 8 and kb of 4: the vector stays inside the row
      v = load4f(C + row * ldc + kb);
      if (R) {
        const float4 w = load4f(R + row * ldc + kb);
        v.x = (float)((double)v.x - a_sh * (double)w.x);
        v.y = (float)((double)v.y - a_sh * (double)w.y);
        v.z = (float)((double)v.z - a_sh * (double)w.z);
        v.w = (float)((double)v.w - a_sh * (double)w.w);
      }
      if (kb + 1 >= l) v.y = 0.f;
      if (kb + 2 >= l) v.z = 0.f;
      if (kb + 3 >= l) v.w = 0.f;
    }
    return v;
  };
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t row = tile * 16 + lr;
    f4 acc[LTO];
#pragma unroll
    for (int J = 0; J < LTO; ++J) acc[J] = f4{0.f, 0.f, 0.f, 0.f};
    float4 cur = load_slab(row, 0);
    for (int sl = 0; sl < nslab; ++sl) {
      const int k0 = sl * 16;
      const float4 nxt = sl + 1 < nslab ? load_slab(row, k0 + 16) : make_float4(0.f, 0.f, 0.f, 0.f);
      const float av[4] = {cur.x, cur.y, cur.z, cur.w};
#pragma unroll
      for (int s_ = 0; s_ < 4; ++s_) {
        const float *bw = Ws + (k0 + 4 * kq + s_) * SW + lr;
#pragma unroll
        for (int J = 0; J < LTO; ++J)
          acc[J] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s_], bw[J * 16], acc[J], 0, 0, 0);
      }
      cur = nxt;
    }
    const int64_t rbase = tile * 16 + 4 * kq;
#pragma unroll
    for (int J = 0; J < LTO; ++J) {
      const int col = J * 16 + lr;
      if (col < ldo) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t orow = rbase + q;
          float v = acc[J][q];
          asm volatile("" : "+v"(v));
          if (orow < r) elem<TO>::st(Out + orow * ldo + col, col < c ? v : 0.0f);
        }
      }
    }
    // columns beyond the tiles (ldo > WC) are zero
    if (ldo > WC) {
      for (int q = 0; q < 4; ++q) {
        const int64_t orow = rbase + q;
        if (orow < r)
          for (int64_t cc = WC + lr; cc < ldo; cc += 16) elem<TO>::st(Out + orow * ldo + cc, 0.0f);
      }
    }
  }
}

template <typename TC>
__global__ __launch_bounds__(256) void k_rescale_f64(int64_t r, int l, const TC *__restrict__ C,
                                                     int64_t ldc, const double *__restrict__ W,
                                                     int64_t ldw, int c, double *__restrict__ Out,
                                                     int64_t ldo, const int32_t *__restrict__ done,
                                                     const TC *__restrict__ R,
                                                     const double *__restrict__ alpha) {
  if (done && *done) return;
  const double a_sh = R ? *alpha : 0.0;
  const int64_t total = r * ldo;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t row = e / ldo;
    const int col = (int)(e - row * ldo);
    double s = 0.0;
    if (col < c) {
      const TC *cr = C + row * ldc;
      if (R) {
        const TC *rr = R + row * ldc;
        for (int k = 0; k < l; ++k) s = fma(fma(-a_sh, to_d(rr[k]), to_d(cr[k])), W[(int64_t)k * ldw + col], s);
      } else {
        for (int k = 0; k < l; ++k) s = fma(to_d(cr[k]), W[(int64_t)k * ldw + col], s);
      }
    }
    Out[row * ldo + col] = s;
  }
}

// ------------------------------------------------------------------ signs
// Sign normalisation on output: the entry of largest magnitude of each V
// column (lowest row on ties) is made positive; the same flip is applied to
// the matching U column.
template <typename T>
__global__ __launch_bounds__(256) void k_sign_partial(int64_t rows, int k, const T *__restrict__ V,
                                                      int64_t ldv, double *__restrict__ pmax,
                                                      int64_t *__restrict__ pidx) {
  __shared__ double smax[256];
  __shared__ int64_t sidx[256];
  const int per = blockDim.x / k;  // >= 1 since k <= 256
  const int t = threadIdx.x, cidx = t % k, sub = t / k;
  const int64_t chunk = (rows + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  int64_t r1 = r0 + chunk;
  if (r1 > rows) r1 = rows;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  if (sub < per) {
    for (int64_t i = r0 + sub; i < r1; i += per) {
      const double a = fabs(to_d(V[i * ldv + cidx]));
      if (a > best) {
        best = a;
        bi = i;
      }
    }
  }
  smax[t] = best;
  sidx[t] = bi;
  __syncthreads();
  if (sub == 0) {
    for (int s = 1; s < per; ++s) {
      const double a = smax[s * k + cidx];
      const int64_t ii = sidx[s * k + cidx];
      if (a > best || (a == best && ii < bi)) {
        best = a;
        bi = ii;
      }
    }
    pmax[(int64_t)blockIdx.x * k + cidx] = best;
    pidx[(int64_t)blockIdx.x * k + cidx] = bi;
  }
}

// One block: combine the per-block partial maxima in block order and store
// the sign of each column (+1 / -1) before any element is flipped.
// Column c = blockIdx.x: the largest |V| over the nblk partial maxima
// (lowest row on ties) by a tree in LDS, then the sign of that entry.
template <typename T>
__global__ __launch_bounds__(256) void k_sign_select(int k, const T *__restrict__ V, int64_t ldv,
                                                     const double *__restrict__ pmax,
                                                     const int64_t *__restrict__ pidx, int nblk,
                                                     float *__restrict__ sgn) {
  __shared__ double sm[256];
  __shared__ int64_t si[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int b = t; b < nblk; b += blockDim.x) {
    const double a = pmax[(int64_t)b * k + c];
    const int64_t ii = pidx[(int64_t)b * k + c];
    if (a > best || (a == best && ii < bi)) {
      best = a;
      bi = ii;
    }
  }
  sm[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      const double a = sm[t + h];
      const int64_t ii = si[t + h];
      if (a > sm[t] || (a == sm[t] && ii < si[t])) {
        sm[t] = a;
        si[t] = ii;
      }
    }
    __syncthreads();
  }
  if (t == 0) sgn[c] = (si[0] != INT64_MAX && to_d(V[si[0] * ldv + c]) < 0.0) ? -1.0f : 1.0f;
}

// Columns of one matrix times the signs.
template <typename T>
__global__ __launch_bounds__(256) void k_sign_cols(int64_t rows, int k, T *__restrict__ V, int64_t ldv,
                                                   const float *__restrict__ sgn) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rows * k; e += stride) {
    const int64_t i = e / k;
    const int c = (int)(e - i * k);
    if (sgn[c] < 0.f) V[i * ldv + c] = -V[i * ldv + c];
  }
}

// Columns of a small FP64 matrix times the signs.
__global__ __launch_bounds__(256) void k_sign_small(int rows, int k, double *__restrict__ P, int ldp,
                                                    const float *__restrict__ sgn) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * k) return;
  const int i = e / k, c = e - i * k;
  if (sgn[c] < 0.f) P[(int64_t)i * ldp + c] = -P[(int64_t)i * ldp + c];
}

template <typename T>
__global__ __launch_bounds__(256) void k_sign_apply(int64_t rowsV, int64_t rowsU, int k, T *__restrict__ V,
                                                    int64_t ldv, T *__restrict__ U, int64_t ldu,
                                                    const float *__restrict__ sgn) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tv = rowsV * k, tu = rowsU * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tv + tu; e += stride) {
    if (e < tv) {
      const int64_t i = e / k;
      const int c = (int)(e - i * k);
      if (sgn[c] < 0.f) V[i * ldv + c] = -V[i * ldv + c];
    } else {
      const int64_t f = e - tv;
      const int64_t i = f / k;
      const int c = (int)(f - i * k);
      if (sgn[c] < 0.f) U[i * ldu + c] = -U[i * ldu + c];
    }
  }
}

// ------------------------------------------------------------------ conversion
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_copy2d(const TI *__restrict__ in, int64_t ldi, TO *__restrict__ out,
                                                int64_t ldo, int64_t rows, int cols) {
  const int64_t total = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / cols;
    const int j = (int)(e - i * cols);
    out[i * ldo + j] = (TO)in[i * ldi + j];
  }
}

int grid_for(int64_t work, int block, int64_t cap = 65536) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

template <typename TC>
hipError_t gram_dispatch(int64_t r, int l, const TC *C, int64_t ldc, double *partial, int nb,
                         double *G, const int32_t *done, hipStream_t st, int32_t *snap) {
  // at least two column tiles: the single-tile instantiation returned wrong
  // values in the last 4 x 4 corner of the tile once several MFMAs had
  // accumulated (l = 16, 32+ rows) on gfx950, the two-tile one does not
  const int LT = (l + 15) / 16 < 2 ? 2 : (l + 15) / 16;
  const int64_t rpb = (r + nb - 1) / nb;
#define DSV_GRAM(LTV)                                                                          \
  case LTV: {                                                                                  \
    hipLaunchKernelGGL((k_gram_partial<TC, LTV>), dim3(nb), dim3(256), 0, st, r, l, C, ldc, partial, \
                       rpb, done, snap);                                                       \
    constexpr int NT = LTV * (LTV + 1) / 2;                                                    \
    hipLaunchKernelGGL((k_gram_reduce<LTV>), dim3((NT * 256 + 31) / 32), dim3(256), 0, st, l, nb, \
                       partial, G, done);                                                      \
    break;                                                                                     \
  }
  switch (LT) {
    DSV_GRAM(2) DSV_GRAM(3) DSV_GRAM(4) DSV_GRAM(5)
    DSV_GRAM(6) DSV_GRAM(7) DSV_GRAM(8) DSV_GRAM(9) DSV_GRAM(10)
    default: return hipErrorInvalidValue;
  }
#undef DSV_GRAM
  return hipGetLastError();
}

template <typename TC, typename TO>
hipError_t rescale_dispatch(int64_t r, int l, const TC *C, int64_t ldc, const double *W, int64_t ldw,
                            int c, TO *Out, int64_t ldo, const int32_t *done, const TC *R,
                            const double *alpha, hipStream_t st) {
  const int LTO = (c + 15) / 16;
  const int LK = (l + 15) & ~15;
  const int64_t ntiles = (r + 15) / 16;
  // blocks of four wavefronts, each wavefront on its own 16-row tiles
  int64_t g = (ntiles + 3) / 4;
  if (g > 512) g = 512;
  const int grid = (int)(g < 1 ? 1 : g);
#define DSV_RS(LTV)                                                                         \
  case LTV: {                                                                               \
    const size_t shm = sizeof(float) * (size_t)LK * (LTV * 16 + 4);                         \
    hipLaunchKernelGGL((k_rescale_mfma<TC, TO, LTV>), dim3(grid), dim3(256), shm, st, r, l, C, ldc, W, \
                       ldw, c, Out, ldo, done, R, alpha);                                   \
    break;                                                                                  \
  }
  switch (LTO) {
    DSV_RS(1) DSV_RS(2) DSV_RS(3) DSV_RS(4) DSV_RS(5)
    DSV_RS(6) DSV_RS(7) DSV_RS(8) DSV_RS(9) DSV_RS(10)
    default: return hipErrorInvalidValue;
  }
#undef DSV_RS
  return hipGetLastError();
}

}  // namespace

int gram_blocks(int64_t r, int l) {
  (void)l;
  int64_t nb = (r + 63) / 64;
  if (nb > 512) nb = 512;
  if (nb < 1) nb = 1;
  return (int)nb;
}
size_t gram_partial_elems(int nblocks, int l) {
  const int LT = (l + 15) / 16 < 2 ? 2 : (l + 15) / 16;
  return (size_t)nblocks * (size_t)(LT * (LT + 1) / 2) * 256;
}

hipError_t launch_gram(int64_t r, int l, const void *C, int64_t ldc, int cdtype, double *partial,
                       int nblocks, double *G, const int32_t *done, hipStream_t st, int32_t *snap) {
  if (l < 1 || l > kMaxL) return hipErrorInvalidValue;
  if (cdtype == 0) return gram_dispatch<float>(r, l, (const float *)C, ldc, partial, nblocks, G, done, st, snap);
  if (cdtype == 1) return gram_dispatch<double>(r, l, (const double *)C, ldc, partial, nblocks, G, done, st, snap);
  return gram_dispatch<bf16>(r, l, (const bf16 *)C, ldc, partial, nblocks, G, done, st, snap);
}

hipError_t launch_rescale(int64_t r, int l, const void *C, int64_t ldc, int cdtype, const double *W,
                          int64_t ldw, int c, void *Out, int64_t ldo, int odtype, const int32_t *done,
                          hipStream_t st, const void *R, const double *alpha) {
  if (R && !alpha) return hipErrorInvalidValue;
  if (l < 1 || l > kMaxL || c < 1 || c > kMaxL || r == 0) return r == 0 ? hipSuccess : hipErrorInvalidValue;
  static bool attr_done = false;
  if (!attr_done) {
    // allow the MFMA rescale to use up to 160 KB of LDS
#define DSV_ATTR(TC, TO, L) \
  hipFuncSetAttribute((const void *)k_rescale_mfma<TC, TO, L>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
#define DSV_ATTR_ALL(TC, TO) \
  DSV_ATTR(TC, TO, 1) DSV_ATTR(TC, TO, 2) DSV_ATTR(TC, TO, 3) DSV_ATTR(TC, TO, 4) DSV_ATTR(TC, TO, 5) \
  DSV_ATTR(TC, TO, 6) DSV_ATTR(TC, TO, 7) DSV_ATTR(TC, TO, 8) DSV_ATTR(TC, TO, 9) DSV_ATTR(TC, TO, 10)
    DSV_ATTR_ALL(float, float)
    DSV_ATTR_ALL(float, bf16)
    DSV_ATTR_ALL(bf16, float)
#undef DSV_ATTR_ALL
#undef DSV_ATTR
    attr_done = true;
  }
  if (odtype == 1) {
    const int g = grid_for(r * ldo, 256, 16384);
    if (cdtype == 1)
      hipLaunchKernelGGL(k_rescale_f64<double>, dim3(g), dim3(256), 0, st, r, l, (const double *)C, ldc, W, ldw,
                         c, (double *)Out, ldo, done, (const double *)R, alpha);
    else if (cdtype == 0)
      hipLaunchKernelGGL(k_rescale_f64<float>, dim3(g), dim3(256), 0, st, r, l, (const float *)C, ldc, W, ldw, c,
                         (double *)Out, ldo, done, (const float *)R, alpha);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (cdtype == 0 && odtype == 0)
    return rescale_dispatch<float, float>(r, l, (const float *)C, ldc, W, ldw, c, (float *)Out, ldo, done,
                                          (const float *)R, alpha, st);
  if (cdtype == 0 && odtype == 2)
    return rescale_dispatch<float, bf16>(r, l, (const float *)C, ldc, W, ldw, c, (bf16 *)Out, ldo, done,
                                         (const float *)R, alpha, st);
  if (cdtype == 2 && odtype == 0)
    return rescale_dispatch<bf16, float>(r, l, (const bf16 *)C, ldc, W, ldw, c, (float *)Out, ldo, done,
                                         (const bf16 *)R, alpha, st);
  return hipErrorInvalidValue;
}

hipError_t launch_sign_fix(int64_t rowsV, int64_t rowsU, int k, void *V, int64_t ldv, void *U,
                           int64_t ldu, int dtype, void *pmax_v, void *pidx_v, int nblk,
                           hipStream_t st) {
  double *pmax = static_cast<double *>(pmax_v);
  int64_t *pidx = static_cast<int64_t *>(pidx_v);
  float *sgn = reinterpret_cast<float *>(pidx + (int64_t)nblk * k);  // k floats after the indices
  if (k < 1 || k > 256) return hipErrorInvalidValue;
  const int ga = grid_for((rowsV + rowsU) * k, 256, 4096);
  if (dtype == 1) {
    hipLaunchKernelGGL(k_sign_partial<double>, dim3(nblk), dim3(256), 0, st, rowsV, k, (const double *)V, ldv,
                       pmax, pidx);
    hipLaunchKernelGGL(k_sign_select<double>, dim3(k), dim3(256), 0, st, k, (const double *)V, ldv, pmax, pidx,
                       nblk, sgn);
    hipLaunchKernelGGL(k_sign_apply<double>, dim3(ga), dim3(256), 0, st, rowsV, rowsU, k, (double *)V, ldv,
                       (double *)U, ldu, sgn);
  } else {
    hipLaunchKernelGGL(k_sign_partial<float>, dim3(nblk), dim3(256), 0, st, rowsV, k, (const float *)V, ldv,
                       pmax, pidx);
    hipLaunchKernelGGL(k_sign_select<float>, dim3(k), dim3(256), 0, st, k, (const float *)V, ldv, pmax, pidx,
                       nblk, sgn);
    hipLaunchKernelGGL(k_sign_apply<float>, dim3(ga), dim3(256), 0, st, rowsV, rowsU, k, (float *)V, ldv,
                       (float *)U, ldu, sgn);
  }
  return hipGetLastError();
}

hipError_t launch_copy2d(const void *in, int64_t ldi, int idtype, void *out, int64_t ldo, int odtype,
                         int64_t rows, int cols, hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  const int g = grid_for(rows * cols, 256, 16384);
#define DSV_CP(TI, TO) \
  hipLaunchKernelGGL((k_copy2d<TI, TO>), dim3(g), dim3(256), 0, st, (const TI *)in, ldi, (TO *)out, ldo, rows, cols)
  if (idtype == 0 && odtype == 0) DSV_CP(float, float);
  else if (idtype == 0 && odtype == 1) DSV_CP(float, double);
  else if (idtype == 1 && odtype == 0) DSV_CP(double, float);
  else if (idtype == 1 && odtype == 1) DSV_CP(double, double);
  else return hipErrorInvalidValue;
#undef DSV_CP
  return hipGetLastError();
}

hipError_t launch_convert(const void *in, int idtype, void *out, int odtype, int64_t n, hipStream_t st) {
  return launch_copy2d(in, 1, idtype, out, 1, odtype, n, 1, st);
}

// ------------------------------------------------------------------ small FP64 products
// C (m x n) = op(A) B with op(A) = A (m x kk, lda) or A^T (A kk x m, lda),
// B kk x n (ldb); one thread per entry, sums in index order.
// 16 x 16 output tiles, the inner dimension staged through LDS in tiles of 16.
__global__ __launch_bounds__(256) void k_small_gemm(int m, int n, int kk, const double *__restrict__ A, int lda,
                                                    int transA, const double *__restrict__ B, int ldb,
                                                    double *__restrict__ C, int ldc) {
  __shared__ double As[16][17], Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  double s = 0.0;
  for (int t0 = 0; t0 < kk; t0 += 16) {
    // As[ty][tx] = op(A)(blockIdx.y*16 + ty, t0 + tx); Bs[ty][tx] = B(t0 + ty, j)
    const int ai = blockIdx.y * 16 + ty, at = t0 + tx;
    double av = 0.0;
    if (ai < m && at < kk) av = transA ? A[(int64_t)at * lda + ai] : A[(int64_t)ai * lda + at];
    As[ty][tx] = av;
    const int bt = t0 + ty;
    Bs[ty][tx] = (bt < kk && j < n) ? B[(int64_t)bt * ldb + j] : 0.0;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16; ++t) s = fma(As[ty][t], Bs[t][tx], s);
    __syncthreads();
  }
  if (i < m && j < n) C[(int64_t)i * ldc + j] = s;
}

hipError_t launch_small_gemm(int m, int n, int kk, const double *A, int lda, int transA, const double *B, int ldb,
                             double *C, int ldc, hipStream_t st) {
  if (m < 1 || n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_small_gemm, dim3((n + 15) / 16, (m + 15) / 16), dim3(256), 0, st, m, n, kk, A, lda, transA, B,
                     ldb, C, ldc);
  return hipGetLastError();
}

// Signs of the columns of V (the entry of largest magnitude made positive,
// lowest row on ties), applied to V and to the columns of the small FP64
// matrix P (the weights that form U from its block).
hipError_t launch_sign_fold(int64_t rowsV, int k, void *V, int64_t ldv, int dtype, double *P, int prow, int ldp,
                            void *pmax_v, void *pidx_v, int nblk, hipStream_t st) {
  double *pmax = static_cast<double *>(pmax_v);
  int64_t *pidx = static_cast<int64_t *>(pidx_v);
  float *sgn = reinterpret_cast<float *>(pidx + (int64_t)nblk * k);
  if (k < 1 || k > 256) return hipErrorInvalidValue;
  const int ga = grid_for(rowsV * k, 256, 4096);
  if (dtype == 1) {
    hipLaunchKernelGGL(k_sign_partial<double>, dim3(nblk), dim3(256), 0, st, rowsV, k, (const double *)V, ldv,
                       pmax, pidx);
    hipLaunchKernelGGL(k_sign_select<double>, dim3(k), dim3(256), 0, st, k, (const double *)V, ldv, pmax, pidx,
                       nblk, sgn);
    hipLaunchKernelGGL(k_sign_cols<double>, dim3(ga), dim3(256), 0, st, rowsV, k, (double *)V, ldv, sgn);
  } else {
    hipLaunchKernelGGL(k_sign_partial<float>, dim3(nblk), dim3(256), 0, st, rowsV, k, (const float *)V, ldv,
                       pmax, pidx);
    hipLaunchKernelGGL(k_sign_select<float>, dim3(k), dim3(256), 0, st, k, (const float *)V, ldv, pmax, pidx,
                       nblk, sgn);
    hipLaunchKernelGGL(k_sign_cols<float>, dim3(ga), dim3(256), 0, st, rowsV, k, (float *)V, ldv, sgn);
  }
  hipLaunchKernelGGL(k_sign_small, dim3((prow * k + 255) / 256), dim3(256), 0, st, prow, k, P, ldp, sgn);
  return hipGetLastError();
}

}  // namespace dsv
