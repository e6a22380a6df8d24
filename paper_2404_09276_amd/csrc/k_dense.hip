// Dense tall-skinny kernels of eigSVD (Alg. 3) and of the final step of
// Alg. 5, plus small utilities.
//
// Gram G = C^T C (Alg. 3 step 1), FP64 accumulation on the FP64 matrix
// cores: the l columns are cut into T = ceil(l/16) tiles and only the
// T(T+1)/2 upper tiles are computed.  The four wavefronts of a block walk the
// same rows of C four at a time, each owning a fixed set of upper tiles: a
// lane loads its element of every column tile straight into a register
// (FP32 and BF16 inputs convert to FP64 exactly), and that register is the A
// or B operand of v_mfma_f64_16x16x4 for every tile in that tile row or
// column.  Every block writes its partial tiles; a second kernel sums the
// partials in block order (deterministic) and mirrors the upper triangle.
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
// Tile t of the upper triangle, numbered row by row: (tile_i, tile_j), i <= j.
constexpr int tile_i(int LT, int t) {
  int I = 0;
  while (t >= LT - I) {
    t -= LT - I;
    ++I;
  }
  return I;
}
constexpr int tile_j(int LT, int t) { return t - (tile_i(LT, t) * (2 * LT - tile_i(LT, t) + 1)) / 2 + tile_i(LT, t); }

// One k-step (4 rows) of the tiles owned by wavefront WV: tiles WV, WV+4, ...
// v[c] holds this lane's element of column tile c (row L/16, column L%16),
// which is its A operand for a tile in row c and its B operand for a tile in
// column c.  Unrolled at compile time so that v and acc stay in registers.
template <int LT, int WV, int I, int TPW>
__device__ __forceinline__ void gram_step(const double (&v)[LT], d4 (&acc)[TPW]) {
  constexpr int t = WV + 4 * I;
  if constexpr (I < TPW && t < LT * (LT + 1) / 2) {
    constexpr int a = tile_i(LT, t), b = tile_j(LT, t);
    double y = v[b];
    // A diagonal tile must not feed the same VGPR pair as both operands (an
    // FP64 MFMA given that returned wrong rows 8-15 on gfx950): make the B
    // copy opaque so it lives in a register of its own.
    if constexpr (a == b) asm volatile("" : "+v"(y));
    acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[a], y, acc[I], 0, 0, 0);
    gram_step<LT, WV, I + 1, TPW>(v, acc);
  }
}

// Raw buffer loads over the block's rows: an offset at or past the end of
// the range reads zero (the hardware range check), so rows past the block
// need no mask.  Word 3 of the descriptor is the gfx9 raw-buffer format.
constexpr int kBufWord3 = 0x00020000;
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, int off, const float *) {
  return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, int off, const double *) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, int off, const bf16 *) {
  return (double)__uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0) << 16);
}

// Rows [row0, row1) of the block, k-steps of 4 rows, loads kept
// kGramPrefetch steps ahead in registers.  Columns past l are zeroed after
// the load (pad columns may hold anything).
constexpr int kGramPrefetch = 4;

template <typename TC, int LT, int WV>
__device__ __forceinline__ void gram_wave(int64_t row0, int64_t row1, int l, const TC *__restrict__ C,
                                          int64_t ldc, double *__restrict__ out) {
  constexpr int NT = LT * (LT + 1) / 2;
  constexpr int TPW = (NT + 3) / 4;
  const int lane = threadIdx.x & 63;
  const int kr = lane >> 4, kc = lane & 15;
  d4 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
  // the range ends at the last element of the block: column l-1 of row row1-1
  const int64_t nbytes = ((row1 - row0 - 1) * ldc + l) * (int64_t)sizeof(TC);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)(C + row0 * ldc), 0, (int)nbytes, kBufWord3);
  bool colok[LT];
#pragma unroll
  for (int c = 0; c < LT; ++c) colok[c] = c * 16 + kc < l;
  const int step_bytes = (int)(4 * ldc * (int64_t)sizeof(TC));
  int off = (int)((kr * ldc + kc) * (int64_t)sizeof(TC));
  double buf[kGramPrefetch][LT];
#pragma unroll
  for (int s = 0; s < kGramPrefetch; ++s) {
#pragma unroll
    for (int c = 0; c < LT; ++c) buf[s][c] = buf_ld(rs, off + c * 16 * (int)sizeof(TC), C);
    off += step_bytes;
  }
  for (int64_t rb = row0; rb < row1; rb += 4 * kGramPrefetch) {
#pragma unroll
    for (int s = 0; s < kGramPrefetch; ++s) {
      double v[LT];
#pragma unroll
      for (int c = 0; c < LT; ++c) v[c] = colok[c] ? buf[s][c] : 0.0;
#pragma unroll
      for (int c = 0; c < LT; ++c) buf[s][c] = buf_ld(rs, off + c * 16 * (int)sizeof(TC), C);
      off += step_bytes;
      gram_step<LT, WV, 0, TPW>(v, acc);
    }
  }
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = WV + 4 * i;
    if (t < NT) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // Move the accumulator through a VGPR before storing: a store that
        // read the FP64 MFMA accumulator registers directly returned stale
        // values for the last rows written by the final MFMA on gfx950.
        double x = acc[i][q];
        asm volatile("" : "+v"(x));
        out[(int64_t)t * 256 + lane * 4 + q] = x;
      }
    }
  }
}

// Block partial of G = C^T C over rows [b * rows_per_block, ...): the four
// wavefronts walk the same rows, each on its own upper tiles, with the MFMA
// operands loaded straight from memory (no LDS, no block barrier).
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
  const int64_t row0 = (int64_t)blockIdx.x * rows_per_block;
  int64_t row1 = row0 + rows_per_block;
  if (row1 > r) row1 = r;
  double *out = partial + (int64_t)blockIdx.x * NT * 256;
  const int wave = threadIdx.x >> 6;
  if (row0 >= row1) {
    for (int i = threadIdx.x; i < NT * 256; i += 256) out[i] = 0.0;
    return;
  }
  switch (wave) {
    case 0: gram_wave<TC, LT, 0>(row0, row1, l, C, ldc, out); break;
    case 1: gram_wave<TC, LT, 1>(row0, row1, l, C, ldc, out); break;
    case 2: gram_wave<TC, LT, 2>(row0, row1, l, C, ldc, out); break;
    default: gram_wave<TC, LT, 3>(row0, row1, l, C, ldc, out); break;
  }
}

// Sum the block partials; write the full symmetric G.  A workgroup owns 32
// consecutive partial elements and eight segments of the blocks: thread
// (s, e) sums blocks [s nb/8, (s+1) nb/8) of element e in block order (the
// 32 elements of a segment are one coalesced read per block), then the
// eight segment sums are added in order s = 0..7 (deterministic).
template <int LT>
__global__ __launch_bounds__(256) void k_gram_reduce(int l, int nblocks, const double *__restrict__ partial,
                                                     double *__restrict__ G,
                                                     const int32_t *__restrict__ done) {
  if (done && *done) return;
  constexpr int NT = LT * (LT + 1) / 2;
  __shared__ double part[8][32];
  const int el = threadIdx.x & 31, seg = threadIdx.x >> 5;
  const int64_t e = (int64_t)blockIdx.x * 32 + el;
  double s = 0.0;
  if (e < (int64_t)NT * 256) {
    const int64_t stride = (int64_t)NT * 256;
    const double *p = partial + e;
    const int per = (nblocks + 7) / 8;
    const int b0 = seg * per;
    const int b1 = b0 + per < nblocks ? b0 + per : nblocks;
    int b = b0;
    for (; b + 3 < b1; b += 4) {
      const double x0 = p[(int64_t)b * stride], x1 = p[(int64_t)(b + 1) * stride];
      const double x2 = p[(int64_t)(b + 2) * stride], x3 = p[(int64_t)(b + 3) * stride];
      s += x0;
      s += x1;
      s += x2;
      s += x3;
    }
    for (; b < b1; ++b) s += p[(int64_t)b * stride];
  }
  part[seg][el] = s;
  __syncthreads();
  if (seg != 0 || e >= (int64_t)NT * 256) return;
  double tot = 0.0;
#pragma unroll
  for (int i = 0; i < 8; ++i) tot += part[i][el];
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
// operand never goes through LDS.  A wavefront's (tile, slab) sequence is
// walked as one stream with the loads two slabs ahead, across tile ends.
// Columns k >= l of C are masked to zero (pad columns may hold anything);
// with R, the input is C - alpha R, formed in FP64 and rounded once.
constexpr int kRescaleThreads = 1024;  // 16 wavefronts share one copy of W

template <typename TC, typename TO, int LTO>
__global__ __launch_bounds__(kRescaleThreads) void k_rescale_mfma(int64_t r, int l, const TC *__restrict__ C,
                                                                  int64_t ldc, const double *__restrict__ W,
                                                                  int64_t ldw, int c, TO *__restrict__ Out,
                                                                  int64_t ldo, const int32_t *__restrict__ done,
                                                                  const TC *__restrict__ R,
                                                                  const double *__restrict__ alpha,
                                                                  const int32_t *__restrict__ row_to) {
  if (done && *done) return;
  constexpr int NW = kRescaleThreads / 64;
  const double a_sh = R ? *alpha : 0.0;
  constexpr int WC = LTO * 16;
  constexpr int SW = WC + 4;
  extern __shared__ float lds[];
  const int LK = (l + 15) & ~15;  // k-slabs of 16
  float *Ws = lds;                // LK x SW
  {
    // Eight independent loads in flight per thread: every load reads a
    // clamped (valid) address unconditionally, and the values pass an
    // opaque copy before the mask, so the compiler cannot sink a load into
    // a branch (which would wait for each load in turn).
    constexpr int kU = 8;
    const int total = LK * WC;
    for (int base = threadIdx.x; base < total; base += kRescaleThreads * kU) {
      double v[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int idx = base + u * kRescaleThreads;
        const int kk = idx / WC, cc = idx - kk * WC;
        v[u] = W[(int64_t)(kk < l ? kk : l - 1) * ldw + (cc < c ? cc : c - 1)];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int idx = base + u * kRescaleThreads;
        const int kk = idx / WC, cc = idx - kk * WC;
        double x = v[u];
        asm volatile("" : "+v"(x));
        if (idx < total) Ws[kk * SW + cc] = (kk < l && cc < c) ? (float)x : 0.0f;
      }
    }
  }
  __syncthreads();
  // the wavefront index is uniform: keep the tile walk in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lr = lane & 15, kq = lane >> 4;  // A row, k quad
  const int64_t ntiles = (r + 15) / 16;
  const int nslab = LK / 16;
  const int64_t tstride = (int64_t)gridDim.x * NW;
  // Raw slab loads, issued ahead of use: the addresses are clamped to valid
  // ones (rows past r are never stored; k >= l is masked at use), and no
  // arithmetic touches the loaded values until they are used, so nothing
  // waits for a load at the point where it is issued.
  struct Slab {
    float4 c, r;
  };
  const TC *Rl = R ? R : C;
  auto load_slab = [&](int64_t tile, int sl) -> Slab {
    int64_t row = tile * 16 + lr;
    if (row >= r) row = r - 1;
    int kb = sl * 16 + 4 * kq;
    if (kb >= l) kb = 0;  // ld is a multiple of 8 and kb of 4: the vector stays inside the row
    Slab x;
    x.c = load4f(C + row * ldc + kb);
    x.r = load4f(Rl + row * ldc + kb);  // without R: a second read of C, ignored
    return x;
  };
  auto advance = [&](int64_t &tile, int &sl) {
    if (++sl == nslab) {
      sl = 0;
      tile += tstride;
    }
  };
  int64_t tile = (int64_t)blockIdx.x * NW + wave;  // slab in use
  int sl = 0;
  int64_t tl = tile;  // next slab to load
  int sll = 0;
  f4 acc[LTO];
#pragma unroll
  for (int J = 0; J < LTO; ++J) acc[J] = f4{0.f, 0.f, 0.f, 0.f};
  // One slab: take the values of b, reload b with the slab three ahead,
  // then the MFMAs; at the end of a tile, store it.  Three buffers used in
  // turn, each reloaded unconditionally (clamped addresses), so no register
  // copy has to wait for a load in flight; past the last tile a step only
  // reloads.
  auto step = [&](Slab &b) {
    const bool live = tile < ntiles;
    const int k0 = sl * 16;
    const float cv[4] = {b.c.x, b.c.y, b.c.z, b.c.w};
    const float rv[4] = {b.r.x, b.r.y, b.r.z, b.r.w};
    float av[4];
#pragma unroll
    for (int s_ = 0; s_ < 4; ++s_) {
      const float v = R ? (float)((double)cv[s_] - a_sh * (double)rv[s_]) : cv[s_];
      av[s_] = k0 + 4 * kq + s_ < l ? v : 0.0f;
    }
    b = load_slab(tl, sll);
    advance(tl, sll);
    if (!live) return;
#pragma unroll
    for (int s_ = 0; s_ < 4; ++s_) {
      const float *bw = Ws + (k0 + 4 * kq + s_) * SW + lr;
#pragma unroll
      for (int J = 0; J < LTO; ++J)
        acc[J] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s_], bw[J * 16], acc[J], 0, 0, 0);
    }
    if (sl == nslab - 1) {
      const int64_t rbase = tile * 16 + 4 * kq;
      int64_t dst[4];  // output rows of this lane's four accumulator rows
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t orow = rbase + q;
        dst[q] = orow < r ? (row_to ? (int64_t)row_to[orow] : orow) : -1;
      }
#pragma unroll
      for (int J = 0; J < LTO; ++J) {
        const int col = J * 16 + lr;
        if (col < ldo) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float v = acc[J][q];
            asm volatile("" : "+v"(v));
            if (dst[q] >= 0) elem<TO>::st(Out + dst[q] * ldo + col, col < c ? v : 0.0f);
          }
        }
        acc[J] = f4{0.f, 0.f, 0.f, 0.f};
      }
      // columns beyond the tiles (ldo > WC) are zero
      if (ldo > WC) {
        for (int q = 0; q < 4; ++q)
          if (dst[q] >= 0)
            for (int64_t cc = WC + lr; cc < ldo; cc += 16) elem<TO>::st(Out + dst[q] * ldo + cc, 0.0f);
      }
    }
    advance(tile, sl);
  };
  Slab b0 = load_slab(tl, sll);
  advance(tl, sll);
  Slab b1 = load_slab(tl, sll);
  advance(tl, sll);
  Slab b2 = load_slab(tl, sll);
  advance(tl, sll);
  while (tile < ntiles) {
    step(b0);
    step(b1);
    step(b2);
  }
}

template <typename TC>
__global__ __launch_bounds__(256) void k_rescale_f64(int64_t r, int l, const TC *__restrict__ C,
                                                     int64_t ldc, const double *__restrict__ W,
                                                     int64_t ldw, int c, double *__restrict__ Out,
                                                     int64_t ldo, const int32_t *__restrict__ done,
                                                     const TC *__restrict__ R,
                                                     const double *__restrict__ alpha,
                                                     const int32_t *__restrict__ row_to) {
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
    Out[(row_to ? (int64_t)row_to[row] : row) * ldo + col] = s;
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
// row_to (optional): input row i goes to output row row_to[i].
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_copy2d(const TI *__restrict__ in, int64_t ldi, TO *__restrict__ out,
                                                int64_t ldo, int64_t rows, int cols,
                                                const int32_t *__restrict__ row_to) {
  const int64_t total = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / cols;
    const int j = (int)(e - i * cols);
    const int64_t io = row_to ? (int64_t)row_to[i] : i;
    elem<TO>::st(out + io * ldo + j, (decltype(elem<TO>::ld(out)))to_d(in[i * ldi + j]));
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
  constexpr int64_t kStep = 4 * kGramPrefetch;  // rows of one unrolled iteration
  const int64_t rpb = ((r + nb - 1) / nb + kStep - 1) / kStep * kStep;
  // byte offsets inside one block's rows (prefetch included) are 32-bit
  if ((rpb + kStep) * ldc * (int64_t)sizeof(TC) >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
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
                            const double *alpha, hipStream_t st, const int32_t *row_to) {
  const int LTO = (c + 15) / 16;
  const int LK = (l + 15) & ~15;
  const int64_t ntiles = (r + 15) / 16;
  // blocks of 16 wavefronts, each wavefront on its own 16-row tiles; one
  // block per CU (the W copy fills most of the LDS)
  constexpr int NW = kRescaleThreads / 64;
  int64_t g = (ntiles + NW - 1) / NW;
  if (g > 256) g = 256;
  const int grid = (int)(g < 1 ? 1 : g);
#define DSV_RS(LTV)                                                                         \
  case LTV: {                                                                               \
    const size_t shm = sizeof(float) * (size_t)LK * (LTV * 16 + 4);                         \
    hipLaunchKernelGGL((k_rescale_mfma<TC, TO, LTV>), dim3(grid), dim3(kRescaleThreads), shm, st, r, l, C, ldc, W, \
                       ldw, c, Out, ldo, done, R, alpha, row_to);                           \
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
                          hipStream_t st, const void *R, const double *alpha, const int32_t *row_to) {
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
                         c, (double *)Out, ldo, done, (const double *)R, alpha, row_to);
    else if (cdtype == 0)
      hipLaunchKernelGGL(k_rescale_f64<float>, dim3(g), dim3(256), 0, st, r, l, (const float *)C, ldc, W, ldw, c,
                         (double *)Out, ldo, done, (const float *)R, alpha, row_to);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (cdtype == 0 && odtype == 0)
    return rescale_dispatch<float, float>(r, l, (const float *)C, ldc, W, ldw, c, (float *)Out, ldo, done,
                                          (const float *)R, alpha, st, row_to);
  if (cdtype == 0 && odtype == 2)
    return rescale_dispatch<float, bf16>(r, l, (const float *)C, ldc, W, ldw, c, (bf16 *)Out, ldo, done,
                                         (const float *)R, alpha, st, row_to);
  if (cdtype == 2 && odtype == 0)
    return rescale_dispatch<bf16, float>(r, l, (const bf16 *)C, ldc, W, ldw, c, (float *)Out, ldo, done,
                                         (const bf16 *)R, alpha, st, row_to);
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

hipError_t launch_copy2d(const void *in, int64_t ldi, int idtype, void *out, int64_t ldo, int odtype, int64_t rows,
                         int cols, hipStream_t st, const int32_t *row_to) {
  if (rows * cols == 0) return hipSuccess;
  const int g = grid_for(rows * cols, 256, 16384);
#define DSV_CP(TI, TO) \
  hipLaunchKernelGGL((k_copy2d<TI, TO>), dim3(g), dim3(256), 0, st, (const TI *)in, ldi, (TO *)out, ldo, rows, cols, \
                     row_to)
  if (idtype == 0 && odtype == 0) DSV_CP(float, float);
  else if (idtype == 0 && odtype == 1) DSV_CP(float, double);
  else if (idtype == 1 && odtype == 0) DSV_CP(double, float);
  else if (idtype == 1 && odtype == 1) DSV_CP(double, double);
  else if (idtype == 0 && odtype == 2) DSV_CP(float, bf16);
  else if (idtype == 1 && odtype == 2) DSV_CP(double, bf16);
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
