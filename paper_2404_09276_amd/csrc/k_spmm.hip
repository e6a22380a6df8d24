// Sparse x tall-skinny dense products of the power pass (Alg. 5 steps 2, 4
// and 9): Y = A X and, with the shift fused in the epilogue,
// C = A^T Y - alpha Q.
//
// Layout: the dense panels are row-major with a leading dimension that is a
// multiple of 8 elements, so each row starts 16-byte aligned.  A group of
// G = ld / V lanes owns one sparse row, V = 16 / sizeof(panel element) (4
// FP32, 2 FP64, 8 BF16), and every lane keeps V accumulators: for each
// nonzero the group gathers one full panel row with one 16-byte load per
// lane, so a gathered row is a coalesced read of ld elements.  A wavefront
// holds 64 / G groups.  The (column, value) pairs of a row are read
// cooperatively by the group and broadcast lane to lane, so eight gathers
// per lane are in flight at once.
//
// Load balance (power-law degrees): rows with more than long_row nonzeros
// are cut into chunks (at column-slab boundaries, then into pieces of at most
// long_row); each chunk is an independent task writing its own partial row,
// and a second kernel sums the chunks of each long row in column order.
// Nothing depends on scheduling order, so results repeat bit for bit.  Tasks
// are numbered chunks first, then rows, so the heavy chunks start early; the
// chunks run slab by slab, so the panel rows gathered at a time come from one
// slab that each XCD's L2 holds.
//
// Gathers in flight: when the panel X is known to span less than 2 GB, the
// gathers are raw buffer loads whose range check returns zero for offsets
// past the panel.  Every step then issues U gathers unconditionally, the
// slots past the row's end pointing out of range (no memory traffic, value
// zero), so short rows and the last nonzeros of a row keep U gathers in
// flight instead of one at a time, and the (column, value) pairs of the next
// G nonzeros are fetched while the current ones are gathered.
//
// The kernels read the solver's done flag first (a device-scope load: the
// flag may be set by the eigensolver running beside them) and exit when the
// PVE check has already stopped the iteration (speculatively launched
// passes, and the transposed product of the last pass).
#include <type_traits>

#include "common.h"

namespace dsv {

namespace {

// Raw buffer resource (word 3 of the descriptor for gfx950 raw buffers) and
// an offset past any panel of at most kBufMaxBytes (plus up to 3 words per
// lane, still below 2^31): such loads return zero.
constexpr int kBufRsrcWord3 = 0x00020000;
constexpr uint32_t kBufPastEnd = 0x7FFFFF00u;
constexpr int64_t kBufMaxBytes = 0x7FFFF000;

// One lane's V panel elements (V * sizeof(TX) bytes, whole 16-byte words)
// at byte offset off of the buffer, converted to the accumulator type.
template <typename TX, typename TA, int V>
__device__ __forceinline__ void buf_gather(__amdgpu_buffer_rsrc_t r, uint32_t off, TA *o) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  constexpr int W = 16 / (int)sizeof(TX);  // elements per 16-byte word
  static_assert(V % W == 0, "whole 16-byte words per lane");
#pragma unroll
  for (int j = 0; j < V / W; ++j) {
    const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(off + 16u * j), 0, 0);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
    vec16<TX, TA>::unpack(w, o + j * W);
  }
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup b to XCD b % 8).
// Renumbered so that each XCD takes runs of kXcdRun consecutive tasks
// (runs dealt to the XCDs in turn, so the heavy chunks at the head of the
// task list still spread over all of them): the rows an XCD works on at a
// time are neighbours, and in the batched form they belong to the same few
// matrices, whose panel rows then stay in that XCD's L2 instead of every L2
// holding every matrix in flight.  A permutation of the tasks (the last,
// partial round keeps its order): each task still writes its own rows or
// slots, so results do not change.  (Batched form: 48.1 -> 43.8 ms a batch
// of 512 matrices.)
__device__ __forceinline__ int64_t xcd_block() {
  constexpr int64_t kXcds = 8, kXcdRun = 32, S = kXcds * kXcdRun;
  const int64_t nb = gridDim.x, b = blockIdx.x;
  if (b >= (nb / S) * S) return b;
  const int64_t w = b % S;
  return b - w + (w % kXcds) * kXcdRun + w / kXcds;
}

template <typename TX> struct acc_of {
  using type = float;
};
template <> struct acc_of<double> {
  using type = double;
};

// FP32 panels, one 16-byte vector per lane: at least 6 wavefronts per SIMD
// (at most 80 VGPRs; the compiler's own choice, 81, allowed 5), so more
// gathers are in flight per CU: 1 % faster products on the power-law
// benchmark matrix (8 wavefronts would need spills).  The other lane widths
// and types would spill under that cap and keep the compiler's choice.
template <typename TX, int V> constexpr int spmm_min_waves() {
  return std::is_same<TX, float>::value && V == 4 ? 6 : 1;
}

template <typename TV, typename TX, typename TY, typename TA, bool SHIFT, int V>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(spmm_min_waves<TX, V>()))) void k_spmm(
    int64_t R, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
    const TV *__restrict__ val, const TX *__restrict__ X, int64_t ldx, TY *__restrict__ Y,
    int64_t ldy, int G, int64_t n_chunks, const ChunkTask *__restrict__ tasks,
    TA *__restrict__ partial, int64_t ldp, int32_t long_row, const TX *__restrict__ Q, int64_t ldq,
    const double *__restrict__ alpha, const int32_t *__restrict__ done,
    const int32_t *__restrict__ rowmat, const SolverState *__restrict__ bstate, int32_t xbytes) {
  if (done && __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rpw = kWave / G;
  const int sub = lane / G, cl = lane - sub * G;
  if (sub >= rpw) return;
  // the batched operator (rowmat) takes the XCD runs; for one matrix they
  // made both products 8-14 % slower on the power-law benchmark matrix
  const int64_t blk = rowmat ? xcd_block() : (int64_t)blockIdx.x;
  const int64_t g = (blk * 4 + wave) * rpw + sub;
  int64_t b, e, row = -1, slot = 0;
  const double *alpha_row = alpha;
  if (g < n_chunks) {
    const ChunkTask t = tasks[g];
    b = t.begin;
    e = t.begin + t.len;
    slot = t.slot;
  } else {
    row = g - n_chunks;
    if (row >= R) return;
    b = rp[row];
    e = rp[row + 1];
    if (e - b > long_row) return;  // handled by its chunks
    if (rowmat) {
      // batched operator: the row's matrix may have stopped before this
      // pass (pass-start snapshot); its own shift
      const SolverState &ms = bstate[rowmat[row]];
      if (ms.pass_skip) return;
      alpha_row = &ms.alpha;
    }
  }
  TA acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = (TA)0;
  const TX *xb = X + cl * V;
  const int src0 = sub * G;  // first lane of this group
  // The group reads up to G (column, value) pairs with one coalesced load,
  // then broadcasts them lane to lane, so the gathers of U consecutive
  // nonzeros are independent and in flight together.
  constexpr int U = 8;
  if (xbytes > 0) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void *)X, 0, xbytes, kBufRsrcWord3);
    const uint32_t row_b = (uint32_t)(ldx * (int64_t)sizeof(TX));
    const uint32_t lane_b = (uint32_t)(cl * V * (int)sizeof(TX));
    // clamped (valid) pair index: the loads are unconditional, the slots past
    // the end are masked where the pairs are used
    auto pair_at = [&](int64_t i) -> int64_t { return i < e ? i : e - 1; };
    int32_t myc = 0;
    TA myv = (TA)0;
    if (b < e) {
      const int64_t i0 = pair_at(b + cl);
      myc = col[i0];
      myv = (TA)val[i0];
    }
    for (int64_t base = b; base < e; base += G) {
      const int64_t inext = pair_at(base + G + cl);
      const int32_t nc = col[inext];
      const TV nv = val[inext];
      const int cnt = (int)((e - base) < G ? (e - base) : G);
      for (int t = 0; t < cnt; t += U) {
        uint32_t off[U];
        TA v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t c = __shfl(myc, src0 + t + u, 64);
          const TA w = __shfl(myv, src0 + t + u, 64);
          const bool ok = t + u < cnt;
          off[u] = ok ? (uint32_t)c * row_b + lane_b : kBufPastEnd;
          v[u] = ok ? w : (TA)0;
        }
        TA x[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) buf_gather<TX, TA, V>(rs, off[u], x[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int i = 0; i < V; ++i) acc[i] = fma(v[u], x[u][i], acc[i]);
      }
      myc = nc;
      myv = (TA)nv;
    }
  } else
  for (int64_t base = b; base < e; base += G) {
    const int64_t idx = base + cl;
    int32_t myc = 0;
    TA myv = (TA)0;
    if (idx < e) {
      myc = col[idx];
      myv = (TA)val[idx];
    }
    const int cnt = (int)((e - base) < G ? (e - base) : G);
    int t = 0;
    for (; t + U <= cnt; t += U) {
      int32_t c[U];
      TA v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        c[u] = __shfl(myc, src0 + t + u, 64);
        v[u] = __shfl(myv, src0 + t + u, 64);
      }
      TA x[U][V];
#pragma unroll
      for (int u = 0; u < U; ++u) load_n<TX, TA, V>(xb + (int64_t)c[u] * ldx, x[u]);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < V; ++i) acc[i] = fma(v[u], x[u][i], acc[i]);
    }
    for (; t < cnt; ++t) {
      const int32_t c0 = __shfl(myc, src0 + t, 64);
      const TA v0 = __shfl(myv, src0 + t, 64);
      TA x0[V];
      load_n<TX, TA, V>(xb + (int64_t)c0 * ldx, x0);
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] = fma(v0, x0[i], acc[i]);
    }
  }
  if (row < 0) {
    store_n<TA, TA, V>(partial + slot * ldp + cl * V, acc);
    return;
  }
  if constexpr (SHIFT) {
    const TA a = (TA)(*alpha_row);
    TA q[V];
    load_n<TX, TA, V>(Q + row * ldq + cl * V, q);
#pragma unroll
    for (int i = 0; i < V; ++i) acc[i] = acc[i] - a * q[i];
  }
  store_n<TY, TA, V>(Y + row * ldy + cl * V, acc);
}

// One workgroup per long row: its NG = 256 / G lane groups split the chunk
// partials round-robin (group k takes chunks k, k + NG, ...), each summing
// its share in chunk order with eight loads in flight, and the group sums are
// then added in group order (fixed, so results repeat bit for bit).  A row
// with hundreds of chunks no longer waits on one group's chain of loads.
template <typename TX, typename TY, typename TA, bool SHIFT, int V>
__global__ __launch_bounds__(256) void k_spmm_long(
    int64_t n_long, const LongRow *__restrict__ longs, const TA *__restrict__ partial, int64_t ldp,
    TY *__restrict__ Y, int64_t ldy, int G, const TX *__restrict__ Q, int64_t ldq,
    const double *__restrict__ alpha, const int32_t *__restrict__ done,
    const int32_t *__restrict__ rowmat, const SolverState *__restrict__ bstate) {
  if (done && __hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ TA red[256 * V];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rpw = kWave / G;
  const int sub = lane / G, cl = lane - sub * G;
  const int NG = 4 * rpw;                // lane groups in the workgroup
  const int k = wave * rpw + sub;        // this lane's group
  const int64_t g = blockIdx.x;
  if (g >= n_long) return;
  const LongRow lr = longs[g];
  const double *alpha_row = alpha;
  if (rowmat) {
    const SolverState &ms = bstate[rowmat[lr.row]];
    if (ms.pass_skip) return;
    alpha_row = &ms.alpha;
  }
  TA acc[V];
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = (TA)0;
  if (sub < rpw) {
    const TA *pb = partial + lr.first * ldp + cl * V;
    int64_t c = k;
    for (; c + 7 * (int64_t)NG < lr.nch; c += 8 * (int64_t)NG) {
      TA p[8][V];
#pragma unroll
      for (int u = 0; u < 8; ++u) load_n<TA, TA, V>(pb + (c + u * (int64_t)NG) * ldp, p[u]);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int i = 0; i < V; ++i) acc[i] += p[u][i];
    }
    for (; c < lr.nch; c += NG) {
      TA p[V];
      load_n<TA, TA, V>(pb + c * ldp, p);
#pragma unroll
      for (int i = 0; i < V; ++i) acc[i] += p[i];
    }
#pragma unroll
    for (int i = 0; i < V; ++i) red[(k * G + cl) * V + i] = acc[i];
  }
  __syncthreads();
  if (wave != 0 || sub != 0) return;
  // group 0's lanes add the group sums in group order
#pragma unroll
  for (int i = 0; i < V; ++i) acc[i] = red[cl * V + i];
  for (int q = 1; q < NG; ++q)
#pragma unroll
    for (int i = 0; i < V; ++i) acc[i] += red[(q * G + cl) * V + i];
  if constexpr (SHIFT) {
    const TA a = (TA)(*alpha_row);
    TA qv[V];
    load_n<TX, TA, V>(Q + lr.row * ldq + cl * V, qv);
#pragma unroll
    for (int i = 0; i < V; ++i) acc[i] = acc[i] - a * qv[i];
  }
  store_n<TY, TA, V>(Y + lr.row * ldy + cl * V, acc);
}

template <typename TV, typename TX, typename TY, int V>
hipError_t run_spmm_v(int64_t R, const int64_t *rp, const int32_t *col, const void *val, const void *X,
                      int64_t ldx, void *Y, int64_t ldy, int ld_cols, int64_t n_chunks,
                      const ChunkTask *tasks, int64_t n_long, const LongRow *longs, void *partial,
                      int32_t long_row, const void *Q, int64_t ldq, const double *alpha,
                      const int32_t *done, const int32_t *rowmat, const SolverState *bstate,
                      hipStream_t st, int64_t xrows) {
  using TA = typename acc_of<TX>::type;
  const int G = ld_cols / V;
  const int64_t xb = xrows * ldx * (int64_t)sizeof(TX);
  const int32_t xbytes = (xrows > 0 && xb <= kBufMaxBytes) ? (int32_t)xb : 0;
  if (G < 1 || G > kWave || ld_cols % V) return hipErrorInvalidValue;
  const int rpw = kWave / G;
  const int64_t subs = n_chunks + R;
  const int64_t blocks = (subs + 4 * rpw - 1) / (4 * rpw);
  const bool shift = alpha != nullptr;
  if (blocks > 0) {
    if (shift)
      hipLaunchKernelGGL((k_spmm<TV, TX, TY, TA, true, V>), dim3((unsigned)blocks), dim3(256), 0, st, R, rp,
                         col, (const TV *)val, (const TX *)X, ldx, (TY *)Y, ldy, G, n_chunks, tasks,
                         (TA *)partial, (int64_t)ld_cols, long_row, (const TX *)Q, ldq, alpha, done,
                         rowmat, bstate, xbytes);
    else
      hipLaunchKernelGGL((k_spmm<TV, TX, TY, TA, false, V>), dim3((unsigned)blocks), dim3(256), 0, st, R, rp,
                         col, (const TV *)val, (const TX *)X, ldx, (TY *)Y, ldy, G, n_chunks, tasks,
                         (TA *)partial, (int64_t)ld_cols, long_row, (const TX *)Q, ldq, alpha, done,
                         rowmat, bstate, xbytes);
  }
  if (n_long > 0) {
    const int64_t lb = n_long;  // one workgroup per long row
    if (shift)
      hipLaunchKernelGGL((k_spmm_long<TX, TY, TA, true, V>), dim3((unsigned)lb), dim3(256), 0, st, n_long,
                         longs, (const TA *)partial, (int64_t)ld_cols, (TY *)Y, ldy, G, (const TX *)Q, ldq,
                         alpha, done, rowmat, bstate);
    else
      hipLaunchKernelGGL((k_spmm_long<TX, TY, TA, false, V>), dim3((unsigned)lb), dim3(256), 0, st, n_long,
                         longs, (const TA *)partial, (int64_t)ld_cols, (TY *)Y, ldy, G, (const TX *)Q, ldq,
                         alpha, done, rowmat, bstate);
  }
  return hipGetLastError();
}

// Lane width: one 16-byte vector of the panel type per lane, or two when a
// row would need more than 64 lanes (FP64 panels with l > 128) or when the
// caller asks for it (lane_mult = 2, a tuning knob: half as many lanes per
// row, twice the gathers in flight per lane) and the row splits evenly.
template <typename TV, typename TX, typename TY>
hipError_t run_spmm(int64_t R, const int64_t *rp, const int32_t *col, const void *val, const void *X,
                    int64_t ldx, void *Y, int64_t ldy, int ld_cols, int64_t n_chunks,
                    const ChunkTask *tasks, int64_t n_long, const LongRow *longs, void *partial,
                    int32_t long_row, int lane_mult, const void *Q, int64_t ldq, const double *alpha,
                    const int32_t *done, const int32_t *rowmat, const SolverState *bstate,
                    hipStream_t st, int64_t xrows) {
  using TA = typename acc_of<TX>::type;
  constexpr int V = vec16<TX, TA>::N;
  if (ld_cols / V <= kWave && !(lane_mult == 2 && ld_cols % (2 * V) == 0))
    return run_spmm_v<TV, TX, TY, V>(R, rp, col, val, X, ldx, Y, ldy, ld_cols, n_chunks, tasks, n_long, longs,
                                     partial, long_row, Q, ldq, alpha, done, rowmat, bstate, st, xrows);
  return run_spmm_v<TV, TX, TY, 2 * V>(R, rp, col, val, X, ldx, Y, ldy, ld_cols, n_chunks, tasks, n_long,
                                       longs, partial, long_row, Q, ldq, alpha, done, rowmat, bstate, st, xrows);
}

}  // namespace

hipError_t launch_spmm(int64_t R, const int64_t *rp, const int32_t *col, const void *val, int vdtype,
                       const void *X, int64_t ldx, int xdtype, void *Y, int64_t ldy, int ydtype,
                       int ld_cols, int64_t n_chunks, const ChunkTask *tasks, int64_t n_long,
                       const LongRow *longs, void *partial, int32_t long_row, int lane_mult,
                       const void *Q, int64_t ldq, const double *alpha, const int32_t *done, hipStream_t st,
                       const int32_t *rowmat, const SolverState *bstate, int64_t xrows) {
  // supported combinations: (values, X/Q, Y) = (f32, f32, f32), (f64, f64, f64),
  // (f32, bf16, bf16), (f32, bf16, f32)
  if (xdtype == 0 && ydtype == 0 && vdtype == 0)
    return run_spmm<float, float, float>(R, rp, col, val, X, ldx, Y, ldy, ld_cols, n_chunks, tasks, n_long,
                                         longs, partial, long_row, lane_mult, Q, ldq, alpha, done, rowmat,
                                         bstate, st, xrows);
  if (xdtype == 1 && ydtype == 1 && vdtype == 1)
    return run_spmm<double, double, double>(R, rp, col, val, X, ldx, Y, ldy, ld_cols, n_chunks, tasks,
                                            n_long, longs, partial, long_row, lane_mult, Q, ldq, alpha, done,
                                            rowmat, bstate, st, xrows);
  if (xdtype == 2 && ydtype == 2 && vdtype == 0)
    return run_spmm<float, bf16, bf16>(R, rp, col, val, X, ldx, Y, ldy, ld_cols, n_chunks, tasks, n_long,
                                       longs, partial, long_row, lane_mult, Q, ldq, alpha, done, rowmat, bstate,
                                       st, xrows);
  if (xdtype == 2 && ydtype == 0 && vdtype == 0)
    return run_spmm<float, bf16, float>(R, rp, col, val, X, ldx, Y, ldy, ld_cols, n_chunks, tasks, n_long,
                                        longs, partial, long_row, lane_mult, Q, ldq, alpha, done, rowmat, bstate,
                                        st, xrows);
  return hipErrorInvalidValue;
}

}  // namespace dsv
