// Sparse-structure kernels: CSR validation, the explicit CSR of A^T used by
// the transposed products of Alg. 5 (steps 2 and 4), and the row-split plan
// of the SpMM.  All integer work; results are independent of scheduling.
//
// CSR(A^T) build (counting sort by column, made deterministic):
//   1. validate + count: one thread per nonzero finds its row by binary
//      search, checks the column (range, strictly increasing in the row) and
//      the value (finite), and counts the column with an integer atomic;
//   2. exclusive scan of the counts -> row pointer of A^T;
//   3. scatter: each nonzero takes a slot in its column with an atomic
//      cursor (order inside a column still arbitrary);
//   4. per-column ordering by row: columns of length <= 64 rank their
//      entries inside one wavefront, up to 2048 with a bitonic sort in LDS,
//      longer ones by ranking against a bitmap of the rows (prefix popcount),
//      so every column lists its rows in increasing order.
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

// ------------------------------------------------------------------ hot-column table
// Power-law matrices have columns shared by a large fraction of the rows, and
// one global atomic per nonzero on such a column serialises.  Each block
// therefore keeps an LDS hash table (column -> count) for the columns of its
// contiguous range of nonzeros and flushes one global atomic per distinct
// column; entries that find no free slot after a few probes use the global
// atomic directly.
constexpr int kHashSlots = 4096;
constexpr int kElemPerThread = 16;
constexpr int kElemPerBlock = 256 * kElemPerThread;

__device__ __forceinline__ int hash_slot(int32_t c) {
  return (int)(((uint32_t)c * 2654435761u) >> 20) & (kHashSlots - 1);
}

// Returns the slot holding column c (inserting it), or -1 when the probes fail.
__device__ __forceinline__ int hash_insert(int32_t *keys, int32_t c) {
  int h = hash_slot(c);
#pragma unroll 1
  for (int probe = 0; probe < 8; ++probe) {
    const int32_t k = keys[h];
    if (k == c) return h;
    if (k == -1) {
      const int32_t old = atomicCAS(keys + h, -1, c);
      if (old == -1 || old == c) return h;
    }
    h = (h + 1) & (kHashSlots - 1);
  }
  return -1;
}

// Row of nonzero e: the last r in [0, m) with rp[r] <= e (in bounds whatever rp holds).
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
                                                  int64_t *__restrict__ colcnt,
                                                  int32_t *__restrict__ rowidx,
                                                  int32_t *__restrict__ flags) {
  __shared__ int32_t keys[kHashSlots];
  __shared__ int32_t cnts[kHashSlots];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // row pointer: starts at 0, nondecreasing, ends at nnz
  for (int64_t r = t0; r < m; r += (int64_t)gridDim.x * blockDim.x) {
    if (rp[r] > rp[r + 1]) atomicOr(flags, 1);
  }
  if (t0 == 0 && (rp[0] != 0 || rp[m] != nnz)) atomicOr(flags, 1);
  if (m == 0) return;
  for (int64_t base = (int64_t)blockIdx.x * kElemPerBlock; base < nnz;
       base += (int64_t)gridDim.x * kElemPerBlock) {
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) {
      keys[i] = -1;
      cnts[i] = 0;
    }
    __syncthreads();
    for (int i = 0; i < kElemPerThread; ++i) {
      const int64_t e = base + (int64_t)i * blockDim.x + threadIdx.x;
      if (e >= nnz) break;
      const int64_t r = row_of(rp, m, e);
      const int32_t c = col[e];
      rowidx[e] = (int32_t)r;
      if (c < 0 || (int64_t)c >= n) {
        atomicOr(flags, 1);
        continue;
      }
      if (e > rp[r] && e > 0 && col[e - 1] >= c) atomicOr(flags, 1);
      const double v = (double)val[e];
      if (!(v - v == 0.0)) atomicOr(flags, 2);
      const int h = hash_insert(keys, c);
      if (h >= 0) atomicAdd(cnts + h, 1);
      else atomicAdd((unsigned long long *)(colcnt + c), 1ull);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) {
      if (keys[i] >= 0) atomicAdd((unsigned long long *)(colcnt + keys[i]), (unsigned long long)cnts[i]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ transpose
// Slot assignment in CSR(A^T): per block, the hot columns reserve one range
// with a single global atomic and hand out positions inside it from LDS.
__global__ __launch_bounds__(256) void k_scatter(int64_t nnz, const int32_t *__restrict__ col,
                                                 const int32_t *__restrict__ rowidx,
                                                 const int64_t *__restrict__ rowT,
                                                 int32_t *__restrict__ cursor,
                                                 int32_t *__restrict__ tmp_row,
                                                 int32_t *__restrict__ tmp_src) {
  __shared__ int32_t keys[kHashSlots];
  __shared__ int32_t cnts[kHashSlots];
  for (int64_t base = (int64_t)blockIdx.x * kElemPerBlock; base < nnz;
       base += (int64_t)gridDim.x * kElemPerBlock) {
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) {
      keys[i] = -1;
      cnts[i] = 0;
    }
    __syncthreads();
    int16_t slot[kElemPerThread];
#pragma unroll
    for (int i = 0; i < kElemPerThread; ++i) {
      const int64_t e = base + (int64_t)i * blockDim.x + threadIdx.x;
      slot[i] = -1;
      if (e < nnz) {
        const int h = hash_insert(keys, col[e]);
        slot[i] = (int16_t)h;
        if (h >= 0) atomicAdd(cnts + h, 1);
      }
    }
    __syncthreads();
    // reserve a contiguous range per hot column; the count becomes the range base
    for (int i = threadIdx.x; i < kHashSlots; i += blockDim.x) {
      if (keys[i] >= 0) cnts[i] = atomicAdd(cursor + keys[i], cnts[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kElemPerThread; ++i) {
      const int64_t e = base + (int64_t)i * blockDim.x + threadIdx.x;
      if (e < nnz) {
        const int32_t c = col[e];
        const int h = slot[i];
        const int32_t within = h >= 0 ? atomicAdd(cnts + h, 1) : atomicAdd(cursor + c, 1);
        const int64_t pos = rowT[c] + within;
        tmp_row[pos] = rowidx[e];
        tmp_src[pos] = (int32_t)e;
      }
    }
    __syncthreads();
  }
}

constexpr int kSmallSeg = 64;
constexpr int kMedSeg = 2048;

template <typename TV>
__global__ __launch_bounds__(256) void k_classify(int64_t n, const int64_t *__restrict__ rowT,
                                                  const int32_t *__restrict__ tmp_row,
                                                  const int32_t *__restrict__ tmp_src,
                                                  const TV *__restrict__ val,
                                                  int32_t *__restrict__ colT, TV *__restrict__ valT,
                                                  int32_t *__restrict__ lists,
                                                  int32_t *__restrict__ counts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  // the loop bound is rounded up to whole waves so every lane joins the ballots
  const int64_t nr = (n + 63) / 64 * 64;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nr; c += stride) {
    int cls = -1;
    if (c < n) {
      const int64_t b = rowT[c], L = rowT[c + 1] - b;
      if (L == 1) {
        colT[b] = tmp_row[b];
        valT[b] = val[tmp_src[b]];
      } else if (L > 1) {
        cls = L <= kSmallSeg ? 0 : (L <= kMedSeg ? 1 : 2);
      }
    }
    // one atomic per class per wavefront
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint64_t mask = __ballot(cls == k);
      if (!mask) continue;
      const int leader = __ffsll((unsigned long long)mask) - 1;
      int32_t base = 0;
      if (lane == leader) base = atomicAdd(counts + k, __popcll(mask));
      base = __shfl(base, leader, 64);
      if (cls == k) {
        const int rank = __popcll(mask & ((1ull << lane) - 1ull));
        lists[(int64_t)k * n + base + rank] = (int32_t)c;
      }
    }
  }
}

// Columns with 2..64 entries: one wavefront each, lane i ranks entry i.
template <typename TV>
__global__ __launch_bounds__(256) void k_sort_small(int32_t count, const int32_t *__restrict__ list,
                                                    const int64_t *__restrict__ rowT,
                                                    const int32_t *__restrict__ tmp_row,
                                                    const int32_t *__restrict__ tmp_src,
                                                    const TV *__restrict__ val,
                                                    int32_t *__restrict__ colT,
                                                    TV *__restrict__ valT) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= count) return;
  const int32_t c = list[w];
  const int64_t b = rowT[c];
  const int L = (int)(rowT[c + 1] - b);
  const int32_t myrow = lane < L ? tmp_row[b + lane] : 0x7fffffff;
  int rank = 0;
  for (int j = 0; j < L; ++j) {
    const int32_t other = __shfl(myrow, j, 64);
    rank += other < myrow;
  }
  if (lane < L) {
    colT[b + rank] = myrow;
    valT[b + rank] = val[tmp_src[b + lane]];
  }
}

// Columns with 65..2048 entries: bitonic sort of (row << 32 | slot) in LDS.
template <typename TV>
__global__ __launch_bounds__(256) void k_sort_medium(int32_t count, const int32_t *__restrict__ list,
                                                     const int64_t *__restrict__ rowT,
                                                     const int32_t *__restrict__ tmp_row,
                                                     const int32_t *__restrict__ tmp_src,
                                                     const TV *__restrict__ val,
                                                     int32_t *__restrict__ colT,
                                                     TV *__restrict__ valT) {
  __shared__ uint64_t key[kMedSeg];
  for (int64_t w = blockIdx.x; w < count; w += gridDim.x) {
    const int32_t c = list[w];
    const int64_t b = rowT[c];
    const int L = (int)(rowT[c + 1] - b);
    int P = 128;
    while (P < L) P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x)
      key[i] = i < L ? (((uint64_t)(uint32_t)tmp_row[b + i]) << 32) | (uint32_t)i : ~0ull;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = threadIdx.x; i < P; i += blockDim.x) {
          const int j = i ^ stride;
          if (j > i) {
            const bool up = (i & size) == 0;
            const uint64_t a = key[i], bb = key[j];
            if ((a > bb) == up) {
              key[i] = bb;
              key[j] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
      const uint64_t kk = key[i];
      colT[b + i] = (int32_t)(kk >> 32);
      valT[b + i] = val[tmp_src[b + (uint32_t)kk]];
    }
    __syncthreads();
  }
}

// Columns with more than 2048 entries: rank each row against a bitmap of the
// column's rows kept in LDS, one window of kWinRows rows at a time
// (prefix popcounts give the rank inside the window).
constexpr int kWinWords = 8192;              // 32 KB bitmap + 32 KB prefix
constexpr int64_t kWinRows = (int64_t)kWinWords * 32;

template <typename TV>
__global__ __launch_bounds__(1024) void k_sort_large(int32_t count, const int32_t *__restrict__ list,
                                                     int64_t m, const int64_t *__restrict__ rowT,
                                                     const int32_t *__restrict__ tmp_row,
                                                     const int32_t *__restrict__ tmp_src,
                                                     const TV *__restrict__ val,
                                                     int32_t *__restrict__ colT,
                                                     TV *__restrict__ valT,
                                                     uint32_t *__restrict__ unused_ws,
                                                     int32_t *__restrict__ unused_ws2) {
  (void)unused_ws;
  (void)unused_ws2;
  __shared__ uint32_t bm[kWinWords];
  __shared__ int32_t pf[kWinWords];
  __shared__ int64_t sh[40];
  constexpr int per = kWinWords / 1024;
  for (int64_t w = blockIdx.x; w < count; w += gridDim.x) {
    const int32_t c = list[w];
    const int64_t b = rowT[c];
    const int64_t L = rowT[c + 1] - b;
    int64_t done_rows = 0;  // entries ranked in earlier windows
    for (int64_t r0 = 0; r0 < m; r0 += kWinRows) {
      for (int i = threadIdx.x; i < kWinWords; i += 1024) bm[i] = 0u;
      __syncthreads();
      for (int64_t i = threadIdx.x; i < L; i += 1024) {
        const int64_t r = (int64_t)tmp_row[b + i] - r0;
        if (r >= 0 && r < kWinRows) atomicOr(bm + (r >> 5), 1u << (r & 31));
      }
      __syncthreads();
      const int w0 = threadIdx.x * per;
      int64_t local = 0;
#pragma unroll
      for (int i = 0; i < per; ++i) local += __popc(bm[w0 + i]);
      int64_t tot;
      int64_t ex = block_excl_scan(local, sh, tot);
#pragma unroll
      for (int i = 0; i < per; ++i) {
        pf[w0 + i] = (int32_t)ex;
        ex += __popc(bm[w0 + i]);
      }
      __syncthreads();
      for (int64_t i = threadIdx.x; i < L; i += 1024) {
        const int64_t r = (int64_t)tmp_row[b + i] - r0;
        if (r >= 0 && r < kWinRows) {
          const uint32_t word = bm[r >> 5];
          const int64_t rank = done_rows + pf[r >> 5] + __popc(word & ((1u << (r & 31)) - 1u));
          colT[b + rank] = (int32_t)(r + r0);
          valT[b + rank] = val[tmp_src[b + i]];
        }
      }
      done_rows += tot;
      __syncthreads();
    }
  }
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
                           const void *val, int dtype, int64_t *colcnt, int32_t *rowidx,
                           int32_t *flags, hipStream_t st) {
  int64_t gb = (nnz + kElemPerBlock - 1) / kElemPerBlock;
  if (gb < (m + 255) / 256) gb = (m + 255) / 256;
  const int g = (int)(gb < 1 ? 1 : (gb > 65536 ? 65536 : gb));
  if (dtype == 1)
    hipLaunchKernelGGL(k_validate<double>, dim3(g), dim3(256), 0, st, m, n, nnz, rp, col,
                       (const double *)val, colcnt, rowidx, flags);
  else
    hipLaunchKernelGGL(k_validate<float>, dim3(g), dim3(256), 0, st, m, n, nnz, rp, col,
                       (const float *)val, colcnt, rowidx, flags);
  return hipGetLastError();
}

hipError_t launch_transpose_scatter(int64_t nnz, const int32_t *col, const int32_t *rowidx,
                                    const int64_t *rowT, int32_t *cursor, int32_t *tmp_row,
                                    int32_t *tmp_src, hipStream_t st) {
  if (nnz == 0) return hipSuccess;
  const int64_t gbs = (nnz + kElemPerBlock - 1) / kElemPerBlock;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)(gbs > 65536 ? 65536 : gbs)), dim3(256), 0, st, nnz, col, rowidx,
                     rowT, cursor, tmp_row, tmp_src);
  return hipGetLastError();
}

hipError_t launch_transpose_classify(int64_t n, const int64_t *rowT, const int32_t *tmp_row,
                                     const int32_t *tmp_src, const void *val, int dtype,
                                     int32_t *colT, void *valT, int32_t *lists, int32_t *counts,
                                     hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int g = grid_for(n, 256, 16384);
  if (dtype == 1)
    hipLaunchKernelGGL(k_classify<double>, dim3(g), dim3(256), 0, st, n, rowT, tmp_row, tmp_src,
                       (const double *)val, colT, (double *)valT, lists, counts);
  else
    hipLaunchKernelGGL(k_classify<float>, dim3(g), dim3(256), 0, st, n, rowT, tmp_row, tmp_src,
                       (const float *)val, colT, (float *)valT, lists, counts);
  return hipGetLastError();
}

int64_t transpose_bitmap_words(int64_t m) { return (m + 31) / 32; }

hipError_t launch_transpose_sort(int64_t m, int64_t n, const int64_t *rowT, const int32_t *tmp_row,
                                 const int32_t *tmp_src, const void *val, int dtype, int32_t *colT,
                                 void *valT, const int32_t *lists, const int32_t *counts_host,
                                 uint32_t *bitmap_ws, int32_t *prefix_ws, int nblk_large,
                                 hipStream_t st) {
  const int32_t cs = counts_host[0], cm = counts_host[1], cl = counts_host[2];
  if (dtype == 1) {
    if (cs) hipLaunchKernelGGL(k_sort_small<double>, dim3((cs + 3) / 4), dim3(256), 0, st, cs, lists, rowT,
                               tmp_row, tmp_src, (const double *)val, colT, (double *)valT);
    if (cm) hipLaunchKernelGGL(k_sort_medium<double>, dim3(cm < 4096 ? cm : 4096), dim3(256), 0, st, cm,
                               lists + n, rowT, tmp_row, tmp_src, (const double *)val, colT, (double *)valT);
    if (cl) hipLaunchKernelGGL(k_sort_large<double>, dim3(cl < nblk_large ? cl : nblk_large), dim3(1024), 0,
                               st, cl, lists + 2 * n, m, rowT, tmp_row, tmp_src, (const double *)val, colT,
                               (double *)valT, bitmap_ws, prefix_ws);
  } else {
    if (cs) hipLaunchKernelGGL(k_sort_small<float>, dim3((cs + 3) / 4), dim3(256), 0, st, cs, lists, rowT,
                               tmp_row, tmp_src, (const float *)val, colT, (float *)valT);
    if (cm) hipLaunchKernelGGL(k_sort_medium<float>, dim3(cm < 4096 ? cm : 4096), dim3(256), 0, st, cm,
                               lists + n, rowT, tmp_row, tmp_src, (const float *)val, colT, (float *)valT);
    if (cl) hipLaunchKernelGGL(k_sort_large<float>, dim3(cl < nblk_large ? cl : nblk_large), dim3(1024), 0,
                               st, cl, lists + 2 * n, m, rowT, tmp_row, tmp_src, (const float *)val, colT,
                               (float *)valT, bitmap_ws, prefix_ws);
  }
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
