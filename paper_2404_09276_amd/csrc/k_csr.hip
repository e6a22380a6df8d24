// Sparse-structure kernels: CSR validation, the explicit CSR of A^T used by
// the transposed products of Alg. 5 (steps 2 and 4), and the row-split plan
// of the SpMM.  All integer work; results are independent of scheduling.
//
// CSR(A^T) build (a stable sort by column):
//   1. validation: one thread per nonzero finds its row by binary search in
//      the row pointer, checks the column (range, strictly increasing in the
//      row) and the value (finite), and records its row;
//   2. the library's stable LSD radix sort (k_sort.hip) of the column
//      indices (only the bits that column numbers below n use) carrying, for
//      FP32 values, the entry's row and value packed in 8 bytes (for FP64
//      values, the nonzero index): every column of A then lists its nonzeros
//      in their CSR order, i.e. by increasing row, with no per-column sort
//      and no atomics on the columns (a Zipf matrix sends a tenth of its
//      nonzeros to its first column);
//   3. one thread per entry writes its row and value (FP64: gathers them by
//      the nonzero index), one thread per column finds where the column
//      starts in the sorted keys.
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
constexpr int kValChunk = 8;  // consecutive nonzeros per thread

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
    // a wavefront takes 64 kValChunk consecutive nonzeros, lane L the ones at
    // L, L + 64, ... (coalesced reads and writes): one binary search for the
    // first, then a walk along the row pointer (a binary search again after
    // more than 64 rows, so runs of empty rows stay cheap); with a
    // malformed row pointer the rows found may be wrong, but the flag above
    // is then set and they are never used
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = t0 - lane;  // first thread of this wavefront
    for (int64_t cbeg = wave0 * kValChunk; cbeg < nnz; cbeg += stride * kValChunk) {
      const int64_t efirst = cbeg + lane;
      if (efirst >= nnz) break;
      // the columns (and each one's predecessor) and values of the lane's
      // nonzeros: all loads issued before any is used (clamped indices,
      // unconditional), then one wait
      int32_t cc[kValChunk], cp[kValChunk];
      double vv[kValChunk];
#pragma unroll
      for (int k = 0; k < kValChunk; ++k) {
        const int64_t e = efirst + 64 * k < nnz ? efirst + 64 * k : nnz - 1;
        cc[k] = col[e];
        cp[k] = col[e > 0 ? e - 1 : 0];
        vv[k] = (double)val[e];
      }
#pragma unroll
      for (int k = 0; k < kValChunk; ++k) asm volatile("" : "+v"(cc[k]), "+v"(cp[k]), "+v"(vv[k]));
      // one binary search per wavefront (its first nonzero, a uniform
      // value: scalar loads); each lane then walks to its own row
      const int64_t cb = ((int64_t)__builtin_amdgcn_readfirstlane((int)(cbeg >> 32)) << 32) |
                         (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)cbeg);
      int64_t r = row_of(rp, m, cb);
      int64_t rbeg = rp[r], rend = rp[r + 1];
#pragma unroll
      for (int k = 0; k < kValChunk; ++k) {
        const int64_t e = efirst + 64 * k;
        if (e >= nnz) break;
        int steps = 0;
        while (e >= rend && r + 1 < m && steps < 64) {
          ++r;
          rbeg = rend;
          rend = rp[r + 1];
          ++steps;
        }
        if (e >= rend) {
          r = row_of(rp, m, e);
          rbeg = rp[r];
          rend = rp[r + 1];
        }
        const int32_t c = cc[k];
        rowidx[e] = (int32_t)r;
        if (c < 0 || (int64_t)c >= n)
          bad = 1;
        else if (e > 0 && e > rbeg && cp[k] >= c)
          bad = 1;
        if (!(vv[k] - vv[k] == 0.0)) nonfinite = 1;
      }
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

// The same gather straight into the degree-ordered structure: sorted entry p
// (column j = keys[p] of A, source nonzero src[p]) goes to row inv_c[j] of
// the permuted A^T at its offset inside column j, with its row r of A
// renumbered inv_r[r].
template <typename TV>
__global__ __launch_bounds__(256) void k_tgather_perm(int64_t nnz, const int32_t *__restrict__ src,
                                                      const uint32_t *__restrict__ keys,
                                                      const int32_t *__restrict__ rowidx,
                                                      const TV *__restrict__ val, const int64_t *__restrict__ rowT,
                                                      const int32_t *__restrict__ inv_r,
                                                      const int32_t *__restrict__ inv_c,
                                                      const int64_t *__restrict__ rp_new,
                                                      int32_t *__restrict__ colT, TV *__restrict__ valT) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
    const int64_t j = (int64_t)keys[p];
    const int32_t s = src[p];
    const int64_t pos = rp_new[inv_c[j]] + (p - rowT[j]);
    colT[pos] = inv_r[rowidx[s]];
    valT[pos] = val[s];
  }
}

// Sorted entry p with its packed (row, value): straight to position p of
// CSR(A^T), or, with the degree order, to row inv_c[j] of the permuted A^T
// at its offset inside column j = keys[p], the row renumbered inv_r[r].
__global__ __launch_bounds__(256) void k_tscatter_packed(int64_t nnz, const uint64_t *__restrict__ rv,
                                                         const uint32_t *__restrict__ keys,
                                                         const int64_t *__restrict__ rowT,
                                                         const int32_t *__restrict__ inv_r,
                                                         const int32_t *__restrict__ inv_c,
                                                         const int64_t *__restrict__ rp_new,
                                                         int32_t *__restrict__ colT, float *__restrict__ valT) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) {
    const uint64_t w = rv[p];
    const int32_t r = (int32_t)(uint32_t)w;
    int64_t pos = p;
    int32_t c = r;
    if (inv_r) {
      const int64_t j = (int64_t)keys[p];
      pos = rp_new[inv_c[j]] + (p - rowT[j]);
      c = inv_r[r];
    }
    colT[pos] = c;
    valT[pos] = __uint_as_float((uint32_t)(w >> 32));
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

// ------------------------------------------------------------------ degree order
// Locality order of the operator: rows (and, on the transposed structure,
// columns) by non-increasing number of nonzeros, ties by index.  Solving
// P_r A P_c^T instead of A leaves the singular values unchanged and permutes
// U and V by P_r and P_c; the products then gather the panel rows of the
// dense columns from one compact region of memory.

// Sort key of row i: its length (a stable descending sort lists long rows
// first and keeps index order in ties).
__global__ __launch_bounds__(256) void k_degree_keys(int64_t R, const int64_t *__restrict__ rp,
                                                     uint32_t *__restrict__ key) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < R; i += stride)
    key[i] = (uint32_t)(rp[i + 1] - rp[i]);
}

// inv[perm[i]] = i, and the row lengths in the new order.
__global__ __launch_bounds__(256) void k_perm_invert(int64_t R, const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ perm, int32_t *__restrict__ inv,
                                                     int64_t *__restrict__ len) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < R; i += stride) {
    const int32_t o = perm[i];
    inv[o] = (int32_t)i;
    len[i] = rp[o + 1] - rp[o];
  }
}

// Entry e of row r moves to row inv_r[r] of the permuted structure, at the
// same offset inside the row; its column c becomes inv_c[c].
template <typename TV, typename TR>
__global__ __launch_bounds__(256) void k_permute_entries(int64_t nnz, const int64_t *__restrict__ rp,
                                                         const TR *__restrict__ row_of,
                                                         const int32_t *__restrict__ col,
                                                         const TV *__restrict__ val,
                                                         const int32_t *__restrict__ inv_r,
                                                         const int32_t *__restrict__ inv_c,
                                                         const int64_t *__restrict__ rp_new,
                                                         int32_t *__restrict__ col_new, TV *__restrict__ val_new) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
    const int64_t r = (int64_t)row_of[e];
    const int64_t pos = rp_new[inv_r[r]] + (e - rp[r]);
    col_new[pos] = inv_c[col[e]];
    val_new[pos] = val[e];
  }
}

// The sizes the host needs to launch the products, in one place for one copy.
__global__ void k_plan_sizes(const int64_t *__restrict__ endM, const int64_t *__restrict__ endT,
                             const int32_t *__restrict__ nlM, const int32_t *__restrict__ nlT,
                             const int32_t *__restrict__ hM, const int32_t *__restrict__ hT,
                             int64_t *__restrict__ out) {
  if (threadIdx.x == 0) {
    out[0] = *endM;
    out[1] = *endT;
    out[2] = *nlM;
    out[3] = *nlT;
    out[4] = hM ? *hM : 0;
    out[5] = hT ? *hT : 0;
  }
}

unsigned key_bits(int64_t n) {
  unsigned b = 1;
  while (b < 31 && ((int64_t)1 << b) < n) ++b;
  return b;
}

// ------------------------------------------------------------------ SpMM plan
// Long rows are cut at column-slab boundaries and then into pieces of at most
// long_row nonzeros; the products run the chunks slab by slab, so the panel
// rows every compute unit gathers at a time come from one slab, which stays
// in each XCD's L2.  Each chunk writes its own partial slot, and the slots of
// a row are summed in slot order, so the results do not depend on the order
// the chunks run in.

// first position in col[lo, hi) whose column is >= key (columns sorted)
__device__ __forceinline__ int64_t lower_col(const int32_t *__restrict__ col, int64_t lo, int64_t hi, int64_t key) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)col[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Rows below *head (the dense head, longer than long_row) get no chunks:
// the product's head kernels write them.
__global__ __launch_bounds__(256) void k_plan_count(int64_t R, const int64_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col, int32_t long_row,
                                                    int slab_log2, int64_t *__restrict__ nch,
                                                    const int32_t *__restrict__ head) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t h = head ? *head : 0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R; r += stride) {
    const int64_t b = rp[r], e = rp[r + 1], len = e - b;
    if (len <= long_row || r < h) {
      nch[r] = 0;
      continue;
    }
    if (slab_log2 >= 31) {
      nch[r] = (len + long_row - 1) / long_row;
      continue;
    }
    int64_t cnt = 0;
    for (int64_t pos = b; pos < e;) {
      const int64_t s = (int64_t)col[pos] >> slab_log2;
      const int64_t q = lower_col(col, pos, e, (s + 1) << slab_log2);
      cnt += (q - pos + long_row - 1) / long_row;
      pos = q;
    }
    nch[r] = cnt;
  }
}

__global__ __launch_bounds__(256) void k_plan_fill(int64_t R, const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col, int32_t long_row,
                                                   int slab_log2, const int64_t *__restrict__ off,
                                                   ChunkTask *__restrict__ tasks, int32_t *__restrict__ tslab,
                                                   LongRow *__restrict__ longs, int32_t *__restrict__ nlong) {
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
    int64_t t = off[r];
    for (int64_t pos = b; pos < e;) {
      const int64_t s = slab_log2 >= 31 ? 0 : (int64_t)col[pos] >> slab_log2;
      const int64_t q = slab_log2 >= 31 ? e : lower_col(col, pos, e, (s + 1) << slab_log2);
      for (int64_t c0 = pos; c0 < q; c0 += long_row, ++t) {
        ChunkTask ct;
        ct.begin = c0;
        ct.len = (int32_t)(c0 + long_row < q ? long_row : q - c0);
        ct.slot = (int32_t)t;
        tasks[t] = ct;
        tslab[t] = (int32_t)s;
      }
      pos = q;
    }
  }
}

// chunks per slab (integer atomics: the counts do not depend on their order)
// (slabs past the last one, which only a caller's short column count can
// produce, join the last slab: the order is a matter of speed only)
__global__ __launch_bounds__(256) void k_plan_slab_hist(int nslabs, const int64_t *__restrict__ n_chunks,
                                                        const int32_t *__restrict__ tslab,
                                                        int32_t *__restrict__ cnt) {
  const int64_t n = *n_chunks;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
    atomicAdd(&cnt[min(tslab[t], nslabs - 1)], 1);
}

// exclusive scan of the nslabs counts, in place (one workgroup)
__global__ __launch_bounds__(1024) void k_plan_slab_scan(int nslabs, int32_t *__restrict__ cnt) {
  __shared__ int32_t part[1024];
  constexpr int kPer = (kMaxSlabs + 1023) / 1024;
  const int tid = threadIdx.x;
  int32_t v[kPer];
  int32_t sum = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int i = tid * kPer + q;
    v[q] = i < nslabs ? cnt[i] : 0;
    sum += v[q];
  }
  part[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int32_t x = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += x;
    __syncthreads();
  }
  int32_t run = part[tid] - sum;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int i = tid * kPer + q;
    if (i < nslabs) cnt[i] = run;
    run += v[q];
  }
}

// chunk t to the next free place of its slab (the order inside a slab is
// free: every chunk writes its own slot)
__global__ __launch_bounds__(256) void k_plan_slab_place(int nslabs, const int64_t *__restrict__ n_chunks,
                                                         const ChunkTask *__restrict__ tasks,
                                                         const int32_t *__restrict__ tslab,
                                                         const int32_t *__restrict__ start,
                                                         int32_t *__restrict__ fill,
                                                         ChunkTask *__restrict__ order) {
  const int64_t n = *n_chunks;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int32_t s = min(tslab[t], nslabs - 1);
    order[start[s] + atomicAdd(&fill[s], 1)] = tasks[t];
  }
}

// one grid row per range
__global__ __launch_bounds__(256) void k_zero_ranges(ZeroRanges z) {
  const int r = blockIdx.y;
  int32_t *p = z.p[r];
  const int64_t n = z.n[r];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
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
  const int64_t chunks = (nnz + kValChunk - 1) / kValChunk;
  const int64_t work = chunks > m ? chunks : m;
  const int g = grid_for(work, 256, 16384);
  if (dtype == 1)
    hipLaunchKernelGGL(k_validate<double>, dim3(g), dim3(256), 0, st, m, n, nnz, rp, col,
                       (const double *)val, rowidx, flags);
  else
    hipLaunchKernelGGL(k_validate<float>, dim3(g), dim3(256), 0, st, m, n, nnz, rp, col,
                       (const float *)val, rowidx, flags);
  return hipGetLastError();
}

// Workspace: sorted keys, the sorted payload (8 bytes per entry: packed row
// and FP32 value, or the FP64 path's 4-byte nonzero index), the sort's
// temporary storage.
size_t tws_keys_bytes(size_t cnt) { return (4 * (cnt + 64) + 255) / 256 * 256; }
size_t tws_payload_bytes(size_t cnt) { return (8 * (cnt + 64) + 255) / 256 * 256; }

size_t transpose_ws_bytes(int64_t n, int64_t nnz) {
  const size_t cnt = nnz > 0 ? (size_t)nnz : 1;
  return tws_keys_bytes(cnt) + tws_payload_bytes(cnt) + sort_ws_bytes((int64_t)cnt, key_bits(n), 8) + 256;
}

hipError_t launch_transpose_keys(int64_t n, int64_t nnz, const int32_t *col, int64_t *rowT, void *ws,
                                 size_t ws_bytes, hipStream_t st, const int32_t *rowidx, const void *val,
                                 int dtype) {
  const size_t cnt = nnz > 0 ? (size_t)nnz : 1;
  uint32_t *keys = (uint32_t *)ws;
  char *payload = (char *)ws + tws_keys_bytes(cnt);
  void *tmp = (void *)(payload + tws_payload_bytes(cnt));
  size_t tmp_bytes = ws_bytes - tws_keys_bytes(cnt) - tws_payload_bytes(cnt);
  if (nnz > 0) {
    // validated columns are in [0, n): sort on their low bits only
    const hipError_t e =
        dtype == 0 ? sort_keys_packed(nnz, (const uint32_t *)col, rowidx, (const float *)val, keys,
                                      (uint64_t *)payload, key_bits(n), tmp, tmp_bytes, st)
                   : sort_keys_index(nnz, (const uint32_t *)col, keys, (int32_t *)payload, key_bits(n), false, tmp,
                                     tmp_bytes, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tbounds, dim3(grid_for(n + 1, 256, 16384)), dim3(256), 0, st, n, nnz, keys, rowT);
  return hipGetLastError();
}

hipError_t launch_transpose_gather(int64_t nnz, const int32_t *rowidx, const void *val, int dtype, const void *ws,
                                   int32_t *colT, void *valT, hipStream_t st, const int64_t *rowT,
                                   const int32_t *inv_r, const int32_t *inv_c, const int64_t *rp_new) {
  if (nnz == 0) return hipSuccess;
  const size_t cnt = (size_t)nnz;
  const uint32_t *keys = (const uint32_t *)ws;
  const char *payload = (const char *)ws + tws_keys_bytes(cnt);
  const int32_t *src = (const int32_t *)payload;
  const int g = grid_for(nnz, 256, 16384);
  if (dtype == 0) {
    hipLaunchKernelGGL(k_tscatter_packed, dim3(g), dim3(256), 0, st, nnz, (const uint64_t *)payload, keys, rowT,
                       inv_r, inv_c, rp_new, colT, (float *)valT);
  } else if (inv_r) {
    if (dtype == 1)
      hipLaunchKernelGGL(k_tgather_perm<double>, dim3(g), dim3(256), 0, st, nnz, src, keys, rowidx,
                         (const double *)val, rowT, inv_r, inv_c, rp_new, colT, (double *)valT);
    else
      hipLaunchKernelGGL(k_tgather_perm<float>, dim3(g), dim3(256), 0, st, nnz, src, keys, rowidx,
                         (const float *)val, rowT, inv_r, inv_c, rp_new, colT, (float *)valT);
  } else {
    if (dtype == 1)
      hipLaunchKernelGGL(k_tgather<double>, dim3(g), dim3(256), 0, st, nnz, src, rowidx, (const double *)val,
                         colT, (double *)valT);
    else
      hipLaunchKernelGGL(k_tgather<float>, dim3(g), dim3(256), 0, st, nnz, src, rowidx, (const float *)val,
                         colT, (float *)valT);
  }
  return hipGetLastError();
}

hipError_t launch_transpose(int64_t n, int64_t nnz, const int32_t *col, const int32_t *rowidx, const void *val,
                            int dtype, int64_t *rowT, int32_t *colT, void *valT, void *ws, size_t ws_bytes,
                            hipStream_t st) {
  const hipError_t e = launch_transpose_keys(n, nnz, col, rowT, ws, ws_bytes, st, rowidx, val, dtype);
  if (e != hipSuccess) return e;
  return launch_transpose_gather(nnz, rowidx, val, dtype, ws, colT, valT, st);
}

size_t degree_order_ws_bytes(int64_t R) {
  const size_t cnt = R > 0 ? (size_t)R : 1;
  return 2 * 4 * (cnt + 64) + 8 * (cnt + 64) + sort_ws_bytes((int64_t)cnt, 32u, 4) + 256;
}

hipError_t launch_degree_order(int64_t R, const int64_t *rp, int64_t max_len, int32_t *perm, int32_t *inv,
                               int64_t *rp_new, void *ws, size_t ws_bytes, int64_t *scan_tmp, hipStream_t st) {
  if (R == 0) return hipMemsetAsync(rp_new, 0, sizeof(int64_t), st);
  const size_t cnt = (size_t)R;
  uint32_t *keys = (uint32_t *)ws;
  uint32_t *keys_sorted = keys + cnt + 64;
  int64_t *len = (int64_t *)(keys_sorted + cnt + 64);
  void *tmp = (void *)(len + cnt + 64);
  size_t tmp_bytes = ws_bytes - 2 * 4 * (cnt + 64) - 8 * (cnt + 64);
  const int g = grid_for(R, 256, 16384);
  hipLaunchKernelGGL(k_degree_keys, dim3(g), dim3(256), 0, st, R, rp, keys);
  // lengths are at most max_len: sort on the bits that can be set
  hipError_t e = sort_keys_index(R, keys, keys_sorted, perm, key_bits(max_len + 1), true, tmp, tmp_bytes, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_perm_invert, dim3(g), dim3(256), 0, st, R, rp, perm, inv, len);
  return launch_scan_i64(len, R, rp_new, scan_tmp, st);
}

hipError_t launch_permute_entries(int64_t nnz, const int64_t *rp, const int32_t *row_of, int row_of_unsigned,
                                  const int32_t *col, const void *val, int dtype, const int32_t *inv_r,
                                  const int32_t *inv_c, const int64_t *rp_new, int32_t *col_new, void *val_new,
                                  hipStream_t st) {
  if (nnz == 0) return hipSuccess;
  const int g = grid_for(nnz, 256, 16384);
#define DSV_PERM(TV, TR)                                                                                   \
  hipLaunchKernelGGL((k_permute_entries<TV, TR>), dim3(g), dim3(256), 0, st, nnz, rp, (const TR *)row_of, \
                     col, (const TV *)val, inv_r, inv_c, rp_new, col_new, (TV *)val_new)
  if (dtype == 1) {
    if (row_of_unsigned) DSV_PERM(double, uint32_t); else DSV_PERM(double, int32_t);
  } else {
    if (row_of_unsigned) DSV_PERM(float, uint32_t); else DSV_PERM(float, int32_t);
  }
#undef DSV_PERM
  return hipGetLastError();
}

hipError_t launch_plan_sizes(const int64_t *endM, const int64_t *endT, const int32_t *nlM, const int32_t *nlT,
                             const int32_t *hM, const int32_t *hT, int64_t *out, hipStream_t st) {
  hipLaunchKernelGGL(k_plan_sizes, dim3(1), dim3(64), 0, st, endM, endT, nlM, nlT, hM, hT, out);
  return hipGetLastError();
}

hipError_t launch_plan_count(int64_t R, const int64_t *rp, const int32_t *col, int32_t long_row, int slab_log2,
                             int64_t *nch, hipStream_t st, const int32_t *head) {
  if (R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_count, dim3(grid_for(R, 256, 16384)), dim3(256), 0, st, R, rp, col, long_row, slab_log2,
                     nch, head);
  return hipGetLastError();
}

hipError_t launch_plan_fill(int64_t R, const int64_t *rp, const int32_t *col, int32_t long_row, int slab_log2,
                            const int64_t *off, ChunkTask *tasks, int32_t *tslab, LongRow *longs, int32_t *nlong,
                            hipStream_t st) {
  if (R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_fill, dim3(grid_for(R, 256, 16384)), dim3(256), 0, st, R, rp, col, long_row, slab_log2,
                     off, tasks, tslab, longs, nlong);
  return hipGetLastError();
}

hipError_t launch_plan_order(int nslabs, const int64_t *n_chunks, const ChunkTask *tasks, const int32_t *tslab,
                             int32_t *slab_cnt, ChunkTask *order, hipStream_t st) {
  if (nslabs < 1 || nslabs > kMaxSlabs) return hipErrorInvalidValue;
  int32_t *cnt = slab_cnt, *fill = slab_cnt + kMaxSlabs + 1;
  hipLaunchKernelGGL(k_plan_slab_hist, dim3(256), dim3(256), 0, st, nslabs, n_chunks, tslab, cnt);
  hipLaunchKernelGGL(k_plan_slab_scan, dim3(1), dim3(1024), 0, st, nslabs, cnt);
  hipLaunchKernelGGL(k_plan_slab_place, dim3(256), dim3(256), 0, st, nslabs, n_chunks, tasks, tslab,
                     (const int32_t *)cnt, fill, order);
  return hipGetLastError();
}

hipError_t launch_zero_ranges(const ZeroRanges &z, hipStream_t st) {
  if (z.count < 0 || z.count > kMaxZeroRanges) return hipErrorInvalidValue;
  if (z.count == 0) return hipSuccess;
  int64_t most = 1;
  for (int i = 0; i < z.count; ++i) {
    if (z.n[i] < 0 || (z.n[i] > 0 && !z.p[i])) return hipErrorInvalidValue;
    if (z.n[i] > most) most = z.n[i];
  }
  const int64_t gx = grid_for(most, 256, 64);
  hipLaunchKernelGGL(k_zero_ranges, dim3((unsigned)gx, (unsigned)z.count), dim3(256), 0, st, z);
  return hipGetLastError();
}

hipError_t launch_fill_zero_i32(int32_t *p, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace dsv
