// Stable LSD radix sort of 32-bit keys with a 4- or 8-byte payload, for the
// integer setup of the solver: the sort by column that builds CSR(A^T)
// (needed by the transposed products of Alg. 5, steps 2 and 4) and the sorts
// by row and column length of the degree order.
//
// Each pass sorts on one digit of d <= 9 bits (the passes split the key bits
// evenly; 17-bit column numbers take 2 passes, 20-bit ones 3):
//   1. k_digit_hist: per tile of kTile keys, the count of every digit
//      (LDS integer atomics; counts do not depend on their order), stored
//      digit-major: hist[digit * tiles + tile];
//   2. an exclusive scan of hist gives each (digit, tile) its first output
//      position: digits in order, and inside a digit the tiles in order;
//   3. k_digit_scatter: each tile ranks its keys within their digit in input
//      order (stable): rounds of 256 keys, one per thread in input order;
//      inside a wavefront the lanes holding the same digit are found with one
//      ballot per digit bit, the rank is the count of such lanes below, and
//      earlier wavefronts and rounds add their counts through LDS.  The tile
//      is reordered by digit in LDS, then written out in digit runs, so
//      writes of one digit are contiguous.
// Every step is integer work in a fixed order: results are identical run to
// run.  A descending sort ranks the complement of the key's bits.
#include "common.h"

namespace dsv {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kTile = kSortThreads * kSortRounds;  // keys per tile
constexpr int kMaxDigitBits = 9;
constexpr int kMaxDigits = 1 << kMaxDigitBits;

int grid_for(int64_t work, int block, int64_t cap) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// Payload of input position i, first pass.
struct PayIndex {  // the position itself
  __device__ int32_t operator()(int64_t i) const { return (int32_t)i; }
};
struct PayPacked {  // a nonzero's row (low word) and FP32 value bits (high word)
  const int32_t *row;
  const float *val;
  __device__ uint64_t operator()(int64_t i) const {
    return (uint64_t)(uint32_t)row[i] | ((uint64_t)__float_as_uint(val[i]) << 32);
  }
};
template <typename P>
struct PayArray {  // later passes: the previous pass's output
  const P *p;
  __device__ P operator()(int64_t i) const { return p[i]; }
};

__device__ __forceinline__ int digit_of(uint32_t key, int shift, uint32_t mask, bool desc) {
  return (int)(((desc ? ~key : key) >> shift) & mask);
}

__global__ __launch_bounds__(kSortThreads) void k_digit_hist(int64_t n, const uint32_t *__restrict__ keys, int shift,
                                                             int bits, int desc, int64_t tiles,
                                                             int64_t *__restrict__ hist) {
  __shared__ int cnt[kMaxDigits];
  const int D = 1 << bits;
  const uint32_t mask = (uint32_t)D - 1;
  for (int d = threadIdx.x; d < D; d += kSortThreads) cnt[d] = 0;
  __syncthreads();
  const int64_t t = blockIdx.x;
  const int64_t b = t * kTile, e = b + kTile < n ? b + kTile : n;
  for (int64_t i = b + threadIdx.x; i < e; i += kSortThreads) atomicAdd(&cnt[digit_of(keys[i], shift, mask, desc)], 1);
  __syncthreads();
  for (int d = threadIdx.x; d < D; d += kSortThreads) hist[(int64_t)d * tiles + t] = cnt[d];
}

template <typename P, typename Src>
__global__ __launch_bounds__(kSortThreads) void k_digit_scatter(int64_t n, const uint32_t *__restrict__ keys,
                                                                Src src, int shift, int bits, int desc,
                                                                int64_t tiles, const int64_t *__restrict__ start,
                                                                uint32_t *__restrict__ keys_out,
                                                                P *__restrict__ pay_out) {
  __shared__ uint32_t s_key[kTile];
  __shared__ P s_pay[kTile];
  __shared__ int s_run[kMaxDigits];                          // keys of each digit ranked so far
  __shared__ short s_wave[kSortThreads / kWave][kMaxDigits]; // this round's count per wavefront (<= 64)
  __shared__ int s_toff[kMaxDigits];                         // first slot of each digit in the tile
  __shared__ int64_t s_goff[kMaxDigits];                     // first output position of each digit
  __shared__ int s_part[kSortThreads / kWave];
  const int D = 1 << bits;
  const uint32_t mask = (uint32_t)D - 1;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int64_t t = blockIdx.x;
  const int64_t b = t * kTile;
  const int cntT = (int)(b + kTile < n ? kTile : n - b);
  // this tile's digit counts from the scanned histogram, their exclusive
  // scan over digits (the tile-local slots), and the output positions
  int myc[kMaxDigits / kSortThreads];
  int mysum = 0;
#pragma unroll
  for (int q = 0; q < kMaxDigits / kSortThreads; ++q) {
    const int d = tid * (kMaxDigits / kSortThreads) + q;
    int c = 0;
    if (d < D) {
      const int64_t idx = (int64_t)d * tiles + t;
      s_goff[d] = start[idx];
      c = (int)(start[idx + 1] - start[idx]);
    }
    myc[q] = c;
    mysum += c;
  }
  // block exclusive scan of mysum (thread order = digit order)
  int incl = mysum;
  for (int o = 1; o < kWave; o <<= 1) {
    const int v = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += v;
  }
  if (lane == kWave - 1) s_part[wave] = incl;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += s_part[w];
  int run = before + incl - mysum;
#pragma unroll
  for (int q = 0; q < kMaxDigits / kSortThreads; ++q) {
    const int d = tid * (kMaxDigits / kSortThreads) + q;
    if (d < D) {
      s_toff[d] = run;
      s_run[d] = 0;
      for (int w = 0; w < kSortThreads / kWave; ++w) s_wave[w][d] = 0;
    }
    run += myc[q];
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  // every round's key and payload loaded up front (coalesced across the
  // block, all loads in flight together)
  uint32_t rk[kSortRounds];
  P rp[kSortRounds];
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int li = r * kSortThreads + tid;
    rk[r] = 0;
    rp[r] = P{};
    if (li < cntT) {
      rk[r] = keys[b + li];
      rp[r] = src(b + li);
    }
  }
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int li = r * kSortThreads + tid;  // input order inside the tile
    const bool valid = li < cntT;
    const uint32_t key = rk[r];
    const P pay = rp[r];
    const int dg = valid ? digit_of(key, shift, mask, desc) : 0;
    // lanes of this wavefront holding the same digit
    uint64_t peers = __ballot(valid);
    for (int bit = 0; bit < bits; ++bit) {
      const uint64_t m = __ballot((dg >> bit) & 1);
      peers &= ((dg >> bit) & 1) ? m : ~m;
    }
    const int below = __popcll(peers & lt);
    const bool leader = valid && below == 0;
    const int cw = __popcll(peers);
    if (leader) s_wave[wave][dg] = (short)cw;
    __syncthreads();
    if (valid) {
      int rank = s_run[dg] + below;
      for (int w = 0; w < wave; ++w) rank += s_wave[w][dg];
      const int pos = s_toff[dg] + rank;
      s_key[pos] = key;
      s_pay[pos] = pay;
    }
    __syncthreads();
    if (leader) {
      atomicAdd(&s_run[dg], cw);
      s_wave[wave][dg] = 0;
    }
    __syncthreads();
  }
  // the tile in digit order: each digit's run goes to its output positions
  for (int p = tid; p < cntT; p += kSortThreads) {
    const uint32_t key = s_key[p];
    const int dg = digit_of(key, shift, mask, desc);
    const int64_t o = s_goff[dg] + (p - s_toff[dg]);
    keys_out[o] = key;
    pay_out[o] = s_pay[p];
  }
}

struct SortLayout {
  int passes = 0, dbits[4] = {0, 0, 0, 0};
  int64_t tiles = 0;
  size_t off_keys = 0, off_pay = 0, off_hist = 0, off_scan = 0, bytes = 0;
};

SortLayout sort_layout(int64_t n, unsigned bits, int pay_bytes) {
  SortLayout L;
  if (bits < 1) bits = 1;
  L.passes = (int)((bits + kMaxDigitBits - 1) / kMaxDigitBits);
  int left = (int)bits;
  for (int p = 0; p < L.passes; ++p) {
    L.dbits[p] = (left + (L.passes - p) - 1) / (L.passes - p);
    left -= L.dbits[p];
  }
  const int64_t cnt = n > 0 ? n : 1;
  L.tiles = (cnt + kTile - 1) / kTile;
  auto up = [](size_t x) { return (x + 255) / 256 * 256; };
  const int64_t hist_n = (int64_t)kMaxDigits * L.tiles;
  L.off_keys = 0;
  L.off_pay = up(4 * (size_t)cnt);
  L.off_hist = L.off_pay + up((size_t)pay_bytes * (size_t)cnt);
  L.off_scan = L.off_hist + up(8 * (size_t)(hist_n + 1));
  L.bytes = L.off_scan + up(8 * (size_t)(hist_n + 1)) + up(8 * scan_tmp_elems(hist_n + 1));
  return L;
}

// Passes alternate between the workspace buffers and the output, so that the
// last pass writes the output.
template <typename P, typename Src0>
hipError_t radix_sort(int64_t n, const uint32_t *keys_in, Src0 src0, uint32_t *keys_out, P *pay_out,
                      unsigned bits, bool desc, void *ws, size_t ws_bytes, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const SortLayout L = sort_layout(n, bits, (int)sizeof(P));
  if (ws_bytes < L.bytes) return hipErrorInvalidValue;
  char *w = (char *)ws;
  uint32_t *tk = (uint32_t *)(w + L.off_keys);
  P *tp = (P *)(w + L.off_pay);
  int64_t *hist = (int64_t *)(w + L.off_hist);
  int64_t *start = (int64_t *)(w + L.off_scan);
  int64_t *scan_tmp = (int64_t *)(w + L.off_scan + (8 * (size_t)((int64_t)kMaxDigits * L.tiles + 1) + 255) / 256 * 256);
  const uint32_t *kin = keys_in;
  const P *pin = nullptr;
  int shift = 0;
  for (int p = 0; p < L.passes; ++p) {
    const int db = L.dbits[p];
    const int64_t hn = ((int64_t)1 << db) * L.tiles;
    uint32_t *kout = ((L.passes - 1 - p) % 2 == 0) ? keys_out : tk;
    P *pout = ((L.passes - 1 - p) % 2 == 0) ? pay_out : tp;
    hipLaunchKernelGGL(k_digit_hist, dim3((unsigned)L.tiles), dim3(kSortThreads), 0, st, n, kin, shift, db, (int)desc,
                       L.tiles, hist);
    hipError_t e = launch_scan_i64(hist, hn, start, scan_tmp, st);
    if (e != hipSuccess) return e;
    if (p == 0)
      hipLaunchKernelGGL((k_digit_scatter<P, Src0>), dim3((unsigned)L.tiles), dim3(kSortThreads), 0, st, n, kin, src0,
                         shift, db, (int)desc, L.tiles, (const int64_t *)start, kout, pout);
    else
      hipLaunchKernelGGL((k_digit_scatter<P, PayArray<P>>), dim3((unsigned)L.tiles), dim3(kSortThreads), 0, st, n,
                         kin, PayArray<P>{pin}, shift, db, (int)desc, L.tiles, (const int64_t *)start, kout, pout);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    kin = kout;
    pin = pout;
    shift += db;
  }
  return hipSuccess;
}

}  // namespace

size_t sort_ws_bytes(int64_t n, unsigned bits, int payload_bytes) { return sort_layout(n, bits, payload_bytes).bytes; }

hipError_t sort_keys_packed(int64_t n, const uint32_t *keys_in, const int32_t *row, const float *val,
                            uint32_t *keys_out, uint64_t *pay_out, unsigned bits, void *ws, size_t ws_bytes,
                            hipStream_t st) {
  return radix_sort<uint64_t>(n, keys_in, PayPacked{row, val}, keys_out, pay_out, bits, false, ws, ws_bytes, st);
}

hipError_t sort_keys_index(int64_t n, const uint32_t *keys_in, uint32_t *keys_out, int32_t *idx_out, unsigned bits,
                           bool descending, void *ws, size_t ws_bytes, hipStream_t st) {
  return radix_sort<int32_t>(n, keys_in, PayIndex{}, keys_out, idx_out, bits, descending, ws, ws_bytes, st);
}

}  // namespace dsv
