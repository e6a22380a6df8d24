// Internal declarations shared by the HIP sources of the dashSVD library.
// Target: gfx950 (CDNA4), wave64.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dsv {

constexpr int kWave = 64;
constexpr int kMaxL = 160;

// ------------------------------------------------------------------ bf16
// Storage-only BF16: round to nearest even on the way in, exact on the way out.
struct bf16 {
  uint16_t x;
};

__device__ __forceinline__ float bf2f(bf16 v) { return __uint_as_float((uint32_t)v.x << 16); }
__device__ __forceinline__ bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  bf16 r;
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) {
    r.x = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  } else {
    u += 0x7fffu + ((u >> 16) & 1u);
    r.x = (uint16_t)(u >> 16);
  }
  return r;
}

// ------------------------------------------------------------------ element I/O
template <typename T> __device__ __forceinline__ double to_d(T v) { return (double)v; }
template <> __device__ __forceinline__ double to_d<bf16>(bf16 v) { return (double)bf2f(v); }

template <typename T> struct elem;
template <> struct elem<float> {
  __device__ static __forceinline__ float ld(const float *p) { return *p; }
  __device__ static __forceinline__ void st(float *p, float v) { *p = v; }
};
template <> struct elem<double> {
  __device__ static __forceinline__ double ld(const double *p) { return *p; }
  __device__ static __forceinline__ void st(double *p, double v) { *p = v; }
};
template <> struct elem<bf16> {
  __device__ static __forceinline__ float ld(const bf16 *p) { return bf2f(*p); }
  __device__ static __forceinline__ void st(bf16 *p, float v) { *p = f2bf(v); }
};

// Vector of 16 bytes of T, converted to/from the accumulator type A.
// N = 16 / sizeof(T) elements.
template <typename T, typename A> struct vec16;
template <typename A> struct vec16<float, A> {
  static constexpr int N = 4;
  __device__ static __forceinline__ void load(const float *p, A *o) {
    float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = (A)v.x; o[1] = (A)v.y; o[2] = (A)v.z; o[3] = (A)v.w;
  }
  __device__ static __forceinline__ void unpack(const uint32_t *w, A *o) {
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = (A)__uint_as_float(w[i]);
  }
  __device__ static __forceinline__ void store(float *p, const A *o) {
    float4 v;
    v.x = (float)o[0]; v.y = (float)o[1]; v.z = (float)o[2]; v.w = (float)o[3];
    *reinterpret_cast<float4 *>(p) = v;
  }
};
template <typename A> struct vec16<double, A> {
  static constexpr int N = 2;
  __device__ static __forceinline__ void load(const double *p, A *o) {
    double2 v = *reinterpret_cast<const double2 *>(p);
    o[0] = (A)v.x; o[1] = (A)v.y;
  }
  __device__ static __forceinline__ void unpack(const uint32_t *w, A *o) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
      o[i] = (A)__longlong_as_double((long long)(((uint64_t)w[2 * i + 1] << 32) | w[2 * i]));
  }
  __device__ static __forceinline__ void store(double *p, const A *o) {
    double2 v;
    v.x = (double)o[0]; v.y = (double)o[1];
    *reinterpret_cast<double2 *>(p) = v;
  }
};
template <typename A> struct vec16<bf16, A> {
  static constexpr int N = 8;
  __device__ static __forceinline__ void load(const bf16 *p, A *o) {
    uint4 v = *reinterpret_cast<const uint4 *>(p);
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = (A)__uint_as_float(w[i] << 16);
      o[2 * i + 1] = (A)__uint_as_float(w[i] & 0xffff0000u);
    }
  }
  __device__ static __forceinline__ void unpack(const uint32_t *w, A *o) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = (A)__uint_as_float(w[i] << 16);
      o[2 * i + 1] = (A)__uint_as_float(w[i] & 0xffff0000u);
    }
  }
  __device__ static __forceinline__ void store(bf16 *p, const A *o) {
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uint32_t lo = f2bf((float)o[2 * i]).x, hi = f2bf((float)o[2 * i + 1]).x;
      w[i] = lo | (hi << 16);
    }
    *reinterpret_cast<uint4 *>(p) = make_uint4(w[0], w[1], w[2], w[3]);
  }
};

// Store N elements of A into a row of T (N = the lane width of the panel
// type that defined the column mapping; may differ from 16 / sizeof(T)).
template <typename T, typename A, int N> __device__ __forceinline__ void store_n(T *p, const A *o) {
  constexpr int M = vec16<T, A>::N;
  if constexpr (N % M == 0) {
#pragma unroll
    for (int i = 0; i < N; i += M) vec16<T, A>::store(p + i, o + i);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) elem<T>::st(p + i, o[i]);
  }
}
template <typename T, typename A, int N> __device__ __forceinline__ void load_n(const T *p, A *o) {
  constexpr int M = vec16<T, A>::N;
  if constexpr (N % M == 0) {
#pragma unroll
    for (int i = 0; i < N; i += M) vec16<T, A>::load(p + i, o + i);
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] = (A)elem<T>::ld(p + i);
  }
}

// ------------------------------------------------------------------ plans
// Row-split SpMM plan: rows longer than long_row nonzeros are cut into
// chunks of long_row; each chunk writes a partial row, then one task per
// long row sums its chunks in order (deterministic).
// A chunk of a long row: nonzeros [begin, begin + len) of the row; its
// partial row goes to slot `slot` of the partial buffer (the slots of a row
// are consecutive, in column order).
struct ChunkTask {
  int64_t begin;
  int32_t len;
  int32_t slot;
};
// Long-row chunks are cut at column-slab boundaries (2^slab_log2 columns of
// the gathered panel) and run slab by slab; at most kMaxSlabs slabs.
constexpr int kMaxSlabs = 4096;
struct LongRow {
  int64_t row, first;
  int64_t nch;
};

// Device-resident solver state (one per solve).
struct SolverState {
  double alpha;       // shift used by the next pass
  double alpha_prev;  // alpha' of the PVE check
  double prev_ratio;
  double prev_ek1;
  double ratio;       // ratio of the last pass
  int32_t pass;       // passes executed
  int32_t done;       // set when the PVE check passes
  int32_t cq_off;     // set by a pass tail once the PVE ratio reached cq_switch x tol:
                      // later blocks are orthonormalised by Jacobi eigSVD (read by the
                      // host together with done)
  int32_t converged;
  int32_t deficient;
  int32_t sched_off;  // schedule dropped (guard)
  int32_t learned_ready;  // the learned schedule has been written (pass 2)
  int32_t learned_n;      // predicted pass count of the learned model
  int32_t skip_rescale;  // set by a pass's eig when the loop had already stopped
  int32_t eig_calls;     // eigSVD calls that ran, and their Jacobi sweeps
  int32_t eig_sweeps;
  int32_t pass_skip;     // snapshot of done at the start of the current pass
  int32_t stagnant;      // consecutive passes with ratio > tol and > 0.8 x the previous ratio
  int32_t promote;       // set once stagnant reaches 2 (BF16 panels: switch to FP32)
  // Cholesky-QR pass solver (k_cholqr.hip): 1 when it declined the current
  // call and the Jacobi eigensolver must run; arrivals of its two
  // workgroups (the second one runs the tail, then clears it); 1 when the
  // Cholesky factorisation of the current call completed
  int32_t cq_fallback;
  int32_t cq_arrive;
  int32_t cq_chol_ok;
  int32_t cq_calls;  // calls it accepted
  // index of the last eigensolver call that has started on the device (the
  // main stream holds its SpMMs back until the call is resident on its CU)
  int32_t eig_started;
  // 1 when the one-sided Jacobi eigensolver declined the current call (its
  // Cholesky factorisation failed) and the two-sided one must run
  int32_t j1_decline;
};

// ------------------------------------------------------------------ launchers
// (defined in the .hip files; all asynchronous on `st`)
hipError_t launch_gaussian(uint64_t seed, int64_t rows, int64_t cols, void *out, int64_t ld,
                           int dtype, hipStream_t st, const int32_t *row_to = nullptr);
// The Omega of a batch in one launch: matrix i (stacked rows off[i] ..
// off[i + 1], device) keyed seed0 + i, boff (device) the prefix of its
// blocks of 4 elements (nblk in all); equal to one launch_gaussian a matrix.
hipError_t launch_gaussian_batched(uint64_t seed0, int count, const int64_t *off, const int64_t *boff,
                                   int64_t nblk, int64_t cols, void *out, int64_t ld, int dtype, hipStream_t st);
hipError_t launch_philox_raw(uint64_t seed, int64_t nwords, uint64_t *out, hipStream_t st);

hipError_t launch_scan_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *tmp, hipStream_t st);
// Stable LSD radix sort (k_sort.hip) on the low `bits` bits of 32-bit keys.
// Workspace: sort_ws_bytes(n, bits, payload bytes).  keys_out / the payload
// output receive the sorted keys and payloads; the inputs are not modified.
size_t sort_ws_bytes(int64_t n, unsigned bits, int payload_bytes);
// payload of input i: row[i] | (bits of val[i]) << 32
hipError_t sort_keys_packed(int64_t n, const uint32_t *keys_in, const int32_t *row, const float *val,
                            uint32_t *keys_out, uint64_t *pay_out, unsigned bits, void *ws, size_t ws_bytes,
                            hipStream_t st);
// payload of input i: i; descending = non-increasing keys, ties in input order
hipError_t sort_keys_index(int64_t n, const uint32_t *keys_in, uint32_t *keys_out, int32_t *idx_out, unsigned bits,
                           bool descending, void *ws, size_t ws_bytes, hipStream_t st);
size_t scan_tmp_elems(int64_t n);

// Validation of a CSR (flags[0] |= 1: malformed structure, |= 2: non-finite
// value) with the row index of every nonzero.
hipError_t launch_validate(int64_t m, int64_t n, int64_t nnz, const int64_t *rp, const int32_t *col,
                           const void *val, int dtype, int32_t *rowidx, int32_t *flags, hipStream_t st);
// CSR(A^T) of a validated CSR (rowidx from launch_validate): workspace bytes
// (sort keys, indices and the sort's own storage) and the build.
size_t transpose_ws_bytes(int64_t n, int64_t nnz);
hipError_t launch_transpose(int64_t n, int64_t nnz, const int32_t *col, const int32_t *rowidx, const void *val,
                            int dtype, int64_t *rowT, int32_t *colT, void *valT, void *ws, size_t ws_bytes,
                            hipStream_t st);

// Degree order of a CSR structure with R rows: perm (new -> old, rows by
// non-increasing length, ties by index), inv (old -> new) and the row
// pointer of the permuted structure.  ws: degree_order_ws_bytes(R).
size_t degree_order_ws_bytes(int64_t R);
hipError_t launch_degree_order(int64_t R, const int64_t *rp, int64_t max_len, int32_t *perm, int32_t *inv,
                               int64_t *rp_new, void *ws, size_t ws_bytes, int64_t *scan_tmp, hipStream_t st);
// Entries of a CSR structure moved to the permuted one: entry e of row
// row_of[e] goes to row inv_r[row], column col[e] becomes inv_c[col[e]].
hipError_t launch_permute_entries(int64_t nnz, const int64_t *rp, const int32_t *row_of, int row_of_unsigned,
                                  const int32_t *col, const void *val, int dtype, const int32_t *inv_r,
                                  const int32_t *inv_c, const int64_t *rp_new, int32_t *col_new, void *val_new,
                                  hipStream_t st);
// The two halves of launch_transpose: the sort of the column keys (carrying
// each nonzero's row and value when dtype is F32, its index otherwise) with
// the row pointer of A^T, then the scatter or gather of rows and values (into
// the degree order when inv_r, inv_c and rp_new, the permuted row pointer,
// are given).  Both halves take the same rowidx, val and dtype.
hipError_t launch_transpose_keys(int64_t n, int64_t nnz, const int32_t *col, int64_t *rowT, void *ws,
                                 size_t ws_bytes, hipStream_t st, const int32_t *rowidx, const void *val,
                                 int dtype);
hipError_t launch_transpose_gather(int64_t nnz, const int32_t *rowidx, const void *val, int dtype, const void *ws,
                                   int32_t *colT, void *valT, hipStream_t st, const int64_t *rowT = nullptr,
                                   const int32_t *inv_r = nullptr, const int32_t *inv_c = nullptr,
                                   const int64_t *rp_new = nullptr);
// out[0..3] = *endM, *endT, *nlM, *nlT (chunk totals and long-row counts of
// the two SpMM plans), so that the host reads them with one copy.
// out[0..5]: chunk counts, long-row counts and dense-head rows (hM, hT may be null: 0) of the two plans
hipError_t launch_plan_sizes(const int64_t *endM, const int64_t *endT, const int32_t *nlM, const int32_t *nlT,
                             const int32_t *hM, const int32_t *hT, int64_t *out, hipStream_t st);
// SpMM row-split plan: rows longer than long_row are cut into chunks at the
// column-slab boundaries (slab_log2 >= 31: no slabs) and into pieces of at
// most long_row nonzeros.  nch[r]: chunks of row r; tasks (slot order) and
// tslab: each chunk and its slab; launch_plan_order then lists the chunks
// slab by slab in `order` (slab_cnt: 2 (kMaxSlabs + 1) zeroed words; the
// chunk count is read on the device at off[R]).
// head (device, may be null): rows below *head get no chunks (a dense head)
hipError_t launch_plan_count(int64_t R, const int64_t *rp, const int32_t *col, int32_t long_row, int slab_log2,
                             int64_t *nch, hipStream_t st, const int32_t *head = nullptr);
hipError_t launch_plan_fill(int64_t R, const int64_t *rp, const int32_t *col, int32_t long_row, int slab_log2,
                            const int64_t *off, ChunkTask *tasks, int32_t *tslab, LongRow *longs, int32_t *nlong,
                            hipStream_t st);
hipError_t launch_plan_order(int nslabs, const int64_t *n_chunks, const ChunkTask *tasks, const int32_t *tslab,
                             int32_t *slab_cnt, ChunkTask *order, hipStream_t st);

// SpMM: Y = A X (- alpha Q).  dtypes: 0 f32, 1 f64, 2 bf16.
hipError_t launch_spmm(int64_t R, const int64_t *rp, const int32_t *col, const void *val, int vdtype,
                       const void *X, int64_t ldx, int xdtype, void *Y, int64_t ldy, int ydtype,
                       int ld_cols, int64_t n_chunks, const ChunkTask *tasks, int64_t n_long,
                       const LongRow *longs, void *partial, int32_t long_row, int lane_mult,
                       const void *Q, int64_t ldq, const double *alpha, const int32_t *done, hipStream_t st,
                       const int32_t *rowmat = nullptr, const SolverState *bstate = nullptr,
                       int64_t xrows = 0);

// Dense head of a degree-ordered operand (k_head.hip): its first H rows
// (at most kHeadMax, each with at least max(long_row + 1, ncols / 16)
// nonzeros, none if fewer than kHeadMinRows qualify or if they hold fewer
// than kHeadNnzPerCol nonzeros per column of M) are multiplied as a
// dense block on the matrix cores; the SpMM plan leaves them out.  Dt holds
// M[0:H, :]^T (ncols x kHeadMax) in the accumulation type of the products
// (tdtype 1 = f64 for FP64 panels, else 0 = f32); part holds kHeadSplits
// partial products.
constexpr int kHeadMax = 128;
constexpr int kHeadMaxCols = 160;  // panel columns (ldc) the head kernels take
constexpr int kHeadMinRows = 16;
constexpr int kHeadSplits = 256;
size_t head_dt_bytes(int64_t ncols, int tdtype);
size_t head_part_bytes(int tdtype);
// the row ranges of the splits stay within 32-bit buffer offsets, ldc <= kHeadMaxCols
bool head_fits(int64_t K, int64_t ldx, int xdtype, int ldc);
// the head's nonzeros must be at least this many times the operator's columns
constexpr int kHeadNnzPerCol = 16;
// *out = H of the rows of a degree-ordered CSR (thr = least nonzeros of a head
// row, min_nnz = least nonzeros of the whole head)
hipError_t launch_head_count(int64_t R, const int64_t *rp, int64_t thr, int64_t min_nnz, int32_t *out,
                             hipStream_t st);
// Dt (ncols x kHeadMax) from the first H rows of the CSR of M
hipError_t launch_head_build(int64_t ncols, const int64_t *rp, const int32_t *col, const void *val, int vdtype,
                             int H, void *Dt, int tdtype, hipStream_t st);
// rows 0..H-1 of Y = M X (- alpha Q), X with K rows; same dtypes and done flag as launch_spmm
hipError_t launch_head_product(int H, int64_t K, const void *X, int64_t ldx, int xdtype, int ldc, const void *Dt,
                               int tdtype, void *part, void *Y, int64_t ldy, int ydtype, const void *Q,
                               int64_t ldq, const double *alpha, const int32_t *done, hipStream_t st);

// snap (optional): receives *done as read at the start of the Gram kernel,
// i.e. whether the iteration had already stopped when this pass began.
hipError_t launch_gram(int64_t r, int l, const void *C, int64_t ldc, int cdtype, double *partial,
                       int nblocks, double *G, const int32_t *done, hipStream_t st, int32_t *snap);
int gram_blocks(int64_t r, int l);
size_t gram_partial_elems(int nblocks, int l);

// Jacobi eigensolver + eigSVD tail.  mode: 0 = plain eig (kernel entry),
// 1 = sketch, 2 = power pass (PVE check + shift update), 3 = final.
// One entry of the tuning database (dashsvd_autotune): SpMM chunk length,
// lane vectors per lane (1 or 2), column-slab KiB (0: none), degree order
// (+1 on, -1 off, 0 by the size rule).
struct TuneVal {
  int32_t T = 0, vm = 1, slab_kib = 0, reorder = 0;
};

struct EigArgs {
  int l, k;
  double skip;      // Jacobi threshold: rotate only if |g_pq| > skip sqrt(|g_pp g_qq|)
  const double *G;
  double *S;        // l, descending
  double *Vs;       // l x l, eigenvectors in descending order (may be null)
  double *W;        // l x l, Vs diag(1/S), zeroed columns below threshold
  int32_t *sweeps;  // optional
  SolverState *state;
  int mode;
  int pve_mode;     // 0 = R2, 1 = R1
  int policy;       // shift policy
  double tol;
  double *Sprev;    // l
  double *trace_alpha, *trace_ratio, *trace_s;  // [cap], [cap], [cap*l]
  int trace_cap;
  const double *sched;  // device multipliers (SCHEDULE / LEARNED), may be null
  int sched_len;
  int stagnation_guard;  // track stagnant / promote (BF16 panel form)
  int32_t *ndone;        // batched form: [0] incremented once when this matrix stops,
                         // [1] once when it asks for FP32 panels
  // learned shift (policy LEARNED): MLP parameters (see k_mlp.hip), its
  // input width D = 3 l + 3 and hidden width H, the cap of c, and the three
  // shape features log m, log n, log(nnz / m) of the operator
  const float *mlp;
  int mlp_D, mlp_H;
  double mlp_cmax;
  double shape_feat[3];
  long long *prof;      // optional step profile (6 counters; 8 for the tridiagonal solver), null in the solver
  int32_t *trace_sweeps;  // sweeps of call c (c = state->eig_calls before this call), [cap + 2]
  const int32_t *run_if;  // Jacobi only: when set, the call does nothing unless *run_if != 0
  const int32_t *skip_if; // Jacobi only: when set, the call does nothing if *skip_if != 0
  double cq_switch;       // pass tail: set state->cq_off once ratio <= cq_switch x tol (0: never)
  int32_t call_idx;       // > 0: store it to state->eig_started when the call starts working
  int32_t *decline;       // one-sided Jacobi: set to 1 when its Cholesky factorisation fails
                          // (the two-sided kernel gated on it then runs), else 0; the
                          // tridiagonal solver: set to 1 on clusters or non-finite G
  double *tri_ws;         // tridiagonal solver: workspace of kTriWsBytes
};
// Store idx to *flag (agent scope): an eigensolver call has started.
__device__ __forceinline__ void signal_started(int32_t *flag, int32_t idx) {
  __hip_atomic_store(flag, idx, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// One wave that returns once *flag >= expect, or after about 200 us (the
// wait only orders dispatch; it never blocks the stream for longer).
hipError_t launch_wait_started(const int32_t *flag, int32_t expect, hipStream_t st);
// MLP of the learned shift (k_mlp.hip)
struct MlpDims {
  int D, H;
};
constexpr int kMlpH = 128;
constexpr float kMlpLambda = 0.1f;  // weight of the log pass-count term of the loss
inline int64_t mlp_num_params(int D, int H) { return (int64_t)H * D + H + (int64_t)H * H + H + 2 * H + 2; }
hipError_t mlp_forward(const MlpDims &d, const float *P, const float *X, int B, float *A1, float *A2, float *O,
                       hipStream_t st);
hipError_t mlp_backward(const MlpDims &d, const float *P, const float *X, const float *T, int B, float cmax,
                        float lambda, float *A1, float *A2, float *O, float *dO, float *dA2, float *dA1, float *G,
                        float *loss, hipStream_t st);
hipError_t mlp_adam(float *P, const float *G, float *m, float *v, int64_t n, float lr, int t, hipStream_t st);

// Evaluation vector kernels (k_eval.hip).  X, V, Z: FP64 column-major, one
// vector of n entries every ld.  partial: eval_partial_elems(J) doubles.
size_t eval_partial_elems(int J);
// out[j] = sum_r X[j ldx + r] y[r], j < J
hipError_t launch_dots(int64_t n, int J, const double *X, int64_t ldx, const double *y, double *partial,
                       double *out, hipStream_t st);
// out[i] = sum_r (Z[i ld + r] - S[i] V[i ld + r])^2, i < k
hipError_t launch_resid_norms(int64_t n, int k, const double *Z, const double *V, int64_t ld, const double *S,
                              double *partial, double *out, hipStream_t st);
// y[r] -= sum_j X[j ldx + r] c[j] (scale[j] c[j] when scale is given)
hipError_t launch_combo(int64_t n, int J, const double *X, int64_t ldx, const double *c, const double *scale,
                        double *y, hipStream_t st);
// out[r] = w[r] / sqrt(*nrm2)
hipError_t launch_scale_by_norm(int64_t n, const double *w, const double *nrm2, double *out, hipStream_t st);
// out[j ldo + row_to(r)] = in[r ldi + j] (in F32 or F64, row-major)
hipError_t launch_to_colmajor(int64_t rows, int cols, const void *in, int64_t ldi, int idtype, double *out,
                              int64_t ldo, const int32_t *row_to, hipStream_t st);
hipError_t launch_eig(const EigArgs &a, hipStream_t st);
// Accuracy control without the surrogate (Sec. 4.3): eq. (18) on the
// squared singular values Sb (l, descending) of B = M Q of the pass just
// run against those of the previous pass (Ebp, zero before the first pass;
// updated unless the check stops the loop).  Writes the ratio to the solver
// state and the pass's trace slot, sets done / converged when it is <= tol
// and cq_off when it is <= cq_switch x tol.  Nothing happens when *gate is
// set (the pass was launched after the stop).  One workgroup.
hipError_t launch_pve_nosurr(int k, int l, const double *Sb, double *Ebp, double tol, double cq_switch,
                             SolverState *state, double *trace_ratio, int trace_cap, const int32_t *gate,
                             hipStream_t st);
// Orthonormalisation of a pass block (modes 1 and 2) without eigenvectors:
// the Cholesky-QR weights W = R^-1 (G = R^T R) and S from the eigenvalues
// of G, then the Jacobi eigensolver on the same arguments, which runs only
// where the first one declined (G not safely positive definite).  Needs
// a.state.
hipError_t launch_eig_pass(const EigArgs &a, hipStream_t st);
// the first kernel of launch_eig_pass alone (state->cq_fallback tells
// whether it declined)
hipError_t launch_cholqr(const EigArgs &a, hipStream_t st);
// arr: count EigArgs in device memory, all with the same l; workgroup b
// solves arr[b]
hipError_t launch_eig_batched(const EigArgs *arr, int count, int l, hipStream_t st);
// One-sided Jacobi on the Cholesky factor of G (k_eig1s.hip): the same
// outputs and tail as launch_eig, for l <= 128 (hipErrorInvalidValue
// above); declines (*a.decline = 1, nothing else written) when G is not
// positive definite to working precision, and the two-sided kernel gated
// on the flag (run_if = decline) then runs.
hipError_t launch_eig1s(const EigArgs &a, hipStream_t st);
// Tridiagonal eigensolver (k_eigtri.hip): Householder reduction in one
// workgroup, then one wave per eigenvalue (multisection, twisted-
// factorisation eigenvector, back-transformation); the same outputs and tail
// as launch_eig for l <= kTriMaxL.  a.W, a.Vs, a.decline and a.tri_ws
// (kTriWsBytes: the tridiagonal, the reflectors, flags) are required.
// Declines (*a.decline = 1; S, Vs and W then hold no result, the state is
// untouched) on eigenvalue clusters and zero or non-finite G.
constexpr int kTriMaxL = 160;
constexpr size_t kTriWsBytes = 8 * (4 * (size_t)kTriMaxL + 16 + (size_t)kTriMaxL * kTriMaxL);
hipError_t launch_eigtri(const EigArgs &a, hipStream_t st);
hipError_t launch_eig1s_batched(const EigArgs *arr, int count, int l, hipStream_t st);

// ------------------------------------------------------------------ batched form
// One matrix of a batch inside the stacked block-diagonal operator.
struct BMatDesc {
  const int64_t *rp;  // source arrays (unused when assembling in place)
  const int32_t *col;
  const void *val;
  int64_t m, n, nnz;
  int64_t row_off, col_off, nnz_off;  // position in the stacked operator
};
// A work item: rows [r0, r1) of matrix mat (stacked row numbers).
struct BItem {
  int32_t mat;
  int32_t pad;
  int64_t r0, r1;
};
constexpr int kBStrip = 64;       // rows staged in LDS at a time
constexpr int kBItemRows = 512;   // rows per work item
constexpr int kBMaxL = 64;        // largest l of the batched dense kernels

hipError_t launch_bassemble(const BMatDesc *d, int count, int64_t max_rows_nnz, int64_t total_rows,
                            int64_t total_nnz, int64_t *rp, int32_t *col, void *val, int vdtype, int in_place,
                            int32_t *flags, hipStream_t st);
hipError_t launch_browmat(const int64_t *off, int count, int64_t max_rows, int32_t *rowmat, hipStream_t st);
hipError_t launch_bsnap(SolverState *state, int count, int snap, hipStream_t st);
size_t bgram_partial_elems(int64_t n_items, int l);
hipError_t launch_bgram(const BItem *items, int64_t n_items, const int64_t *item_off, int count, int l,
                        const void *C, int64_t ldc, int cdtype, double *partial, double *G, int64_t g_stride,
                        const SolverState *state, int gate, hipStream_t st);
hipError_t launch_brescale(const BItem *items, int64_t n_items, int l, const void *C, const void *R, int64_t ldc,
                           int cdtype, const double *W, int64_t w_stride, int64_t ldw, int c, void *Out,
                           int64_t ldo, int odtype, const SolverState *state, int gate, hipStream_t st);
hipError_t launch_bsign(const int64_t *voff, const int64_t *uoff, int count, int k, void *V, void *U, int64_t ld,
                        int dtype, hipStream_t st);

// Out = (C - alpha R) W when R is given (R laid out like C, alpha on the
// device), else Out = C W.
// Out = (C - alpha R) W; row_to (optional): row i of the product is stored
// in row row_to[i] of Out.
hipError_t launch_rescale(int64_t r, int l, const void *C, int64_t ldc, int cdtype, const double *W,
                          int64_t ldw, int c, void *Out, int64_t ldo, int odtype,
                          const int32_t *done, hipStream_t st, const void *R = nullptr,
                          const double *alpha = nullptr, const int32_t *row_to = nullptr);

// pmax: nblk*k doubles, pidx: nblk*k int64 followed by k floats (workspace)
// C (m x n) = op(A) B for small FP64 matrices (op(A) = A^T if transA)
hipError_t launch_small_gemm(int m, int n, int kk, const double *A, int lda, int transA, const double *B, int ldb,
                             double *C, int ldc, hipStream_t st);
// Sign normalisation of V (entry of largest magnitude positive per column,
// lowest row on ties) with the same flips applied to the columns of P
// (prow x k, FP64), the weights that form U afterwards.
hipError_t launch_sign_fold(int64_t rowsV, int k, void *V, int64_t ldv, int dtype, double *P, int prow, int ldp,
                            void *pmax, void *pidx, int nblk, hipStream_t st);
hipError_t launch_sign_fix(int64_t rowsV, int64_t rowsU, int k, void *V, int64_t ldv, void *U,
                           int64_t ldu, int dtype, void *pmax, void *pidx, int nblk,
                           hipStream_t st);
hipError_t launch_convert(const void *in, int idtype, void *out, int odtype, int64_t n,
                          hipStream_t st);
hipError_t launch_copy2d(const void *in, int64_t ldi, int idtype, void *out, int64_t ldo,
                         int odtype, int64_t rows, int cols, hipStream_t st, const int32_t *row_to = nullptr);
hipError_t launch_fill_zero_i32(int32_t *p, int64_t n, hipStream_t st);
// Zero several small buffers (sizes in 4-byte words) with one launch.
constexpr int kMaxZeroRanges = 12;
struct ZeroRanges {
  int32_t *p[kMaxZeroRanges];
  int64_t n[kMaxZeroRanges];
  int count;
  void add(void *ptr, size_t bytes) {
    p[count] = (int32_t *)ptr;
    n[count] = (int64_t)(bytes / 4);
    ++count;
  }
};
hipError_t launch_zero_ranges(const ZeroRanges &z, hipStream_t st);

}  // namespace dsv
