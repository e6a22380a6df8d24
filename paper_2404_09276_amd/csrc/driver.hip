// C ABI and host driver of the dashSVD library (Alg. 5 of the paper, with
// Alg. 3 for every orthonormalisation and Alg. 4 as the tol = 0 case).
//
// The driver is a stream-ordered sequence of the library's kernels:
//   setup   : CSR validation -> CSR(A^T) -> SpMM plans -> Omega
//   sketch  : Y0 = M^T Omega -> eigSVD -> Q                 (Alg. 5 step 2)
//   pass j  : Y = M Q ; C = M^T Y - alpha Q ; G = C^T C ;
//             eig + PVE check + shift update (device) ; Q = C W   (steps 4-7)
//   final   : B = M Q ; eigSVD(B) ; U = B W_B(:,1:k) ; V = Q V_B(:,1:k) (9-11)
// where M = A if m >= n and M = A^T otherwise (Sec. 3.1).  The shift, the
// previous singular values and the done flag live on the device; the host
// reads the done flag once every check_interval passes (in the overlapped
// order, one chunk behind, while the next chunk runs), and passes launched
// after the flag is set return at their first instruction.
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <algorithm>

#include "../../include/dashsvd.h"
#include "common.h"

using namespace dsv;

namespace {

thread_local std::string g_create_error;

constexpr int kDefaultLongRow = 128;
// Default chunk length from DASHSVD_REORDER_MIN_NNZ nonzeros: on the
// degree-ordered power-law operators of that size with their dense head,
// chunks of 1024 nonzeros gave the fastest FP32 products (fewer partial rows;
// on the 10M-nonzero benchmark matrix the solve took 7.38 ms against 7.66,
// 7.56 and 7.60 ms with 512, 768 and 1536, timed in one process; the
// 100M-nonzero matrix is within 1 % from 768 to 2048).  BF16 panels gather
// rows half as wide, and 768 stays faster for them (8.10 against 8.38 ms).
constexpr int kDefaultLongRowLarge = 1024;
constexpr int kDefaultLongRowLargeBf16 = 768;
constexpr int kDefaultPmax = 64;

size_t dsz(int dt) { return dt == DASHSVD_F64 ? 8 : (dt == DASHSVD_BF16 ? 2 : 4); }
int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Pinned host staging area of a handle: flag slots and plan sizes in the
// first 256 bytes, then the solver state and the per-pass traces copied back
// at the end of a solve.
constexpr size_t kPinState = 256, kPinAlpha = 1024, kPinRatio = kPinAlpha + 8 * DASHSVD_MAX_TRACE,
                 kPinSweeps = kPinRatio + 8 * DASHSVD_MAX_TRACE, kPinBytes = 8192;
static_assert(sizeof(SolverState) <= kPinAlpha - kPinState, "solver state fits its staging slot");
static_assert(kPinSweeps + 4 * (DASHSVD_MAX_TRACE + 2) <= kPinBytes, "traces fit the staging area");

// Bump allocator over one device arena.
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0;
  bool measuring = false;
  void reset(bool measure) {
    used = 0;
    measuring = measure;
  }
  void *take(size_t bytes) {
    const size_t off = (size_t)round_up((int64_t)used, 256);
    used = off + (size_t)round_up((int64_t)bytes, 256);
    if (measuring) return nullptr;
    return base + off;
  }
};

struct Plan {
  int64_t R = 0;
  int64_t n_chunks = 0, n_long = 0;
  int64_t *nch = nullptr, *off = nullptr;
  ChunkTask *tasks = nullptr;  // chunks in slot order
  ChunkTask *order = nullptr;  // the same chunks slab by slab (the launch order)
  int32_t *tslab = nullptr;    // slab of each chunk (slot order)
  int32_t *slab_cnt = nullptr; // 2 (kMaxSlabs + 1) words, zero before the build
  int slab_log2 = 31, nslabs = 1;
  LongRow *longs = nullptr;
  int32_t *nlong = nullptr;
  void *partial = nullptr;
  // dense head (k_head.hip): the first `head` rows of a degree-ordered
  // operator, left out of the chunks and multiplied as a dense block
  int32_t *head_dev = nullptr;  // H as counted on the device (null: no head)
  int32_t head = 0;             // H as read back by the host
  int64_t head_cols = 0;        // columns of the operator (rows of the panel it multiplies)
  int head_t = 0;               // type of Dt and of the partial products: 1 f64, 0 f32
  void *dt = nullptr;           // M[0:H, :]^T, head_cols x kHeadMax
  void *hpart = nullptr;        // kHeadSplits partial products
};

// Column-slab width (log2, in columns of the operator = rows of the gathered
// panel) of the long-row chunks: about slab_bytes of panel rows, a power of
// two, at most kMaxSlabs slabs; 31 = no cuts (one slab, or slab_bytes <= 0,
// the default: on the 10M-nonzero power-law benchmark matrix, slabs of 512
// KiB to 8 MiB made the product of A 8-10 % slower, every chunk of the long
// rows being resident at once anyway).
int slab_log2_for(int64_t ncols, int64_t row_bytes, int64_t slab_bytes) {
  if (ncols <= 0 || slab_bytes <= 0 || row_bytes <= 0) return 31;
  int64_t w = slab_bytes / row_bytes;
  if (w < 1) w = 1;
  int lg = 0;
  while (lg < 30 && ((int64_t)2 << lg) <= w) ++lg;
  while (lg < 30 && ((ncols - 1) >> lg) + 1 > kMaxSlabs) ++lg;
  if (((int64_t)1 << lg) >= ncols) return 31;
  return lg;
}

}  // namespace

struct dashsvd_handle {
  dashsvd_options opt;
  std::vector<double> sched;
  std::string err;
  hipStream_t st = nullptr;
  Arena ar;
  bool ar_external = false;  // the arena is a caller buffer (dashsvd_set_workspace)
  // results of the last run (device pointers into the arena)
  bool have = false;
  int64_t m = 0, n = 0;
  int k = 0, l = 0;
  int out_dt = DASHSVD_F32;
  void *U = nullptr, *V = nullptr;
  double *S = nullptr;
  double *trace_s = nullptr;
  int trace_cap = 0;
  dashsvd_info info;
  // kernel-group timing (options.timing)
  std::vector<hipEvent_t> ev;
  struct Mark {
    int group, pass, e0, e1;
  };
  std::vector<Mark> marks;
  int ev_used = 0;
  int open_group = -1, open_pass = 0, open_e0 = 0;
  // second stream for the eigensolver, overlapped with the next SpMM
  hipStream_t st2 = nullptr;
  hipEvent_t ev_gram = nullptr, ev_eig = nullptr;
  // pinned host memory for the reads the host waits on: [0, 16) the stop
  // test one chunk behind (two slots of done, cq_off, each filled by a copy
  // queued behind a chunk of passes); [64, 96) the SpMM plan sizes;
  // [128, 144) the CSR validation flags
  int32_t *hflags = nullptr;
  hipEvent_t ev_flag[2] = {nullptr, nullptr};
  // what dashsvd_evaluate needs of the last run: the operator M (A, or A^T
  // when m < n) and its transpose with their SpMM plans, and free panels
  struct EvalCtx {
    bool ok = false;
    int64_t nnz = 0, Mm = 0, Mn = 0;
    bool wide = false;
    int vdt = 0, cdt = 0, ld = 0;
    int32_t T = 0;
    const int64_t *rp[2] = {nullptr, nullptr};
    const int32_t *col[2] = {nullptr, nullptr};
    const void *val[2] = {nullptr, nullptr};
    Plan plan[2];
    void *panel_m = nullptr, *panel_n = nullptr;  // Mm x ld and Mn x ld, cdt
    double *gpart = nullptr, *G = nullptr;
    const int32_t *u_row_to = nullptr;  // degree order: row r of U goes to row u_row_to[r] of the panel
    const int32_t *v_row_to = nullptr;  // and row r of V to row v_row_to[r]
  } ev_ctx;
  // results of the last batched run
  struct BatchOut {
    bool have = false;
    int count = 0, k = 0, l = 0, cap = 0, out_dt = 0;
    std::vector<int64_t> m, n, row_off, col_off;
    void *Uo = nullptr, *Vo = nullptr;
    double *S = nullptr;  // count x l
    SolverState *state = nullptr;
    double *tr_alpha = nullptr, *tr_ratio = nullptr;  // count x cap
    int32_t *tr_sweeps = nullptr;                     // count x (cap + 2)
    dashsvd_info info;
  } bat;
  // results of a batch run in several sub-batches, gathered member by
  // member (the arena holds one sub-batch at a time); own device memory,
  // grown as needed and kept across runs
  struct BatchAll {
    void *base = nullptr;
    size_t cap = 0;
  } ball;
  // learned-shift MLP (its own device memory, kept across runs)
  struct Mlp {
    bool ok = false;
    int l = 0, D = 0, H = 0;
    double cmax = 0.9;
    int64_t np = 0;
    float *P = nullptr, *G = nullptr, *m = nullptr, *v = nullptr;
    int step = 0;
    float *buf = nullptr;  // batch buffers of forward / backward
    int buf_batch = 0;
  } mlp;
  // SpMM chunk lengths by shape bucket (tuning database)
  std::vector<std::pair<std::string, TuneVal>> tune;
  // internal stream of the batched form (its pass is captured as a graph)
  hipStream_t stg = nullptr;
  hipEvent_t ev_b0 = nullptr, ev_b1 = nullptr;
};

namespace {

hipEvent_t take_event(dashsvd_handle *h, int &idx) {
  if (h->ev_used == (int)h->ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev.push_back(e);
  }
  idx = h->ev_used++;
  return h->ev[idx];
}

// Open / close a timed kernel group on the handle's stream (no-op unless
// options.timing is set; with DASHSVD_TIMING_SPMM only the SpMM groups).
void tmark_begin(dashsvd_handle *h, int group, int pass, hipStream_t on = nullptr) {
  if (!h->opt.timing) return;
  if (h->opt.timing == DASHSVD_TIMING_SPMM && group != DASHSVD_KT_SPMM && group != DASHSVD_KT_SPMM_T) {
    h->open_group = -1;
    return;
  }
  int i;
  hipEvent_t e = take_event(h, i);
  if (!e || hipEventRecord(e, on ? on : h->st) != hipSuccess) return;
  h->open_group = group;
  h->open_pass = pass;
  h->open_e0 = i;
}
void tmark_end(dashsvd_handle *h, hipStream_t on = nullptr) {
  if (!h->opt.timing || h->open_group < 0) return;
  int i;
  hipEvent_t e = take_event(h, i);
  if (e && hipEventRecord(e, on ? on : h->st) == hipSuccess)
    h->marks.push_back({h->open_group, h->open_pass, h->open_e0, i});
  h->open_group = -1;
}

dashsvd_status fail(dashsvd_handle *h, dashsvd_status s, const std::string &what) {
  if (h) h->err = what;
  else g_create_error = what;
  return s;
}

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess)                                                                      \
      return fail(h, DASHSVD_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_));        \
  } while (0)

void default_options(dashsvd_options *o) {
  std::memset(o, 0, sizeof(*o));
  o->precision = DASHSVD_PREC_FP32;
  o->shift_policy = DASHSVD_SHIFT_PAPER;
  o->pve_mode = DASHSVD_PVE_R2;
  o->p_max = -1;
  o->omega_dtype = DASHSVD_F64;
}

// Shape bucket of the tuning database.
std::string tune_key(int prec, int ld, int64_t rows, int64_t nnz, bool batched) {
  auto lg = [](double x) { return (int)std::lround(std::log2(x > 1.0 ? x : 1.0)); };
  return "p" + std::to_string(prec) + "_ld" + std::to_string(ld) + "_r" + std::to_string(lg((double)rows)) +
         "_d" + std::to_string(lg((double)nnz / (double)(rows > 0 ? rows : 1))) + (batched ? "_b" : "_s");
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

dashsvd_status ensure_arena(dashsvd_handle *h, size_t bytes) {
  if (bytes <= h->ar.cap) return DASHSVD_OK;
  if (h->ar_external)
    return fail(h, DASHSVD_ERR_OOM, "the caller's workspace holds " + std::to_string(h->ar.cap) +
                                        " bytes; this run needs " + std::to_string(bytes));
  if (h->ar.base) {
    (void)hipStreamSynchronize(h->st);
    if (h->st2) (void)hipStreamSynchronize(h->st2);
    (void)hipFree(h->ar.base);
    h->ar.base = nullptr;
    h->ar.cap = 0;
    h->have = false;
  }
  void *p = nullptr;
  const size_t want = bytes + bytes / 16;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, DASHSVD_ERR_OOM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  h->ar.base = (char *)p;
  h->ar.cap = want;
  return DASHSVD_OK;
}

// Row-split plan of a CSR with R rows and ncols columns (two phases around a
// host read).  A long row has at most len / T + 1 chunks of T plus one cut
// per slab boundary it crosses.
dashsvd_status plan_alloc(dashsvd_handle *h, Arena &ar, Plan &p, int64_t R, int64_t nnz, int32_t T,
                          int ld, size_t acc_sz, int64_t ncols = 0, int64_t row_bytes = 0,
                          int64_t slab_bytes = 0, int head_t = -1) {
  p.R = R;
  p.slab_log2 = slab_log2_for(ncols, row_bytes, slab_bytes);
  p.nslabs = p.slab_log2 >= 31 ? 1 : (int)(((ncols - 1) >> p.slab_log2) + 1);
  const int64_t max_long = nnz / T + 1;
  const int64_t max_chunks = 2 * (nnz / T) + 1 + (p.nslabs > 1 ? max_long * (p.nslabs - 1) : 0);
  p.nch = (int64_t *)ar.take(sizeof(int64_t) * (size_t)(R + 1));
  p.off = (int64_t *)ar.take(sizeof(int64_t) * (size_t)(R + 2));
  p.tasks = (ChunkTask *)ar.take(sizeof(ChunkTask) * (size_t)max_chunks);
  p.order = (ChunkTask *)ar.take(sizeof(ChunkTask) * (size_t)max_chunks);
  p.tslab = (int32_t *)ar.take(sizeof(int32_t) * (size_t)max_chunks);
  p.slab_cnt = (int32_t *)ar.take(sizeof(int32_t) * 2 * (size_t)(kMaxSlabs + 1));
  p.longs = (LongRow *)ar.take(sizeof(LongRow) * (size_t)max_long);
  p.nlong = (int32_t *)ar.take(sizeof(int32_t) * 4);
  p.partial = ar.take(acc_sz * (size_t)ld * (size_t)max_chunks);
  // a dense head (head_t >= 0): its count, Dt and the partial products
  p.head = 0;
  p.head_cols = ncols;
  p.head_dev = nullptr;
  p.dt = p.hpart = nullptr;
  if (head_t >= 0 && ncols > 0) {
    p.head_t = head_t;
    p.head_dev = (int32_t *)ar.take(16);
    p.dt = ar.take(head_dt_bytes(ncols, head_t));
    p.hpart = ar.take(head_part_bytes(head_t));
  }
  (void)h;
  return DASHSVD_OK;
}

// The plan's kernels: chunk counts, their scan, the chunks in slot order and
// then slab by slab (p.nlong and p.slab_cnt zeroed beforehand).
hipError_t plan_build(Plan &p, const int64_t *rp, const int32_t *col, int32_t T, int64_t *scan_tmp, hipStream_t st) {
  hipError_t e = launch_plan_count(p.R, rp, col, T, p.slab_log2, p.nch, st, p.head_dev);
  if (e == hipSuccess) e = launch_scan_i64(p.nch, p.R, p.off, scan_tmp, st);
  if (e == hipSuccess) e = launch_plan_fill(p.R, rp, col, T, p.slab_log2, p.off, p.tasks, p.tslab, p.longs, p.nlong, st);
  // one slab: the chunks run in slot order (row by row)
  if (p.nslabs <= 1) {
    p.order = p.tasks;
    return e;
  }
  if (e == hipSuccess) e = launch_plan_order(p.nslabs, p.off + p.R, p.tasks, p.tslab, p.slab_cnt, p.order, st);
  return e;
}

// A product with a plan's operator: the row-split SpMM over the rows of the
// plan, then its dense head rows (k_head.hip) when it has them.  Same
// arguments as launch_spmm; X has p.head_cols rows.
hipError_t plan_spmm(const Plan &p, int64_t R, const int64_t *rp, const int32_t *col, const void *val, int vdt,
                     const void *X, int64_t ldx, int xdt, void *Y, int64_t ldy, int ydt, int ldc, int32_t T, int vm,
                     const void *Q, int64_t ldq, const double *alpha, const int32_t *done, hipStream_t st) {
  hipError_t e = launch_spmm(R, rp, col, val, vdt, X, ldx, xdt, Y, ldy, ydt, ldc, p.n_chunks, p.order, p.n_long,
                             p.longs, p.partial, T, vm, Q, ldq, alpha, done, st, nullptr, nullptr, p.head_cols);
  if (e == hipSuccess && p.head > 0)
    e = launch_head_product(p.head, p.head_cols, X, ldx, xdt, ldc, p.dt, p.head_t, p.hpart, Y, ldy, ydt, Q, ldq,
                            alpha, done, st);
  return e;
}

struct RunBufs {
  // CSR of M and M^T on device (compute value type)
  const int64_t *rpA = nullptr;
  const int32_t *colA = nullptr;
  const void *valA = nullptr;
  int64_t *rpT = nullptr;
  int32_t *colT = nullptr;
  void *valT = nullptr;
  // transposition temporaries
  int32_t *rowidx = nullptr, *flags = nullptr;
  int64_t *sizes = nullptr;  // 4 plan sizes for the host
  void *tws = nullptr;  // CSR(A^T) build workspace
  size_t tws_bytes = 0;
  int64_t *scan_tmp = nullptr;
  Plan planM, planT;
  // panels
  void *Y = nullptr;   // M_m x ld, panel type (also Omega)
  void *Q = nullptr;   // M_n x ld, panel type
  void *C = nullptr;   // M_n x ld, C type (f32 / f64)
  void *B = nullptr;   // M_m x ld, C type (final block)
  void *Z = nullptr;   // M_m x ld, C type: M C of the current block
  void *X = nullptr;   // M_n x ld, C type: M^T M C of the current block (overlapped order)
  void *Q32 = nullptr, *Y32 = nullptr;  // FP32 panels after a BF16 promotion
  double *gpart = nullptr, *G = nullptr, *W = nullptr, *Vs = nullptr, *S = nullptr, *Sprev = nullptr;
  double *G2 = nullptr, *T2 = nullptr, *W2 = nullptr, *PU = nullptr, *PV = nullptr;  // final step
  double *Sb = nullptr, *Ebp = nullptr;  // check without the surrogate: sigma(M Q), previous sigma(M Q)^2
  SolverState *state = nullptr;
  double *tri_ws = nullptr;  // tridiagonal eigensolver workspace
  double *tr_alpha = nullptr, *tr_ratio = nullptr, *tr_s = nullptr;
  int32_t *tr_sweeps = nullptr;
  double *sched = nullptr;
  void *Uo = nullptr, *Vo = nullptr;
  double *So = nullptr;
  void *sgn_max = nullptr, *sgn_idx = nullptr;
  // degree order (options.reorder): perm new -> old, inv old -> new, for the
  // rows (r, m of them) and columns (c, n) of A; the permuted A and A^T
  int32_t *perm_r = nullptr, *inv_r = nullptr, *perm_c = nullptr, *inv_c = nullptr;
  int64_t *rpP = nullptr, *rpPT = nullptr;
  int32_t *colP = nullptr;  // the permuted A^T takes colT and valT
  void *valP = nullptr;
  void *dws = nullptr;
  size_t dws_bytes = 0;
  void *omega_dev = nullptr;
};

}  // namespace

// ===================================================================== C ABI
extern "C" {

const char *dashsvd_status_string(dashsvd_status s) {
  switch (s) {
    case DASHSVD_OK: return "ok";
    case DASHSVD_NOT_CONVERGED: return "not converged within p_max passes (results valid)";
    case DASHSVD_RANK_DEFICIENT: return "rank deficient block: some columns zeroed (results valid)";
    case DASHSVD_ERR_INVALID_ARG: return "invalid argument";
    case DASHSVD_ERR_BAD_CSR: return "malformed CSR matrix";
    case DASHSVD_ERR_NONFINITE: return "non-finite value in the matrix";
    case DASHSVD_ERR_OOM: return "out of device memory";
    case DASHSVD_ERR_HIP: return "HIP runtime error";
    case DASHSVD_ERR_STATE: return "call out of order";
    default: return "unknown status";
  }
}

const char *dashsvd_last_error(const dashsvd_handle *h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

dashsvd_status dashsvd_set_options(dashsvd_handle *h, const dashsvd_options *opt) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  dashsvd_options o;
  default_options(&o);
  if (opt) o = *opt;
  if (o.precision < 0 || o.precision > 2) return fail(h, DASHSVD_ERR_INVALID_ARG, "precision");
  if (o.shift_policy < 0 || o.shift_policy > 4) return fail(h, DASHSVD_ERR_INVALID_ARG, "shift_policy");
  if (o.pve_mode < 0 || o.pve_mode > 2) return fail(h, DASHSVD_ERR_INVALID_ARG, "pve_mode");
  if (o.eig_method < 0 || o.eig_method > 4) return fail(h, DASHSVD_ERR_INVALID_ARG, "eig_method");
  if (o.reorder < -1 || o.reorder > 1) return fail(h, DASHSVD_ERR_INVALID_ARG, "reorder");
  if (o.dense_head < -1 || o.dense_head > 0) return fail(h, DASHSVD_ERR_INVALID_ARG, "dense_head");
  if (o.lane_vectors > 2) return fail(h, DASHSVD_ERR_INVALID_ARG, "lane_vectors (1 or 2; <= 0: tuned or 1)");
  if (o.p_max < 0) o.p_max = kDefaultPmax;
  if (o.p_max > 100000) return fail(h, DASHSVD_ERR_INVALID_ARG, "p_max too large");
  h->sched.clear();
  if (o.shift_policy == DASHSVD_SHIFT_LEARNED) h->sched.assign((size_t)o.p_max + 1, 0.5);
  if (o.shift_policy == DASHSVD_SHIFT_SCHEDULE) {
    if (!o.schedule) return fail(h, DASHSVD_ERR_INVALID_ARG, "SCHEDULE policy needs options.schedule");
    h->sched.assign(o.schedule, o.schedule + o.p_max + 1);
  }
  o.schedule = nullptr;
  h->tune.clear();
  if (o.tuning_db) {
    if (FILE *f = std::fopen(o.tuning_db, "r")) {
      // lines "key T [lanes slab_kib reorder]" (a line with only T keeps the
      // other knobs at their defaults)
      char line[512];
      while (std::fgets(line, sizeof(line), f)) {
        char key[256];
        TuneVal v;
        const int got = std::sscanf(line, "%255s %d %d %d %d", key, &v.T, &v.vm, &v.slab_kib, &v.reorder);
        if (got < 2 || v.T <= 0) continue;
        if (got < 3 || (v.vm != 1 && v.vm != 2)) v.vm = 1;
        if (got < 4 || v.slab_kib < 0) v.slab_kib = 0;
        if (got < 5 || v.reorder < -1 || v.reorder > 1) v.reorder = 0;
        h->tune.emplace_back(key, v);
      }
      std::fclose(f);
    }
  }
  o.tuning_db = nullptr;
  h->opt = o;
  h->st = (hipStream_t)o.hip_stream;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_create(dashsvd_handle **out, const dashsvd_options *opt) {
  if (!out) return fail(nullptr, DASHSVD_ERR_INVALID_ARG, "null handle pointer");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    (void)hipGetLastError();
    return fail(nullptr, DASHSVD_ERR_HIP, "no HIP device available");
  }
  dashsvd_handle *h = new dashsvd_handle();
  std::memset(&h->info, 0, sizeof(h->info));
  dashsvd_status s = dashsvd_set_options(h, opt);
  if (s != DASHSVD_OK) {
    g_create_error = h->err;
    delete h;
    return s;
  }
  *out = h;
  return DASHSVD_OK;
}

void dashsvd_destroy(dashsvd_handle *h) {
  if (!h) return;
  if (h->ar.base) {
    (void)hipStreamSynchronize(h->st);
    if (h->st2) (void)hipStreamSynchronize(h->st2);
    if (h->stg) (void)hipStreamSynchronize(h->stg);
    if (!h->ar_external) (void)hipFree(h->ar.base);
  }
  for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
  if (h->ev_gram) (void)hipEventDestroy(h->ev_gram);
  if (h->ev_eig) (void)hipEventDestroy(h->ev_eig);
  for (hipEvent_t e : h->ev_flag)
    if (e) (void)hipEventDestroy(e);
  if (h->hflags) (void)hipHostFree(h->hflags);
  if (h->st2) (void)hipStreamDestroy(h->st2);
  if (h->stg) {
    (void)hipStreamSynchronize(h->stg);
    (void)hipStreamDestroy(h->stg);
  }
  if (h->ev_b0) (void)hipEventDestroy(h->ev_b0);
  if (h->ev_b1) (void)hipEventDestroy(h->ev_b1);
  if (h->mlp.P) (void)hipFree(h->mlp.P);
  if (h->mlp.buf) (void)hipFree(h->mlp.buf);
  if (h->ball.base) (void)hipFree(h->ball.base);
  delete h;
}

dashsvd_status dashsvd_set_workspace(dashsvd_handle *h, void *dev_ptr, size_t bytes) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  h->err.clear();
  if (dev_ptr && ((uintptr_t)dev_ptr & 255))
    return fail(h, DASHSVD_ERR_INVALID_ARG, "workspace must start on a 256-byte boundary");
  if (dev_ptr && bytes == 0) return fail(h, DASHSVD_ERR_INVALID_ARG, "workspace of 0 bytes");
  // work still queued may use the current arena
  if (h->ar.base) {
    (void)hipStreamSynchronize(h->st);
    if (h->st2) (void)hipStreamSynchronize(h->st2);
    if (h->stg) (void)hipStreamSynchronize(h->stg);
    if (!h->ar_external) (void)hipFree(h->ar.base);
  }
  h->ar.base = (char *)dev_ptr;
  h->ar.cap = dev_ptr ? bytes : 0;
  h->ar_external = dev_ptr != nullptr;
  // results and evaluation buffers of earlier runs lived in the old arena
  h->have = false;
  h->bat.have = false;
  h->ev_ctx.ok = false;
  return DASHSVD_OK;
}

// SpMM chunk length of a run: the option, else the tuned value of the
// bucket (last entry wins), else the default.
// The tuning database's entry for a shape bucket (the latest one), or null.
static const TuneVal *tuned(const dashsvd_handle *h, const std::string &key) {
  for (auto it = h->tune.rbegin(); it != h->tune.rend(); ++it)
    if (it->first == key) return &it->second;
  return nullptr;
}

static int32_t chunk_length(const dashsvd_handle *h, const std::string &key, int64_t nnz) {
  if (h->opt.long_row > 0) return h->opt.long_row;
  if (const TuneVal *t = tuned(h, key)) return t->T;
  if (nnz < DASHSVD_REORDER_MIN_NNZ) return kDefaultLongRow;
  return h->opt.precision == DASHSVD_PREC_BF16_PANELS ? kDefaultLongRowLargeBf16 : kDefaultLongRowLarge;
}

// SpMM lanes per row: one 16-byte vector per lane (1) or two (2), from the
// option, else the tuning database, else 1.
static int lane_mult(const dashsvd_handle *h, const std::string &key) {
  if (h->opt.lane_vectors > 0) return h->opt.lane_vectors;
  const TuneVal *t = tuned(h, key);
  return t ? t->vm : 1;
}

// Column-slab bytes of the SpMM plan: the option, else the tuning database.
static int64_t slab_bytes(const dashsvd_handle *h, const std::string &key) {
  if (h->opt.slab_kib > 0) return (int64_t)h->opt.slab_kib << 10;
  const TuneVal *t = tuned(h, key);
  return t && t->slab_kib > 0 ? (int64_t)t->slab_kib << 10 : 0;
}

static dashsvd_status check_args(dashsvd_handle *h, const dashsvd_csr *A, int32_t k, int32_t p, double tol) {
  if (!A) return fail(h, DASHSVD_ERR_INVALID_ARG, "null matrix");
  if (A->m < 1 || A->n < 1 || A->nnz < 0) return fail(h, DASHSVD_ERR_INVALID_ARG, "matrix dimensions");
  if (A->m > INT32_MAX || A->n > INT32_MAX || A->nnz > INT32_MAX)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "matrix too large for 32-bit indices");
  if (A->value_dtype != DASHSVD_F32 && A->value_dtype != DASHSVD_F64)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "value_dtype");
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->values)))
    return fail(h, DASHSVD_ERR_INVALID_ARG, "null CSR array");
  if (k < 1) return fail(h, DASHSVD_ERR_INVALID_ARG, "k must be >= 1");
  if (p < 1) return fail(h, DASHSVD_ERR_INVALID_ARG, "oversampling must be >= 1 (the check reads S_{k+1})");
  const int64_t mn = A->m < A->n ? A->m : A->n;
  if ((int64_t)k + p > mn) return fail(h, DASHSVD_ERR_INVALID_ARG, "k + oversampling exceeds min(m, n)");
  if (k + p > DASHSVD_MAX_L) return fail(h, DASHSVD_ERR_INVALID_ARG, "k + oversampling exceeds DASHSVD_MAX_L");
  if (!(tol >= 0.0) || std::isinf(tol)) return fail(h, DASHSVD_ERR_INVALID_ARG, "tol must be finite and >= 0");
  return DASHSVD_OK;
}

dashsvd_status dashsvd_workspace_size(const dashsvd_csr *A, int32_t k, int32_t p, int32_t precision,
                                      size_t *bytes);

static dashsvd_status run_impl(dashsvd_handle *h, const dashsvd_csr *A, int32_t k, int32_t p, double tol,
                               bool measure_only, size_t *measured) {
  const double t0 = now_ms();
  const int prec = h->opt.precision;
  const int vdt = prec == DASHSVD_PREC_FP64 ? DASHSVD_F64 : DASHSVD_F32;  // compute value type
  const int pdt = prec == DASHSVD_PREC_FP64 ? DASHSVD_F64 : (prec == DASHSVD_PREC_BF16_PANELS ? DASHSVD_BF16 : DASHSVD_F32);
  const int cdt = prec == DASHSVD_PREC_FP64 ? DASHSVD_F64 : DASHSVD_F32;  // C, B, U, V type
  const size_t accsz = prec == DASHSVD_PREC_FP64 ? 8 : 4;
  const int64_t m = A->m, n = A->n, nnz = A->nnz;
  const bool wide = m < n;
  const int64_t Mm = wide ? n : m, Mn = wide ? m : n;
  const int l = k + p;
  // Panel rows: the SpMM's lanes cover ldc = l rounded up to 8 columns.  The
  // leading dimension ld starts every row on a 128-byte boundary where that
  // costs at most 1/8 more memory, so a gathered row touches fewer cache
  // lines (480-byte FP32 rows at l = 120: 4 lines each instead of 4.5 on
  // average; 240-byte BF16 rows: 2 instead of 2.75).
  const int ldc = (int)round_up(l, 8);
  const int64_t line_elems = (int64_t)(128 / (dsz(pdt) < dsz(cdt) ? dsz(pdt) : dsz(cdt)));
  const int ld = round_up(l, line_elems) * 8 <= (int64_t)ldc * 9 ? (int)round_up(l, line_elems) : ldc;
  const std::string tkey = tune_key(prec, ldc, Mm, nnz, false);
  const int32_t T = chunk_length(h, tkey, nnz);
  const int vm = lane_mult(h, tkey);
  const int pmax = h->opt.p_max;
  const int cap = pmax > 0 ? pmax : 1;
  hipStream_t st = h->st;

  // ---------------------------------------------------------------- arena
  Arena &ar = h->ar;
  RunBufs b;
  ar.reset(measure_only || ar.base == nullptr);
  if (!measure_only) {
    size_t need = 0;
    run_impl(h, A, k, p, tol, true, &need);
    dashsvd_status s = ensure_arena(h, need);
    if (s != DASHSVD_OK) return s;
    ar.reset(false);
  }
  h->have = false;
  h->bat.have = false;
  const bool need_copy_struct = !A->on_device;
  const bool need_copy_val = !A->on_device || A->value_dtype != vdt;
  int64_t *rp_in = need_copy_struct ? (int64_t *)ar.take(8 * (size_t)(m + 1)) : nullptr;
  int32_t *col_in = need_copy_struct ? (int32_t *)ar.take(4 * (size_t)(nnz + 1)) : nullptr;
  void *val_raw = !A->on_device ? ar.take(dsz(A->value_dtype) * (size_t)(nnz + 1)) : nullptr;
  void *val_in = need_copy_val ? ar.take(dsz(vdt) * (size_t)(nnz + 1)) : nullptr;
  b.rpT = (int64_t *)ar.take(8 * (size_t)(n + 1));
  b.colT = (int32_t *)ar.take(4 * (size_t)(nnz + 1));
  b.valT = ar.take(dsz(vdt) * (size_t)(nnz + 1));
  b.rowidx = (int32_t *)ar.take(4 * (size_t)(nnz + 1));
  b.flags = (int32_t *)ar.take(4 * 8);
  b.sizes = (int64_t *)ar.take(8 * 6);
  b.tws_bytes = transpose_ws_bytes(n, nnz);
  b.tws = ar.take(b.tws_bytes);
  const int64_t scan_n = (m > n ? m : n) + 1;
  b.scan_tmp = (int64_t *)ar.take(8 * scan_tmp_elems(scan_n));
  // long-row chunks cut at slabs of the gathered panel: M gathers rows of
  // the n-side panels (C, Q), M^T rows of the m-side ones (Z, Y)
  const int64_t prow_b = (int64_t)ld * (int64_t)dsz(pdt);
  const int64_t slab_b = slab_bytes(h, tkey);
  const TuneVal *tv = tuned(h, tkey);
  const bool reorder = h->opt.reorder == DASHSVD_REORDER_ON ||
                       (h->opt.reorder == DASHSVD_REORDER_AUTO &&
                        (tv && tv->reorder ? tv->reorder > 0 : nnz >= DASHSVD_REORDER_MIN_NNZ));
  // dense heads of M and M^T: only in the degree order (the head is then a
  // prefix of the rows), and for panels whose rows fit the head kernels
  const int head_t = prec == DASHSVD_PREC_FP64 ? 1 : 0;
  const bool heads = reorder && h->opt.dense_head != DASHSVD_HEAD_OFF && ldc <= kHeadMaxCols &&
                     head_fits(Mn > Mm ? Mn : Mm, ld, cdt, ldc);
  plan_alloc(h, ar, b.planM, Mm, nnz, T, ldc, accsz, Mn, prow_b, slab_b, heads ? head_t : -1);
  plan_alloc(h, ar, b.planT, Mn, nnz, T, ldc, accsz, Mm, prow_b, slab_b, heads ? head_t : -1);
  b.Y = ar.take(dsz(pdt) * (size_t)Mm * ld);
  b.Q = ar.take(dsz(pdt) * (size_t)Mn * ld);
  b.C = ar.take(dsz(cdt) * (size_t)Mn * ld);
  b.B = pdt == cdt ? b.Y : ar.take(dsz(cdt) * (size_t)Mm * ld);
  b.Z = ar.take(dsz(cdt) * (size_t)Mm * ld);
  b.X = pdt == cdt ? ar.take(dsz(cdt) * (size_t)Mn * ld) : nullptr;
  // BF16 panels: FP32 panels for the passes after a promotion
  b.Q32 = pdt != cdt ? ar.take(dsz(cdt) * (size_t)Mn * ld) : nullptr;
  b.Y32 = pdt != cdt ? ar.take(dsz(cdt) * (size_t)Mm * ld) : nullptr;
  const int nb_n = gram_blocks(Mn, l), nb_m = gram_blocks(Mm, l);
  b.gpart = (double *)ar.take(8 * gram_partial_elems(nb_n > nb_m ? nb_n : nb_m, l));
  b.G = (double *)ar.take(8 * (size_t)l * l);
  b.W = (double *)ar.take(8 * (size_t)l * l);
  b.Vs = (double *)ar.take(8 * (size_t)l * l);
  b.G2 = (double *)ar.take(8 * (size_t)l * l);
  b.T2 = (double *)ar.take(8 * (size_t)l * l);
  b.W2 = (double *)ar.take(8 * (size_t)l * l);
  b.PU = (double *)ar.take(8 * (size_t)l * l);
  b.PV = (double *)ar.take(8 * (size_t)l * l);
  b.S = (double *)ar.take(8 * (size_t)l);
  b.Sprev = (double *)ar.take(8 * (size_t)l);
  b.Sb = (double *)ar.take(8 * (size_t)l);
  b.Ebp = (double *)ar.take(8 * (size_t)l);
  b.state = (SolverState *)ar.take(sizeof(SolverState));
  b.tri_ws = (double *)ar.take(kTriWsBytes);
  b.tr_alpha = (double *)ar.take(8 * (size_t)cap);
  b.tr_ratio = (double *)ar.take(8 * (size_t)cap);
  b.tr_s = (double *)ar.take(8 * (size_t)cap * l);
  b.tr_sweeps = (int32_t *)ar.take(4 * (size_t)(cap + 2));
  b.sched = (double *)ar.take(8 * (size_t)(pmax + 2));
  b.Uo = ar.take(dsz(cdt) * (size_t)Mm * k);
  b.Vo = ar.take(dsz(cdt) * (size_t)Mn * k);
  const int sgn_blk = 1024;  // blocks of the column-maximum search of the sign step
  b.sgn_max = ar.take(8 * (size_t)sgn_blk * k);
  b.sgn_idx = ar.take(8 * (size_t)sgn_blk * k + 4 * (size_t)k);
  if (h->opt.omega && !h->opt.omega_on_device)
    b.omega_dev = ar.take(dsz(h->opt.omega_dtype) * (size_t)Mm * l);
  if (reorder) {
    b.perm_r = (int32_t *)ar.take(4 * (size_t)(m + 1));
    b.inv_r = (int32_t *)ar.take(4 * (size_t)(m + 1));
    b.perm_c = (int32_t *)ar.take(4 * (size_t)(n + 1));
    b.inv_c = (int32_t *)ar.take(4 * (size_t)(n + 1));
    b.rpP = (int64_t *)ar.take(8 * (size_t)(m + 1));
    b.rpPT = (int64_t *)ar.take(8 * (size_t)(n + 1));
    b.colP = (int32_t *)ar.take(4 * (size_t)(nnz + 1));
    b.valP = ar.take(dsz(vdt) * (size_t)(nnz + 1));
    b.dws_bytes = degree_order_ws_bytes(m > n ? m : n);
    b.dws = ar.take(b.dws_bytes);
  }
  if (measure_only) {
    *measured = ar.used;
    return DASHSVD_OK;
  }

  // ---------------------------------------------------------------- setup
  h->marks.clear();
  h->ev_used = 0;
  h->open_group = -1;
  if (!h->st2) {
    HIPCHK(hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&h->ev_gram, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_eig, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_flag[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_flag[1], hipEventDisableTiming));
    HIPCHK(hipHostMalloc((void **)&h->hflags, kPinBytes, hipHostMallocDefault));
  }
  hipStream_t st2 = h->st2;
  // Omega (Alg. 5 step 1) depends on nothing but the row order: it is
  // formed on the second stream while the main stream validates, transposes
  // and reorders the CSR (the second stream first waits for the main
  // stream's work so far, which may still read the panel Omega is written
  // to).  With the degree order, Omega is drawn in the caller's row order
  // and row r is stored in row row_to[r] of the panel.
  auto launch_omega = [&](const int32_t *row_to) -> hipError_t {
    hipError_t e = hipEventRecord(h->ev_gram, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st2, h->ev_gram, 0);
    if (e != hipSuccess) return e;
    if (h->opt.omega) {
      const void *src = h->opt.omega;
      if (!h->opt.omega_on_device) {
        e = hipMemcpyAsync(b.omega_dev, h->opt.omega, dsz(h->opt.omega_dtype) * (size_t)Mm * l,
                           hipMemcpyHostToDevice, st2);
        if (e != hipSuccess) return e;
        src = b.omega_dev;
      }
      e = launch_copy2d(src, l, h->opt.omega_dtype, b.Y, ld, pdt, Mm, l, st2, row_to);
    } else {
      e = launch_gaussian(h->opt.seed, Mm, l, b.Y, ld, pdt, st2, row_to);
    }
    if (e == hipSuccess) e = hipEventRecord(h->ev_eig, st2);
    return e;
  };
  if (!reorder) HIPCHK(launch_omega(nullptr));
  // control buffers start at zero; panels need no clearing (pad columns are
  // never read into the first l columns)
  {
    ZeroRanges z{};
    z.add(b.flags, 4 * 8);
    z.add(b.planM.nlong, 16);
    z.add(b.planT.nlong, 16);
    z.add(b.planM.slab_cnt, 8 * (size_t)(kMaxSlabs + 1));
    z.add(b.planT.slab_cnt, 8 * (size_t)(kMaxSlabs + 1));
    z.add(b.state, sizeof(SolverState));
    z.add(b.Sprev, 8 * (size_t)l);
    z.add(b.Ebp, 8 * (size_t)l);
    z.add(b.tr_alpha, 8 * (size_t)cap);
    z.add(b.tr_ratio, 8 * (size_t)cap);
    z.add(b.tr_sweeps, 4 * (size_t)(cap + 2));
    HIPCHK(launch_zero_ranges(z, st));
  }
  const int64_t *rpA = A->on_device ? A->row_ptr : rp_in;
  const int32_t *colA = A->on_device ? A->col_idx : col_in;
  const int64_t *rpAT = b.rpT;
  const int32_t *colAT = b.colT;
  const void *valAT = b.valT;
  const void *val_src = A->on_device ? A->values : val_raw;
  if (!A->on_device) {
    HIPCHK(hipMemcpyAsync(rp_in, A->row_ptr, 8 * (size_t)(m + 1), hipMemcpyHostToDevice, st));
    if (nnz > 0) {
      HIPCHK(hipMemcpyAsync(col_in, A->col_idx, 4 * (size_t)nnz, hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(val_raw, A->values, dsz(A->value_dtype) * (size_t)nnz, hipMemcpyHostToDevice, st));
    }
  }
  const void *valA = val_src;
  if (need_copy_val) {
    HIPCHK(launch_convert(val_src, A->value_dtype, val_in, vdt, nnz, st));
    valA = val_in;
  }
  tmark_begin(h, DASHSVD_KT_TRANSPOSE, 0);
  HIPCHK(launch_validate(m, n, nnz, rpA, colA, valA, vdt, b.rowidx, b.flags, st));
  int32_t *hflags = h->hflags + 32;  // pinned
  HIPCHK(hipMemcpyAsync(hflags, b.flags, 16, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflags[0] & 3) (void)hipStreamSynchronize(st2);  // Omega's writes end before the arena is reused
  if (hflags[0] & 1) return fail(h, DASHSVD_ERR_BAD_CSR, "row_ptr/col_idx malformed");
  if (hflags[0] & 2) return fail(h, DASHSVD_ERR_NONFINITE, "NaN or Inf among the values");
  // CSR(A^T): the sort of the column keys gives its row pointer
  HIPCHK(launch_transpose_keys(n, nnz, colA, b.rpT, b.tws, b.tws_bytes, st, b.rowidx, valA, vdt));
  if (reorder) {
    // degree order of the rows (from the row pointer of A) and of the
    // columns (from that of A^T); the transposed entries are gathered
    // straight into the permuted A^T, and A's entries move to the permuted A
    HIPCHK(launch_degree_order(m, rpA, n, b.perm_r, b.inv_r, b.rpP, b.dws, b.dws_bytes, b.scan_tmp, st));
    HIPCHK(launch_degree_order(n, b.rpT, m, b.perm_c, b.inv_c, b.rpPT, b.dws, b.dws_bytes, b.scan_tmp, st));
    HIPCHK(launch_omega(wide ? b.inv_c : b.inv_r));
    HIPCHK(launch_transpose_gather(nnz, b.rowidx, valA, vdt, b.tws, b.colT, b.valT, st, b.rpT, b.inv_r, b.inv_c,
                                   b.rpPT));
    HIPCHK(launch_permute_entries(nnz, rpA, b.rowidx, 0, colA, valA, vdt, b.inv_r, b.inv_c, b.rpP, b.colP, b.valP,
                                  st));
    rpA = b.rpP;
    colA = b.colP;
    valA = b.valP;
    rpAT = b.rpPT;
  } else {
    HIPCHK(launch_transpose_gather(nnz, b.rowidx, valA, vdt, b.tws, b.colT, b.valT, st));
  }
  tmark_end(h);
  // M and M^T
  const int64_t *rpM = wide ? rpAT : rpA;
  const int32_t *colM = wide ? colAT : colA;
  const void *valM = wide ? valAT : valA;
  const int64_t *rpMT = wide ? rpA : rpAT;
  const int32_t *colMT = wide ? colA : colAT;
  const void *valMT = wide ? valA : valAT;
  // rows of M and of M^T: where row i of the solver's U and V goes in the
  // caller's order (null without the degree order)
  const int32_t *mapM = reorder ? (wide ? b.perm_c : b.perm_r) : nullptr;
  const int32_t *mapN = reorder ? (wide ? b.perm_r : b.perm_c) : nullptr;
  // dense heads: the leading rows with at least max(T + 1, columns / 16)
  // nonzeros (the plans leave them out)
  if (b.planM.head_dev)
    HIPCHK(launch_head_count(Mm, rpM, std::max<int64_t>(T + 1, (Mn + 15) / 16), kHeadNnzPerCol * Mn,
                             b.planM.head_dev, st));
  if (b.planT.head_dev)
    HIPCHK(launch_head_count(Mn, rpMT, std::max<int64_t>(T + 1, (Mm + 15) / 16), kHeadNnzPerCol * Mm,
                             b.planT.head_dev, st));
  // SpMM plans
  HIPCHK(plan_build(b.planM, rpM, colM, T, b.scan_tmp, st));
  HIPCHK(plan_build(b.planT, rpMT, colMT, T, b.scan_tmp, st));
  // the four plan sizes in one device buffer (the scan workspace is free
  // again), one copy to pinned memory, one wait
  int64_t *sizes_d = b.sizes;
  int64_t *sizes_h = (int64_t *)(h->hflags + 16);
  HIPCHK(launch_plan_sizes(b.planM.off + b.planM.R, b.planT.off + b.planT.R, b.planM.nlong, b.planT.nlong,
                           b.planM.head_dev, b.planT.head_dev, sizes_d, st));
  HIPCHK(hipMemcpyAsync(sizes_h, sizes_d, 48, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  b.planM.n_chunks = sizes_h[0];
  b.planT.n_chunks = sizes_h[1];
  b.planM.n_long = (int32_t)sizes_h[2];
  b.planT.n_long = (int32_t)sizes_h[3];
  b.planM.head = (int32_t)sizes_h[4];
  b.planT.head = (int32_t)sizes_h[5];
  // Dt of each head from its first rows
  if (b.planM.head > 0)
    HIPCHK(launch_head_build(Mn, rpM, colM, valM, vdt, b.planM.head, b.planM.dt, b.planM.head_t, st));
  if (b.planT.head > 0)
    HIPCHK(launch_head_build(Mm, rpMT, colMT, valMT, vdt, b.planT.head, b.planT.dt, b.planT.head_t, st));
  if (!h->sched.empty())
    HIPCHK(hipMemcpyAsync(b.sched, h->sched.data(), 8 * h->sched.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamWaitEvent(st, h->ev_eig, 0));  // Omega is ready
  const double t_setup = now_ms();  // host time: the setup kernels may still run

  // ---------------------------------------------------------------- eigSVD pieces
  // Sketch and pass blocks: the tridiagonal eigensolver, Cholesky-QR with
  // eigenvalues, one-sided or two-sided Jacobi (the two-sided kernel where
  // the others decline).  Cholesky-QR keeps the span but not the principal
  // (Ritz) basis, and the next block C = A Q of a non-principal Q has nearly
  // collinear columns whose FP32 storage loses the small directions by about
  // eps kappa(C).  The last two blocks before the final step fix the
  // accuracy of its products, so they are always Jacobi: CHOLQR switches to
  // Jacobi after the first pass whose PVE ratio is within kCqSwitch x tol
  // (set on the device by the pass tail), and for the blocks of passes
  // p_max - 1 and p_max.
  // AUTO: TRIDIAG in the FP32 and BF16 forms, CHOLQR in the FP64 form
  const int meth = h->opt.eig_method != DASHSVD_EIG_AUTO ? h->opt.eig_method
                   : prec == DASHSVD_PREC_FP64         ? DASHSVD_EIG_CHOLQR
                                                       : DASHSVD_EIG_TRIDIAG;
  const bool cholqr = meth == DASHSVD_EIG_CHOLQR;
  // ONESIDED: one-sided Jacobi on the Cholesky factor (l <= 128), the
  // two-sided kernel where it declines
  const bool onesided = meth == DASHSVD_EIG_ONESIDED && l <= 128;
  // TRIDIAG: the tridiagonal eigensolver (l <= kTriMaxL), the two-sided
  // kernel where it declines
  const bool tridiag = meth == DASHSVD_EIG_TRIDIAG && l <= kTriMaxL && prec != DASHSVD_PREC_FP64;
  auto eig_solve = [&](const EigArgs &ea, hipStream_t s) -> hipError_t {
    const bool tri = tridiag && ea.Vs && ea.W;
    if (!onesided && !tri) return launch_eig(ea, s);
    EigArgs e1 = ea;
    e1.decline = &b.state->j1_decline;
    e1.tri_ws = b.tri_ws;
    hipError_t e = tri ? launch_eigtri(e1, s) : launch_eig1s(e1, s);
    if (e != hipSuccess) return e;
    EigArgs e2 = ea;
    e2.run_if = &b.state->j1_decline;
    return launch_eig(e2, s);
  };
  constexpr double kCqSwitch = 100.0;
  const bool nosurr = h->opt.pve_mode == DASHSVD_PVE_NOSURR;
  auto make_eig = [&](int mode) {
    EigArgs ea;
    std::memset(&ea, 0, sizeof(ea));
    ea.l = l;
    ea.k = k;
    // Jacobi stops when every |g_pq| <= skip sqrt(g_pp g_qq).  V is a
    // product of rotations, so Q = C V S^-1 then has Q^T Q = I + E with
    // |E_pq| <= skip whatever the eigenvalue gaps, and the eigenvalues are
    // off by O(skip^2).  FP64 form: half an ulp; FP32 / BF16 panels store Q
    // with 2^-24 relative rounding, so 2^-23 is below what they hold.
    ea.skip = prec == DASHSVD_PREC_FP64 ? 0x1.0p-53 : 0x1.0p-23;
    ea.G = b.G;
    ea.S = b.S;
    ea.Vs = b.Vs;
    ea.W = b.W;
    ea.state = b.state;
    ea.mode = mode;
    ea.pve_mode = h->opt.pve_mode;
    ea.policy = h->opt.shift_policy;
    // without the surrogate, the pass tail only updates the shift; the
    // check of sigma(M Q) decides termination
    ea.tol = nosurr ? 0.0 : tol;
    ea.Sprev = b.Sprev;
    ea.trace_alpha = b.tr_alpha;
    ea.trace_ratio = b.tr_ratio;
    ea.trace_s = b.tr_s;
    ea.trace_cap = cap;
    ea.trace_sweeps = b.tr_sweeps;
    ea.cq_switch = cholqr ? kCqSwitch : 0.0;
    ea.sched = h->sched.empty() ? nullptr : b.sched;
    ea.sched_len = (int)h->sched.size();
    if (h->opt.shift_policy == DASHSVD_SHIFT_LEARNED && h->mlp.ok) {
      ea.mlp = h->mlp.P;
      ea.mlp_D = h->mlp.D;
      ea.mlp_H = h->mlp.H;
      ea.mlp_cmax = h->mlp.cmax;
      ea.shape_feat[0] = std::log((double)Mm);
      ea.shape_feat[1] = std::log((double)Mn);
      ea.shape_feat[2] = std::log((double)(nnz > 0 ? nnz : 1) / (double)Mm);
    }
    return ea;
  };
  const int32_t *done = &b.state->done;
  const int32_t *pass_skip = &b.state->pass_skip;
  const int every = h->opt.check_interval > 0 ? h->opt.check_interval : 1;
  // Host copy of state->cq_off (read with done at each stop test): once set,
  // the pass blocks go straight to the Jacobi eigensolver.
  int32_t host_cq_off = 0;
  auto launch_block_eig = [&](EigArgs &ea, int pass, hipStream_t s) -> hipError_t {
    const bool cq = cholqr && !host_cq_off && pass + 1 < pmax;
    if (!cq) {
      tmark_begin(h, DASHSVD_KT_EIG, pass, s);
      const hipError_t e = eig_solve(ea, s);
      tmark_end(h, s);
      return e;
    }
    // Cholesky-QR, then the Jacobi eigensolver gated on its hand-over or
    // decline (each timed in its own group)
    tmark_begin(h, DASHSVD_KT_CHOLQR, pass, s);
    hipError_t e = launch_cholqr(ea, s);
    tmark_end(h, s);
    if (e != hipSuccess) return e;
    EigArgs gated = ea;
    gated.run_if = &b.state->cq_fallback;
    tmark_begin(h, DASHSVD_KT_EIG, pass, s);
    e = eig_solve(gated, s);
    tmark_end(h, s);
    return e;
  };
  // Stop test one chunk behind (both pass orders): the flags of a chunk are
  // copied to pinned host memory behind its work, and the host reads them
  // only once the next chunk is queued, so the GPU does not idle while the
  // host decides; a chunk queued after the stop returns at the first
  // instruction of each kernel.
  struct Flags {  // copy of SolverState from `ratio` to `cq_off`, then `stagnant` and `promote`
    double ratio;
    int32_t pass, done, cq_off, stagnant, promote, pad;
  };
  static_assert(offsetof(SolverState, pass) == offsetof(SolverState, ratio) + 8 &&
                    offsetof(SolverState, done) == offsetof(SolverState, ratio) + 12 &&
                    offsetof(SolverState, cq_off) == offsetof(SolverState, ratio) + 16 &&
                    offsetof(SolverState, promote) == offsetof(SolverState, stagnant) + 4,
                "flag copy layout");
  // two slots in front of the plan sizes (bytes 64..95 of the pinned area)
  static_assert(2 * sizeof(Flags) <= 64, "flag slots");
  Flags *hf = reinterpret_cast<Flags *>(h->hflags);
  double r_old = 0.0, r_new = 0.0;  // the last two ratios read
  bool stop = false;
  bool promote_read = false;  // BF16 panels: the pass tail asked for FP32 panels
  int stagnant_read = 0;      // BF16 panels: flat passes so far (2 ask for FP32)
  int stop_pass = 0;  // passes executed, as read with the stop flag
  auto copy_flags = [&](int slot, hipStream_t s) -> hipError_t {
    hipError_t e = hipMemcpyAsync(&hf[slot], &b.state->ratio, 20, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&hf[slot].stagnant, &b.state->stagnant, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(h->ev_flag[slot], s);
    return e;
  };
  auto read_slot = [&](int slot) -> hipError_t {
    const hipError_t e = hipEventSynchronize(h->ev_flag[slot]);
    if (e != hipSuccess) return e;
    host_cq_off = hf[slot].cq_off;
    stop = hf[slot].done != 0;
    stop_pass = hf[slot].pass;
    promote_read = hf[slot].promote != 0;
    stagnant_read = hf[slot].stagnant;
    r_old = r_new;
    r_new = hf[slot].ratio;
    return hipSuccess;
  };
  int32_t eig_launches = 0;  // eigensolver calls launched beside the SpMMs (signal index)
  int last_pass = 0;  // passes whose eigSVD ran (the final block's C, Z, W)
  int promoted = 0;   // BF16 panels switched to FP32 by the stagnation guard
  void *Qfin = b.Q, *Yfin = b.Y;  // final Q and M Q (plain order)
  int pfin = pdt;
  if (pdt == cdt) {
    // Overlapped order (FP32 and FP64 forms).  With C the current block and
    // W its eigSVD weights (Q = C W), the next pass is
    //   Y+ = M Q = (M C) W = Z W,  C+ = M^T Y+ - alpha Q = (M^T Z - alpha C) W,
    // so both products of the next pass, Z = M C and X = M^T Z, need only C
    // and run on the main stream while the eigensolver works on the second
    // one; after it, one rescale forms C+ = (X - alpha C) W with the updated
    // shift.  Q and Y are formed only for the final Rayleigh-Ritz step.
    void *Cb[2] = {b.C, b.Q};
    auto side = [&](int mode, int pass, void *Cin, const int32_t *gate) -> hipError_t {
      tmark_begin(h, DASHSVD_KT_GRAM, pass);
      hipError_t e = launch_gram(Mn, l, Cin, ld, cdt, b.gpart, nb_n, b.G, gate, st, (int32_t *)pass_skip);
      tmark_end(h);
      if (e != hipSuccess) return e;
      EigArgs ea = make_eig(mode);
      ea.call_idx = ++eig_launches;
      const int32_t *skip = gate ? pass_skip : nullptr;
      if ((e = hipEventRecord(h->ev_gram, st)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(st2, h->ev_gram, 0)) != hipSuccess) return e;
      e = launch_block_eig(ea, pass, st2);
      if (e != hipSuccess) return e;
      if ((e = hipEventRecord(h->ev_eig, st2)) != hipSuccess) return e;
      // The eigensolver needs whole CUs (1024 threads); the SpMMs would take
      // every CU first, so they wait (bounded) until it is resident.
      if ((e = launch_wait_started(&b.state->eig_started, ea.call_idx, st)) != hipSuccess) return e;
      tmark_begin(h, DASHSVD_KT_SPMM, pass);
      e = plan_spmm(b.planM, Mm, rpM, colM, valM, vdt, Cin, ld, cdt, b.Z, ld, cdt, ldc, T, vm, nullptr, 0, nullptr,
                    skip, st);
      tmark_end(h);
      if (e != hipSuccess) return e;
      tmark_begin(h, DASHSVD_KT_SPMM_T, pass);
      // X = M^T Z feeds only the next pass: when the eigensolver of this
      // block stops the iteration before the product's workgroups start,
      // they return at once (the live flag, not the pass-start snapshot;
      // Z above is kept, the final step uses it)
      e = plan_spmm(b.planT, Mn, rpMT, colMT, valMT, vdt, b.Z, ld, cdt, b.X, ld, cdt, ldc, T, vm, nullptr, 0, nullptr,
                    gate, st);
      tmark_end(h);
      if (e != hipSuccess) return e;
      return hipStreamWaitEvent(st, h->ev_eig, 0);
    };
    // Accuracy control without the surrogate (Sec. 4.3): sigma(B) of
    // B = M Q = Z W after the pass, from B^T B = W^T (Z^T Z) W (the final
    // step's identity), its eigenvalues by the Jacobi kernel, then eq. (18)
    // on their squares.  On the main stream after the pass's eigensolver,
    // so a stop leaves C, Z and W of the stopping pass for the final step.
    auto check_nosurr = [&](int pass) -> hipError_t {
      tmark_begin(h, DASHSVD_KT_CHECK, pass);
      hipError_t e = launch_gram(Mm, l, b.Z, ld, cdt, b.gpart, nb_m, b.G2, pass_skip, st, nullptr);
      if (e == hipSuccess) e = launch_small_gemm(l, l, l, b.G2, l, 0, b.W, l, b.T2, l, st);
      if (e == hipSuccess) e = launch_small_gemm(l, l, l, b.W, l, 1, b.T2, l, b.PU, l, st);
      if (e == hipSuccess) {
        EigArgs ev;
        std::memset(&ev, 0, sizeof(ev));
        ev.l = l;
        ev.k = k;
        ev.skip = prec == DASHSVD_PREC_FP64 ? 0x1.0p-53 : 0x1.0p-23;
        ev.G = b.PU;
        ev.S = b.Sb;
        ev.W = b.W2;
        ev.skip_if = pass_skip;
        e = eig_solve(ev, st);
      }
      if (e == hipSuccess)
        e = launch_pve_nosurr(k, l, b.Sb, b.Ebp, tol, cholqr ? kCqSwitch : 0.0, b.state, b.tr_ratio, cap, pass_skip,
                              st);
      tmark_end(h);
      return e;
    };
    // sketch (Alg. 5 step 2): C = M^T Omega, its eigSVD || M C, M^T M C
    tmark_begin(h, DASHSVD_KT_SKETCH, 0);
    HIPCHK(plan_spmm(b.planT, Mn, rpMT, colMT, valMT, vdt, b.Y, ld, pdt, Cb[0], ld, cdt, ldc, T, vm, nullptr, 0,
                     nullptr, nullptr, st));
    tmark_end(h);
    HIPCHK(side(1, 0, Cb[0], nullptr));
    // power passes (steps 3-8), the stop test one chunk behind.
    // When the ratios read so far predict that the chunk just queued meets
    // tol, the host waits for that chunk's flags instead (one host round
    // trip, against a whole chunk of launches that would return at once).
    int launched = 0;
    int pending = -1;  // flag slot copied but not read yet
    while (launched < pmax) {
      const int chunk = (pmax - launched) < every ? (pmax - launched) : every;
      for (int c = 0; c < chunk; ++c) {
        const int pass = launched + c + 1;
        tmark_begin(h, DASHSVD_KT_RESCALE, pass);
        HIPCHK(launch_rescale(Mn, l, b.X, ld, cdt, b.W, l, l, Cb[pass & 1], ld, cdt, done, st, Cb[(pass - 1) & 1],
                              &b.state->alpha));
        tmark_end(h);
        HIPCHK(side(2, pass, Cb[pass & 1], done));
        if (nosurr) HIPCHK(check_nosurr(pass));
      }
      launched += chunk;
      if (!(tol > 0.0 && launched < pmax)) continue;
      const int slot = pending == 0 ? 1 : 0;
      HIPCHK(copy_flags(slot, st));
      if (pending >= 0) {
        HIPCHK(read_slot(pending));
        if (stop) break;
      }
      pending = slot;
      // geometric extrapolation of the ratio over the chunk just queued
      if (r_old > 0.0 && r_new > 0.0 && r_new < r_old) {
        const double q = r_new / r_old;
        double pred = r_new;
        for (int c = 0; c < chunk; ++c) pred *= q;
        if (pred <= 1.5 * tol) {
          HIPCHK(read_slot(slot));
          pending = -1;
          if (stop) break;
        }
      }
    }
    if (stop) {
      // no pass runs after the flag is set: the count read with it is final
      last_pass = stop_pass;
    } else {
      HIPCHK(hipMemcpyAsync(&last_pass, &b.state->pass, 4, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
  } else {
    // Plain order (BF16 panels): C = M^T Y - alpha Q from the BF16 panels,
    // G = C^T C, eig, Q = C W, Y = M Q.  Stagnation guard: once the PVE
    // ratio has gained less than 20 % per pass for two passes while above
    // tol, the BF16 rounding of the panels limits the attainable accuracy, and the
    // remaining passes run with FP32 panels (Q = C W of the last block,
    // formed again in FP32, and Y = M Q).
    void *Qc = b.Q, *Yc = b.Y;
    int pcur = pdt;
    auto block_step = [&](int mode, int pass, const int32_t *gate) -> hipError_t {
      tmark_begin(h, DASHSVD_KT_GRAM, pass);
      hipError_t e = launch_gram(Mn, l, b.C, ld, cdt, b.gpart, nb_n, b.G, gate, st, (int32_t *)pass_skip);
      tmark_end(h);
      if (e != hipSuccess) return e;
      EigArgs ea = make_eig(mode);
      ea.stagnation_guard = pcur == DASHSVD_BF16;
      const int32_t *skip = gate ? pass_skip : nullptr;
      e = launch_block_eig(ea, pass, st);
      if (e != hipSuccess) return e;
      tmark_begin(h, DASHSVD_KT_RESCALE, pass);
      e = launch_rescale(Mn, l, b.C, ld, cdt, b.W, l, l, Qc, ld, pcur, skip, st);
      tmark_end(h);
      if (e != hipSuccess) return e;
      tmark_begin(h, DASHSVD_KT_SPMM, pass);
      e = plan_spmm(b.planM, Mm, rpM, colM, valM, vdt, Qc, ld, pcur, Yc, ld, pcur, ldc, T, vm, nullptr, 0, nullptr,
                    skip, st);
      tmark_end(h);
      return e;
    };
    // sketch (Alg. 5 step 2): C = M^T Omega ; Q = eigSVD(C).U ; Y = M Q
    tmark_begin(h, DASHSVD_KT_SKETCH, 0);
    HIPCHK(plan_spmm(b.planT, Mn, rpMT, colMT, valMT, vdt, b.Y, ld, pdt, b.C, ld, cdt, ldc, T, vm, nullptr, 0, nullptr,
                     nullptr, st));
    tmark_end(h);
    HIPCHK(block_step(1, 0, nullptr));
    // power passes (steps 3-8): C = M^T Y - alpha Q ; eigSVD(C) ; check ;
    // shift; the stop test one chunk behind, as in the overlapped order.  A
    // request for FP32 panels follows a flat pass: once the flags read show
    // one, the host reads the chunk just queued at once, so the panels
    // switch before the next chunk, as with a read after every chunk.
    int launched = 0;
    int pending = -1;  // flag slot copied but not read yet
    auto promote_now = [&]() -> hipError_t {
      pcur = cdt;
      Qc = b.Q32;
      Yc = b.Y32;
      promoted = 1;
      // not gated on the stop flag: when the chunk queued behind the request
      // stopped, the final step reads these FP32 panels (Q = C W of its
      // last block, as its BF16 ones)
      hipError_t e = launch_rescale(Mn, l, b.C, ld, cdt, b.W, l, l, Qc, ld, pcur, nullptr, st);
      if (e == hipSuccess)
        e = plan_spmm(b.planM, Mm, rpM, colM, valM, vdt, Qc, ld, pcur, Yc, ld, pcur, ldc, T, vm, nullptr, 0, nullptr,
                      nullptr, st);
      return e;
    };
    while (launched < pmax) {
      const int chunk = (pmax - launched) < every ? (pmax - launched) : every;
      for (int c = 0; c < chunk; ++c) {
        const int pass = launched + c + 1;
        tmark_begin(h, DASHSVD_KT_SPMM_T, pass);
        HIPCHK(plan_spmm(b.planT, Mn, rpMT, colMT, valMT, vdt, Yc, ld, pcur, b.C, ld, cdt, ldc, T, vm, Qc, ld,
                         &b.state->alpha, done, st));
        tmark_end(h);
        HIPCHK(block_step(2, pass, done));
      }
      launched += chunk;
      if (!(tol > 0.0 && launched < pmax)) continue;
      const int slot = pending == 0 ? 1 : 0;
      HIPCHK(copy_flags(slot, st));
      if (pending >= 0) {
        HIPCHK(read_slot(pending));
        if (stop) break;
        if (promote_read && pcur == DASHSVD_BF16) HIPCHK(promote_now());
      }
      pending = slot;
      // geometric extrapolation of the ratio over the chunk just queued, or
      // a flat pass before it (the chunk may ask for FP32 panels)
      bool now = pcur == DASHSVD_BF16 && stagnant_read >= 1;
      if (r_old > 0.0 && r_new > 0.0 && r_new < r_old) {
        const double q = r_new / r_old;
        double pred = r_new;
        for (int c = 0; c < chunk; ++c) pred *= q;
        now = now || pred <= 1.5 * tol;
      }
      if (now) {
        HIPCHK(read_slot(slot));
        pending = -1;
        if (stop) break;
        if (promote_read && pcur == DASHSVD_BF16) HIPCHK(promote_now());
      }
    }
    HIPCHK(hipStreamSynchronize(st));
    Qfin = Qc;
    Yfin = Yc;
    pfin = pcur;
  }
  const double t_loop = now_ms();
  // final Rayleigh-Ritz (steps 9-11): B = M Q ; eigSVD(B) ; U = B W(:,1:k) ;
  // V = Q Vs(:,1:k).
  tmark_begin(h, DASHSVD_KT_FINAL, 0);
  if (pdt == cdt) {
    // Overlapped order: the last block C (its buffer alternates with the
    // pass), Z = M C and W, with Q = C W and B = M Q = Z W never formed:
    //   B^T B = W^T (Z^T Z) W,  U = B W_B = Z (W W_B),  V = Q V_B = C (W V_B)
    // (W_B, V_B the final eigSVD's weights and eigenvectors): one Gram of Z,
    // l x l FP64 products, and one rescale each for U and V.
    void *Cl = (last_pass & 1) ? b.Q : b.C;
    HIPCHK(launch_gram(Mm, l, b.Z, ld, cdt, b.gpart, nb_m, b.G2, nullptr, st, nullptr));
    HIPCHK(launch_small_gemm(l, l, l, b.G2, l, 0, b.W, l, b.T2, l, st));
    HIPCHK(launch_small_gemm(l, l, l, b.W, l, 1, b.T2, l, b.G, l, st));
    {
      EigArgs ea = make_eig(3);
      ea.W = b.W2;
      HIPCHK(eig_solve(ea, st));
    }
    HIPCHK(launch_small_gemm(l, k, l, b.W, l, 0, b.W2, l, b.PU, k, st));
    HIPCHK(launch_small_gemm(l, k, l, b.W, l, 0, b.Vs, l, b.PV, k, st));
    // V first; its sign normalisation flips V and the columns of W W_B, so
    // U comes out with the matching signs
    HIPCHK(launch_rescale(Mn, l, Cl, ld, cdt, b.PV, k, k, b.Vo, k, cdt, nullptr, st, nullptr, nullptr, mapN));
    HIPCHK(launch_sign_fold(Mn, k, b.Vo, k, cdt, b.PU, l, k, b.sgn_max, b.sgn_idx, sgn_blk, st));
    HIPCHK(launch_rescale(Mm, l, b.Z, ld, cdt, b.PU, k, k, b.Uo, k, cdt, nullptr, st, nullptr, nullptr, mapM));
  } else {
    void *Qf = Qfin, *Bf = b.B;
    if (pfin != cdt) {
      // the BF16 form keeps an FP32 B
      HIPCHK(plan_spmm(b.planM, Mm, rpM, colM, valM, vdt, Qfin, ld, pfin, b.B, ld, cdt, ldc, T, vm, nullptr, 0,
                       nullptr, nullptr, st));
    } else {
      // promoted to FP32 panels: B is the last M Q
      Bf = Yfin;
    }
    HIPCHK(launch_gram(Mm, l, Bf, ld, cdt, b.gpart, nb_m, b.G, nullptr, st, nullptr));
    {
      EigArgs ea = make_eig(3);
      HIPCHK(eig_solve(ea, st));
    }
    HIPCHK(launch_rescale(Mm, l, Bf, ld, cdt, b.W, l, k, b.Uo, k, cdt, nullptr, st, nullptr, nullptr, mapM));
    HIPCHK(launch_rescale(Mn, l, Qf, ld, pfin, b.Vs, l, k, b.Vo, k, cdt, nullptr, st, nullptr, nullptr, mapN));
    HIPCHK(launch_sign_fix(Mn, Mm, k, b.Vo, k, b.Uo, k, cdt, b.sgn_max, b.sgn_idx, sgn_blk, st));
  }
  tmark_end(h);
  // solver state and traces through the pinned staging area (asynchronous
  // copies, one wait)
  char *pin = reinterpret_cast<char *>(h->hflags);
  SolverState hs;
  HIPCHK(hipMemcpyAsync(pin + kPinState, b.state, sizeof(hs), hipMemcpyDeviceToHost, st));
  dashsvd_info &inf = h->info;
  std::memset(&inf, 0, sizeof(inf));
  const int ntr = pmax < DASHSVD_MAX_TRACE ? pmax : DASHSVD_MAX_TRACE;
  if (ntr > 0) {
    HIPCHK(hipMemcpyAsync(pin + kPinAlpha, b.tr_alpha, 8 * (size_t)ntr, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(pin + kPinRatio, b.tr_ratio, 8 * (size_t)ntr, hipMemcpyDeviceToHost, st));
  }
  // entries past the calls that ran are zero (cleared at setup)
  const int nsw = cap + 2 < DASHSVD_MAX_TRACE + 2 ? cap + 2 : DASHSVD_MAX_TRACE + 2;
  HIPCHK(hipMemcpyAsync(pin + kPinSweeps, b.tr_sweeps, 4 * (size_t)nsw, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::memcpy(&hs, pin + kPinState, sizeof(hs));
  if (ntr > 0) {
    std::memcpy(inf.alpha_used, pin + kPinAlpha, 8 * (size_t)ntr);
    std::memcpy(inf.ratio, pin + kPinRatio, 8 * (size_t)ntr);
  }
  std::memcpy(inf.sweeps_per_call, pin + kPinSweeps, 4 * (size_t)nsw);
  const double t_end = now_ms();
  inf.passes = hs.pass;
  inf.eig_calls = hs.eig_calls;
  inf.eig_sweeps = hs.eig_sweeps;
  inf.converged = hs.converged;
  inf.rank_deficient = hs.deficient;
  inf.l = l;
  inf.learned_fallback = hs.sched_off;
  inf.final_alpha = hs.alpha;
  inf.promoted = promoted;
  inf.cholqr_calls = hs.cq_calls;
  inf.learned_n = hs.learned_ready ? hs.learned_n : 0;
  inf.long_row_used = T;
  inf.lane_vectors_used = vm;
  inf.slab_kib_used = (int32_t)(slab_b >> 10);
  inf.reordered = reorder ? 1 : 0;
  inf.head_rows = b.planM.head;
  inf.head_rows_t = b.planT.head;
  inf.time_total_ms = t_end - t0;
  inf.time_setup_ms = t_setup - t0;
  inf.time_loop_ms = t_loop - t_setup;
  inf.time_final_ms = t_end - t_loop;
  inf.long_chunks_A = wide ? b.planT.n_chunks : b.planM.n_chunks;
  inf.long_chunks_AT = wide ? b.planM.n_chunks : b.planT.n_chunks;
  for (const auto &mk : h->marks) {
    if (mk.pass > hs.pass) continue;  // passes launched after the stop returned at once
    // the transposed product of the stopping pass may have returned early
    if (hs.done && pdt == cdt && mk.group == DASHSVD_KT_SPMM_T && mk.pass == hs.pass) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev[mk.e0], h->ev[mk.e1]) == hipSuccess) {
      inf.kt_ms[mk.group] += ms;
      inf.kt_count[mk.group] += 1;
    }
  }
  // results in the caller's orientation
  h->m = m;
  h->n = n;
  h->k = k;
  h->l = l;
  h->out_dt = cdt;
  h->U = wide ? b.Vo : b.Uo;
  h->V = wide ? b.Uo : b.Vo;
  h->S = b.S;
  h->trace_s = b.tr_s;
  h->trace_cap = cap;
  h->have = true;
  {
    auto &c = h->ev_ctx;
    c.ok = true;
    c.nnz = nnz;
    c.Mm = Mm;
    c.Mn = Mn;
    c.wide = wide;
    c.vdt = vdt;
    c.cdt = cdt;
    c.ld = ld;
    c.T = T;
    c.rp[0] = rpM;
    c.rp[1] = rpMT;
    c.col[0] = colM;
    c.col[1] = colMT;
    c.val[0] = valM;
    c.val[1] = valMT;
    c.plan[0] = b.planM;
    c.plan[1] = b.planT;
    // panels no longer needed once U and V are formed: B and C (C type)
    c.panel_m = b.B;
    c.panel_n = b.C;
    c.gpart = b.gpart;
    c.G = b.G;
    c.u_row_to = reorder ? b.inv_r : nullptr;
    c.v_row_to = reorder ? b.inv_c : nullptr;
  }
  dashsvd_status s = DASHSVD_OK;
  if (tol > 0.0 && !hs.converged) s = DASHSVD_NOT_CONVERGED;
  else if (hs.deficient) s = DASHSVD_RANK_DEFICIENT;
  inf.status = s;
  return s;
}

dashsvd_status dashsvd_run(dashsvd_handle *h, const dashsvd_csr *A, int32_t k, int32_t p, double tol) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  h->err.clear();
  dashsvd_status s = check_args(h, A, k, p, tol);
  if (s != DASHSVD_OK) return s;
  if (h->opt.shift_policy == DASHSVD_SHIFT_LEARNED && (!h->mlp.ok || h->mlp.l != k + p))
    return fail(h, DASHSVD_ERR_INVALID_ARG,
                "LEARNED policy needs an MLP for l = k + oversampling (dashsvd_mlp_init / set_params)");
  if (h->opt.omega && h->opt.precision == DASHSVD_PREC_BF16_PANELS)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "a caller-provided Omega is not supported with BF16 panels");
  if (h->opt.pve_mode == DASHSVD_PVE_NOSURR && h->opt.precision == DASHSVD_PREC_BF16_PANELS)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "pve_mode NOSURR needs FP32 or FP64 panels");
  s = run_impl(h, A, k, p, tol, false, nullptr);
  h->info.status = s;
  return s;
}

dashsvd_status dashsvd_workspace_size(const dashsvd_csr *A, int32_t k, int32_t p, int32_t precision,
                                      size_t *bytes) {
  if (!bytes) return DASHSVD_ERR_INVALID_ARG;
  dashsvd_handle tmp;
  dashsvd_options o;
  default_options(&o);
  o.precision = precision;
  dashsvd_status s = dashsvd_set_options(&tmp, &o);
  if (s != DASHSVD_OK) return s;
  s = check_args(&tmp, A, k, p, 0.0);
  if (s != DASHSVD_OK) return s;
  return run_impl(&tmp, A, k, p, 0.0, true, bytes);
}

static dashsvd_status run_batched_impl(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k,
                                       int32_t p, double tol, bool measure_only, size_t *measured,
                                       int32_t member0 = 0);
static std::vector<std::pair<int32_t, int32_t>> batch_groups(const dashsvd_handle *h, const dashsvd_csr *As,
                                                             int32_t count);
// Arena bytes of a batched run: the largest of its sub-batches.
static dashsvd_status batched_arena_need(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k,
                                         int32_t p, size_t *bytes) {
  size_t need = 0;
  for (const auto &g : batch_groups(h, As, count)) {
    size_t b = 0;
    const dashsvd_status s = run_batched_impl(h, As + g.first, g.second, k, p, 0.0, true, &b, g.first);
    if (s != DASHSVD_OK) return s;
    need = std::max(need, b);
  }
  *bytes = need;
  return DASHSVD_OK;
}
static dashsvd_status check_batch(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k, int32_t p,
                                  double tol);

dashsvd_status dashsvd_workspace_size_batched(const dashsvd_csr *As, int32_t count, int32_t k, int32_t p,
                                              int32_t precision, size_t *bytes) {
  if (!bytes) return DASHSVD_ERR_INVALID_ARG;
  dashsvd_handle tmp;
  dashsvd_options o;
  default_options(&o);
  o.precision = precision;
  dashsvd_status s = dashsvd_set_options(&tmp, &o);
  if (s == DASHSVD_OK) s = check_batch(&tmp, As, count, k, p, 0.0);
  if (s != DASHSVD_OK) return s;
  return batched_arena_need(&tmp, As, count, k, p, bytes);
}

dashsvd_status dashsvd_handle_workspace_size(const dashsvd_handle *h, const dashsvd_csr *As, int32_t count,
                                             int32_t batched, int32_t k, int32_t p, size_t *bytes) {
  if (!h || !bytes) return DASHSVD_ERR_INVALID_ARG;
  // the sizing pass reads only the options, the schedule and the tuning
  // table, so it runs on a copy that owns no HIP resources
  dashsvd_handle tmp;
  tmp.opt = h->opt;
  tmp.sched = h->sched;
  tmp.tune = h->tune;
  dashsvd_status s = batched ? check_batch(&tmp, As, count, k, p, 0.0) : check_args(&tmp, As, k, p, 0.0);
  if (s != DASHSVD_OK) return s;
  return batched ? batched_arena_need(&tmp, As, count, k, p, bytes) : run_impl(&tmp, As, k, p, 0.0, true, bytes);
}

dashsvd_status dashsvd_get_USV(dashsvd_handle *h, void *U, int64_t ldu, double *S, void *V, int64_t ldv,
                               int32_t dtype, int32_t on_device) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  if (!h->have) return fail(h, DASHSVD_ERR_STATE, "no results: run first");
  if (dtype != DASHSVD_F32 && dtype != DASHSVD_F64) return fail(h, DASHSVD_ERR_INVALID_ARG, "dtype");
  if ((U && ldu < h->k) || (V && ldv < h->k)) return fail(h, DASHSVD_ERR_INVALID_ARG, "leading dimension");
  hipStream_t st = h->st;
  const size_t es = dsz(dtype);
  struct Item {
    void *dst;
    int64_t ldd;
    const void *src;
    int64_t rows;
  } items[2] = {{U, ldu, h->U, h->m}, {V, ldv, h->V, h->n}};
  for (auto &it : items) {
    if (!it.dst) continue;
    if (on_device) {
      HIPCHK(launch_copy2d(it.src, h->k, h->out_dt, it.dst, it.ldd, dtype, it.rows, h->k, st));
    } else {
      void *tmp = nullptr;
      HIPCHK(hipMalloc(&tmp, es * (size_t)it.rows * h->k + 16));
      hipError_t e = launch_copy2d(it.src, h->k, h->out_dt, tmp, h->k, dtype, it.rows, h->k, st);
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(it.dst, es * it.ldd, tmp, es * h->k, es * h->k, it.rows, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      (void)hipFree(tmp);
      HIPCHK(e);
    }
  }
  if (S) HIPCHK(hipMemcpyAsync(S, h->S, 8 * (size_t)h->k, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return DASHSVD_OK;
}

}  // extern "C"

// eps_PVE and eps_sigma of the last run (Sec. 4).  Leaves Z = A^T U (in the
// solver's column order) in the n-row evaluation panel, leading dimension
// k rounded up to 8, for the residual metric.
static dashsvd_status evaluate_core(dashsvd_handle *h, const dashsvd_csr *A, const double *sigma_ref,
                                    int32_t n_ref, double *eps_pve, double *eps_sigma) {
  if (!h->have || !h->ev_ctx.ok) return fail(h, DASHSVD_ERR_STATE, "no results: run first");
  auto &c = h->ev_ctx;
  if (!A || A->m != h->m || A->n != h->n || A->nnz != c.nnz)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "A is not the matrix of the last run");
  if (!sigma_ref || n_ref < h->k + 1) return fail(h, DASHSVD_ERR_INVALID_ARG, "sigma_ref needs k + 1 values");
  if (!(sigma_ref[h->k] > 0.0)) return fail(h, DASHSVD_ERR_INVALID_ARG, "sigma_ref[k] must be positive");
  hipStream_t st = h->st;
  const int k = h->k;
  const int ld8 = (int)round_up(k, 8);
  // Z = A^T U with U (m x k) in the caller's orientation: A^T is M^T when
  // A = M, and M itself when M = A^T (m < n)
  const int side = c.wide ? 0 : 1;
  const int64_t zrows = c.wide ? c.Mm : c.Mn, urows = h->m;
  void *Upad = c.wide ? c.panel_n : c.panel_m;  // urows x ld8
  void *Z = c.wide ? c.panel_m : c.panel_n;     // zrows x ld8
  // with the degree order, U (rows of A) enters in the permuted row order
  HIPCHK(launch_copy2d(h->U, k, h->out_dt, Upad, ld8, c.cdt, urows, k, st, c.u_row_to));
  const Plan &pl = c.plan[side];
  HIPCHK(plan_spmm(pl, zrows, c.rp[side], c.col[side], c.val[side], c.vdt, Upad, ld8, c.cdt, Z, ld8, c.cdt, ld8, c.T,
                   1, nullptr, 0, nullptr, nullptr, st));
  // ||A^T u_i||^2 = (Z^T Z)_ii in FP64
  HIPCHK(launch_gram(zrows, k, Z, ld8, c.cdt, c.gpart, gram_blocks(zrows, k), c.G, nullptr, st, nullptr));
  std::vector<double> G((size_t)k * k), S(k);
  HIPCHK(hipMemcpyAsync(G.data(), c.G, 8 * (size_t)k * k, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(S.data(), h->S, 8 * (size_t)k, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // eps_PVE = max_i |sigma_i^2 - ||A^T u_i||^2| / sigma_{k+1}^2 and
  // eps_sigma = max_i |sigma_i - S_i| / sigma_i (Sec. 4 accuracy metrics)
  const double sk1 = sigma_ref[k] * sigma_ref[k];
  double pve = 0.0, es = 0.0;
  for (int i = 0; i < k; ++i) {
    const double d = std::fabs(sigma_ref[i] * sigma_ref[i] - G[(size_t)i * k + i]) / sk1;
    if (d > pve || d != d) pve = d;
    const double e = std::fabs(sigma_ref[i] - S[i]) / sigma_ref[i];
    if (e > es || e != e) es = e;
  }
  if (eps_pve) *eps_pve = pve;
  if (eps_sigma) *eps_sigma = es;
  return DASHSVD_OK;
}

// Largest eigenvalue of the symmetric tridiagonal matrix with diagonal
// al[0..j) and off-diagonal be[0..j-1), by bisection on Sturm counts
// (the number of negative pivots of T - x I is the number of eigenvalues
// below x).
static double tridiag_max_eig(int j, const std::vector<double> &al, const std::vector<double> &be) {
  double lo = 0.0, hi = 0.0;
  for (int i = 0; i < j; ++i) {
    const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < j ? std::fabs(be[i]) : 0.0);
    lo = i == 0 ? al[i] - r : std::min(lo, al[i] - r);
    hi = i == 0 ? al[i] + r : std::max(hi, al[i] + r);
  }
  auto below = [&](double x) {
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < j; ++i) {
      d = al[i] - x - (i > 0 ? be[i - 1] * be[i - 1] / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d < 0.0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 4e-16 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) >= j) hi = mid;
    else lo = mid;
  }
  return hi;
}

extern "C" {

dashsvd_status dashsvd_evaluate(dashsvd_handle *h, const dashsvd_csr *A, const double *sigma_ref, int32_t n_ref,
                                double *eps_pve, double *eps_sigma) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  h->err.clear();
  return evaluate_core(h, A, sigma_ref, n_ref, eps_pve, eps_sigma);
}

dashsvd_status dashsvd_evaluate_all(dashsvd_handle *h, const dashsvd_csr *A, const double *sigma_ref, int32_t n_ref,
                                    int32_t max_steps, uint64_t seed, dashsvd_metrics *out) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  h->err.clear();
  if (!out || max_steps < 1) return fail(h, DASHSVD_ERR_INVALID_ARG, "metrics output and max_steps >= 1 needed");
  std::memset(out, 0, sizeof(*out));
  dashsvd_status s = evaluate_core(h, A, sigma_ref, n_ref, &out->eps_pve, &out->eps_sigma);
  if (s != DASHSVD_OK) return s;
  auto &c = h->ev_ctx;
  hipStream_t st = h->st;
  const int k = h->k;
  const int ld8 = (int)round_up(k, 8);
  const int64_t m = h->m, n = h->n;
  const int steps = (int)std::min<int64_t>(max_steps, n);
  const int J = std::max(k, steps + 1);
  // panels of the solver's arena (free once U and V are formed): the n-row
  // one holds Z = A^T U from evaluate_core, then serves with the m-row one
  // the SpMMs of the Lanczos process (8 columns, the first used)
  void *pan_n = c.wide ? c.panel_m : c.panel_n;
  void *pan_m = c.wide ? c.panel_n : c.panel_m;
  const int sideA = c.wide ? 1 : 0, sideAT = c.wide ? 0 : 1;
  // FP64 evaluation buffers (column-major)
  const size_t nU = (size_t)m * k, nV = (size_t)n * k, nQ = (size_t)J * n, nP = eval_partial_elems(J);
  const size_t total = nU + nV + nQ + (size_t)m + (size_t)n + (size_t)J * 2 + nP + 8;
  double *buf = nullptr;
  if (hipMalloc(&buf, 8 * total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, DASHSVD_ERR_OOM, "evaluation buffers");
  }
  double *Ucm = buf, *Vcm = Ucm + nU, *Q = Vcm + nV, *y = Q + nQ, *w = y + m, *t1 = w + n, *t2 = t1 + J,
         *part = t2 + J, *scal = part + nP;
  hipError_t e = hipSuccess;
  auto run = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  std::vector<double> hs((size_t)k);
  // eps_res = max_i ||A^T u_i - S_i v_i|| / sigma_i: Z (in the solver's
  // column order) and V brought to that order, both column-major
  run(launch_to_colmajor(n, k, pan_n, ld8, c.cdt, Q, n, nullptr, st));
  run(launch_to_colmajor(n, k, h->V, k, h->out_dt, Vcm, n, c.v_row_to, st));
  run(launch_resid_norms(n, k, Q, Vcm, n, h->S, part, t1, st));
  run(hipMemcpyAsync(hs.data(), t1, 8 * (size_t)k, hipMemcpyDeviceToHost, st));
  run(hipStreamSynchronize(st));
  double res = 0.0;
  for (int i = 0; i < k && e == hipSuccess; ++i) {
    const double r = std::sqrt(hs[i]) / sigma_ref[i];
    if (r > res || r != r) res = r;
  }
  out->eps_res = res;
  // ||A - U S V^T||_2: Lanczos with full reorthogonalisation on E^T E in
  // the solver's row and column orders (norms do not depend on them),
  // started from the Gaussian vector of the Philox stream keyed by seed
  run(launch_to_colmajor(m, k, h->U, k, h->out_dt, Ucm, m, c.u_row_to, st));
  run(hipMemsetAsync(pan_n, 0, dsz(c.cdt) * (size_t)n * 8, st));
  run(hipMemsetAsync(pan_m, 0, dsz(c.cdt) * (size_t)m * 8, st));
  run(launch_gaussian(seed, n, 1, Q, 1, DASHSVD_F64, st, c.v_row_to));
  run(launch_dots(n, 1, Q, n, Q, part, scal, st));
  run(launch_scale_by_norm(n, Q, scal, Q, st));
  const double conv = c.cdt == DASHSVD_F64 ? 1e-14 : 1e-9;
  std::vector<double> al, be;
  double lam = 0.0, lam_old = -1.0;
  double hv[3];
  int taken = 0;
  for (int j = 0; j < steps && e == hipSuccess; ++j) {
    double *q = Q + (size_t)j * n;
    const Plan &pA = c.plan[sideA], &pT = c.plan[sideAT];
    // y = A q - U (S .* (V^T q))
    run(launch_copy2d(q, 1, DASHSVD_F64, pan_n, 8, c.cdt, n, 1, st));
    run(plan_spmm(pA, m, c.rp[sideA], c.col[sideA], c.val[sideA], c.vdt, pan_n, 8, c.cdt, pan_m, 8, c.cdt, 8, c.T, 1,
                  nullptr, 0, nullptr, nullptr, st));
    run(launch_dots(n, k, Vcm, n, q, part, t1, st));
    run(launch_copy2d(pan_m, 8, c.cdt, y, 1, DASHSVD_F64, m, 1, st));
    run(launch_combo(m, k, Ucm, m, t1, h->S, y, st));
    // w = A^T y - V (S .* (U^T y))
    run(launch_copy2d(y, 1, DASHSVD_F64, pan_m, 8, c.cdt, m, 1, st));
    run(plan_spmm(pT, n, c.rp[sideAT], c.col[sideAT], c.val[sideAT], c.vdt, pan_m, 8, c.cdt, pan_n, 8, c.cdt, 8, c.T,
                  1, nullptr, 0, nullptr, nullptr, st));
    run(launch_dots(m, k, Ucm, m, y, part, t1, st));
    run(launch_copy2d(pan_n, 8, c.cdt, w, 1, DASHSVD_F64, n, 1, st));
    run(launch_combo(n, k, Vcm, n, t1, h->S, w, st));
    // two rounds of Gram-Schmidt against q_0..q_j; alpha_j = q_j^T w is
    // the sum of the two rounds' coefficients of q_j
    run(launch_dots(n, j + 1, Q, n, w, part, t1, st));
    run(launch_combo(n, j + 1, Q, n, t1, nullptr, w, st));
    run(launch_dots(n, j + 1, Q, n, w, part, t2, st));
    run(launch_combo(n, j + 1, Q, n, t2, nullptr, w, st));
    run(launch_dots(n, 1, w, n, w, part, scal, st));
    run(launch_scale_by_norm(n, w, scal, Q + (size_t)(j + 1) * n, st));
    run(hipMemcpyAsync(&hv[0], t1 + j, 8, hipMemcpyDeviceToHost, st));
    run(hipMemcpyAsync(&hv[1], t2 + j, 8, hipMemcpyDeviceToHost, st));
    run(hipMemcpyAsync(&hv[2], scal, 8, hipMemcpyDeviceToHost, st));
    run(hipStreamSynchronize(st));
    if (e != hipSuccess) break;
    const double a = hv[0] + hv[1], b = std::sqrt(hv[2] > 0.0 ? hv[2] : 0.0);
    al.push_back(a);
    be.push_back(b);
    taken = j + 1;
    const bool last = j + 1 == steps || !(b > 1e-14 * std::fabs(a));
    if (last || (j + 1) % 5 == 0) {
      lam = tridiag_max_eig(j + 1, al, be);
      if (last || std::fabs(lam - lam_old) <= conv * lam) break;
      lam_old = lam;
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipFree(buf);
  if (e != hipSuccess) return fail(h, DASHSVD_ERR_HIP, std::string("evaluation: ") + hipGetErrorString(e));
  const double en = std::sqrt(lam > 0.0 ? lam : 0.0);
  out->spec_norm = en;
  out->eps_spec = (en - sigma_ref[k]) / sigma_ref[k];
  out->lanczos_steps = taken;
  return DASHSVD_OK;
}

// ===================================================================== batched form
// All matrices of the batch advance pass-synchronously (Alg. 5 on each):
// their operators are stacked into one block-diagonal CSR, so every step of
// a pass is one launch over the whole batch, each matrix with its own shift,
// PVE check, stop flag and traces.  One pass is captured as a graph on the
// handle's internal stream and replayed; stopped matrices skip their work
// items.  The run is ordered after prior work on the handle's stream, which
// waits for it in turn.
static dashsvd_status run_batched_impl(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k,
                                       int32_t p, double tol, bool measure_only, size_t *measured,
                                       int32_t member0) {
  const int prec = h->opt.precision;
  const int vdt = prec == DASHSVD_PREC_FP64 ? DASHSVD_F64 : DASHSVD_F32;
  const int pdt = prec == DASHSVD_PREC_FP64 ? DASHSVD_F64 : (prec == DASHSVD_PREC_BF16_PANELS ? DASHSVD_BF16 : DASHSVD_F32);
  const int cdt = prec == DASHSVD_PREC_FP64 ? DASHSVD_F64 : DASHSVD_F32;
  const size_t accsz = prec == DASHSVD_PREC_FP64 ? 8 : 4;
  const int l = k + p;
  const int ld = (int)round_up(l, 8);
  const int pmax = h->opt.p_max;
  const int cap = pmax > 0 ? pmax : 1;
  const int in_dt = As[0].value_dtype;
  const bool on_dev = As[0].on_device != 0;
  // stacked sizes
  std::vector<int64_t> roff(count + 1, 0), coff(count + 1, 0), zoff(count + 1, 0);
  int64_t max_rn = 1, max_m = 1, max_n = 1;
  for (int b = 0; b < count; ++b) {
    roff[b + 1] = roff[b] + As[b].m;
    coff[b + 1] = coff[b] + As[b].n;
    zoff[b + 1] = zoff[b] + As[b].nnz;
    max_rn = std::max(max_rn, std::max(As[b].m + 1, As[b].nnz));
    max_m = std::max(max_m, As[b].m);
    max_n = std::max(max_n, As[b].n);
  }
  const int64_t m = roff[count], n = coff[count], nnz = zoff[count];
  const std::string tkey = tune_key(prec, ld, m, nnz, true);
  const int32_t T = chunk_length(h, tkey, 0);
  const int vm = lane_mult(h, tkey);
  if (m > INT32_MAX - 1 || n > INT32_MAX - 1 || nnz > INT32_MAX - 1)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "batch too large for 32-bit indices of the stacked operator");
  // work items of both sides (rows of M: U, B; rows of M^T: C, Q, V)
  std::vector<BItem> itM, itN;
  std::vector<int64_t> ioffM(count + 1, 0), ioffN(count + 1, 0);
  for (int b = 0; b < count; ++b) {
    for (int64_t r = roff[b]; r < roff[b + 1]; r += kBItemRows)
      itM.push_back({b, 0, r, std::min(r + kBItemRows, roff[b + 1])});
    ioffM[b + 1] = (int64_t)itM.size();
    for (int64_t r = coff[b]; r < coff[b + 1]; r += kBItemRows)
      itN.push_back({b, 0, r, std::min(r + kBItemRows, coff[b + 1])});
    ioffN[b + 1] = (int64_t)itN.size();
  }
  hipStream_t st = h->stg;

  Arena &ar = h->ar;
  ar.reset(measure_only || ar.base == nullptr);
  if (!measure_only) {
    size_t need = 0;
    run_batched_impl(h, As, count, k, p, tol, true, &need, member0);
    dashsvd_status s = ensure_arena(h, need);
    if (s != DASHSVD_OK) return s;
    ar.reset(false);
  }
  h->have = false;
  h->bat.have = false;
  RunBufs b;
  int64_t *rpA = (int64_t *)ar.take(8 * (size_t)(m + 1));
  int32_t *colA = (int32_t *)ar.take(4 * (size_t)(nnz + 1));
  void *val_raw = ar.take(dsz(in_dt) * (size_t)(nnz + 1));
  void *valA = in_dt == vdt ? val_raw : ar.take(dsz(vdt) * (size_t)(nnz + 1));
  BMatDesc *desc = (BMatDesc *)ar.take(sizeof(BMatDesc) * (size_t)count);
  b.rpT = (int64_t *)ar.take(8 * (size_t)(n + 1));
  b.colT = (int32_t *)ar.take(4 * (size_t)(nnz + 1));
  b.valT = ar.take(dsz(vdt) * (size_t)(nnz + 1));
  b.rowidx = (int32_t *)ar.take(4 * (size_t)(nnz + 1));
  b.flags = (int32_t *)ar.take(4 * 8);
  b.tws_bytes = transpose_ws_bytes(n, nnz);
  b.tws = ar.take(b.tws_bytes);
  b.scan_tmp = (int64_t *)ar.take(8 * scan_tmp_elems(std::max(m, n) + 1));
  const int64_t bprow_b = (int64_t)ld * (int64_t)dsz(pdt);
  const int64_t bslab_b = slab_bytes(h, tkey);
  plan_alloc(h, ar, b.planM, m, nnz, T, ld, accsz, n, bprow_b, bslab_b);
  plan_alloc(h, ar, b.planT, n, nnz, T, ld, accsz, m, bprow_b, bslab_b);
  b.Y = ar.take(dsz(pdt) * (size_t)m * ld);
  b.Q = ar.take(dsz(pdt) * (size_t)n * ld);
  b.C = ar.take(dsz(cdt) * (size_t)n * ld);
  b.B = pdt == cdt ? b.Y : ar.take(dsz(cdt) * (size_t)m * ld);
  const size_t ll = (size_t)l * l;
  b.G = (double *)ar.take(8 * ll * count);
  b.W = (double *)ar.take(8 * ll * count);
  b.Vs = (double *)ar.take(8 * ll * count);
  b.S = (double *)ar.take(8 * (size_t)l * count);
  b.Sprev = (double *)ar.take(8 * (size_t)l * count);
  b.state = (SolverState *)ar.take(sizeof(SolverState) * (size_t)count);
  b.tr_alpha = (double *)ar.take(8 * (size_t)cap * count);
  b.tr_ratio = (double *)ar.take(8 * (size_t)cap * count);
  b.tr_s = (double *)ar.take(8 * (size_t)cap * l * count);
  b.tr_sweeps = (int32_t *)ar.take(4 * (size_t)(cap + 2) * count);
  b.sched = (double *)ar.take(8 * (size_t)(pmax + 2));
  b.Uo = ar.take(dsz(cdt) * (size_t)m * k);
  b.Vo = ar.take(dsz(cdt) * (size_t)n * k);
  // BF16 panels: FP32 panels for the passes after a promotion
  b.Q32 = pdt != cdt ? ar.take(dsz(cdt) * (size_t)n * ld) : nullptr;
  b.Y32 = pdt != cdt ? ar.take(dsz(cdt) * (size_t)m * ld) : nullptr;
  // per matrix and mode: the arguments of the first eigensolver, then (one-
  // sided solver) those of the two-sided one gated on its decline
  EigArgs *eargs = (EigArgs *)ar.take(sizeof(EigArgs) * 6 * (size_t)count);
  int64_t *offM = (int64_t *)ar.take(8 * (size_t)(count + 1));
  int64_t *offN = (int64_t *)ar.take(8 * (size_t)(count + 1));
  int64_t *ioffM_d = (int64_t *)ar.take(8 * (size_t)(count + 1));
  int64_t *ioffN_d = (int64_t *)ar.take(8 * (size_t)(count + 1));
  int64_t *boffM = (int64_t *)ar.take(8 * (size_t)(count + 1));  // Omega's blocks of 4 per matrix, prefix
  BItem *itM_d = (BItem *)ar.take(sizeof(BItem) * itM.size());
  BItem *itN_d = (BItem *)ar.take(sizeof(BItem) * itN.size());
  double *bpart = (double *)ar.take(8 * bgram_partial_elems((int64_t)std::max(itM.size(), itN.size()), l));
  int32_t *rowmatM = (int32_t *)ar.take(4 * (size_t)m);
  int32_t *rowmatN = (int32_t *)ar.take(4 * (size_t)n);
  int32_t *ndone = (int32_t *)ar.take(16);
  if (measure_only) {
    *measured = ar.used;
    return DASHSVD_OK;
  }

  // ---------------------------------------------------------------- setup
  HIPCHK(hipMemsetAsync(b.flags, 0, 4 * 8, st));
  HIPCHK(hipMemsetAsync(b.planM.nlong, 0, 16, st));
  HIPCHK(hipMemsetAsync(b.planT.nlong, 0, 16, st));
  HIPCHK(hipMemsetAsync(b.planM.slab_cnt, 0, 8 * (size_t)(kMaxSlabs + 1), st));
  HIPCHK(hipMemsetAsync(b.planT.slab_cnt, 0, 8 * (size_t)(kMaxSlabs + 1), st));
  HIPCHK(hipMemsetAsync(b.state, 0, sizeof(SolverState) * (size_t)count, st));
  HIPCHK(hipMemsetAsync(b.Sprev, 0, 8 * (size_t)l * count, st));
  HIPCHK(hipMemsetAsync(b.tr_alpha, 0, 8 * (size_t)cap * count, st));
  HIPCHK(hipMemsetAsync(b.tr_ratio, 0, 8 * (size_t)cap * count, st));
  HIPCHK(hipMemsetAsync(b.tr_sweeps, 0, 4 * (size_t)(cap + 2) * count, st));
  HIPCHK(hipMemsetAsync(ndone, 0, 16, st));
  // stacked operator
  std::vector<BMatDesc> hd(count);
  for (int i = 0; i < count; ++i) {
    hd[i] = {As[i].row_ptr, As[i].col_idx, As[i].values, As[i].m, As[i].n, As[i].nnz, roff[i], coff[i], zoff[i]};
    if (!on_dev) {
      if (As[i].row_ptr[0] != 0 || As[i].row_ptr[As[i].m] != As[i].nnz)
        return fail(h, DASHSVD_ERR_BAD_CSR, "row_ptr of matrix " + std::to_string(i) + " malformed");
      HIPCHK(hipMemcpyAsync(rpA + roff[i], As[i].row_ptr, 8 * (size_t)As[i].m, hipMemcpyHostToDevice, st));
      if (As[i].nnz > 0) {
        HIPCHK(hipMemcpyAsync(colA + zoff[i], As[i].col_idx, 4 * (size_t)As[i].nnz, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync((char *)val_raw + dsz(in_dt) * zoff[i], As[i].values,
                              dsz(in_dt) * (size_t)As[i].nnz, hipMemcpyHostToDevice, st));
      }
    }
  }
  HIPCHK(hipMemcpyAsync(desc, hd.data(), sizeof(BMatDesc) * (size_t)count, hipMemcpyHostToDevice, st));
  HIPCHK(launch_bassemble(desc, count, max_rn, m, nnz, rpA, colA, val_raw, in_dt, on_dev ? 0 : 1, b.flags + 2, st));
  if (in_dt != vdt) HIPCHK(launch_convert(val_raw, in_dt, valA, vdt, nnz, st));
  HIPCHK(launch_validate(m, n, nnz, rpA, colA, valA, vdt, b.rowidx, b.flags, st));
  int32_t hflags[4] = {0, 0, 0, 0};
  HIPCHK(hipMemcpyAsync(hflags, b.flags, sizeof(hflags), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if ((hflags[0] & 1) || (hflags[2] & 1)) return fail(h, DASHSVD_ERR_BAD_CSR, "row_ptr/col_idx malformed");
  if (hflags[0] & 2) return fail(h, DASHSVD_ERR_NONFINITE, "NaN or Inf among the values");
  HIPCHK(launch_transpose(n, nnz, colA, b.rowidx, valA, vdt, b.rpT, b.colT, b.valT, b.tws, b.tws_bytes, st));
  HIPCHK(plan_build(b.planM, rpA, colA, T, b.scan_tmp, st));
  HIPCHK(plan_build(b.planT, b.rpT, b.colT, T, b.scan_tmp, st));
  int64_t totals[2] = {0, 0};
  int32_t nlongs[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(&totals[0], b.planM.off + b.planM.R, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&totals[1], b.planT.off + b.planT.R, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&nlongs[0], b.planM.nlong, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&nlongs[1], b.planT.nlong, 4, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(offM, roff.data(), 8 * (size_t)(count + 1), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(offN, coff.data(), 8 * (size_t)(count + 1), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ioffM_d, ioffM.data(), 8 * (size_t)(count + 1), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ioffN_d, ioffN.data(), 8 * (size_t)(count + 1), hipMemcpyHostToDevice, st));
  std::vector<int64_t> boff(count + 1, 0);
  for (int i = 0; i < count; ++i) boff[i + 1] = boff[i] + (As[i].m * (int64_t)l + 3) / 4;
  HIPCHK(hipMemcpyAsync(boffM, boff.data(), 8 * (size_t)(count + 1), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(itM_d, itM.data(), sizeof(BItem) * itM.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(itN_d, itN.data(), sizeof(BItem) * itN.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  b.planM.n_chunks = totals[0];
  b.planT.n_chunks = totals[1];
  b.planM.n_long = nlongs[0];
  b.planT.n_long = nlongs[1];
  HIPCHK(launch_browmat(offM, count, max_m, rowmatM, st));
  HIPCHK(launch_browmat(offN, count, max_n, rowmatN, st));
  // Omega of matrix i of the whole batch from the Philox stream keyed
  // (seed + i, 0); this sub-batch starts at member0; one launch
  HIPCHK(launch_gaussian_batched(h->opt.seed + (uint64_t)member0, count, offM, boffM, boff[count], l, b.Y, ld, pdt,
                                 st));
  if (!h->sched.empty())
    HIPCHK(hipMemcpyAsync(b.sched, h->sched.data(), 8 * h->sched.size(), hipMemcpyHostToDevice, st));
  // per-matrix eigSVD arguments for the sketch (mode 1), the passes (2) and
  // the final step (3)
  std::vector<EigArgs> ea(6 * (size_t)count);
  for (int mode = 1; mode <= 3; ++mode)
    for (int i = 0; i < count; ++i) {
      EigArgs &e = ea[(size_t)(mode - 1) * count + i];
      std::memset(&e, 0, sizeof(e));
      e.l = l;
      e.k = k;
      e.skip = prec == DASHSVD_PREC_FP64 ? 0x1.0p-53 : 0x1.0p-23;
      e.G = b.G + ll * i;
      e.S = b.S + (size_t)l * i;
      e.Vs = b.Vs + ll * i;
      e.W = b.W + ll * i;
      e.state = b.state + i;
      e.mode = mode;
      e.pve_mode = h->opt.pve_mode;
      e.policy = h->opt.shift_policy;
      e.tol = tol;
      e.Sprev = b.Sprev + (size_t)l * i;
      e.trace_alpha = b.tr_alpha + (size_t)cap * i;
      e.trace_ratio = b.tr_ratio + (size_t)cap * i;
      e.trace_s = b.tr_s + (size_t)cap * l * i;
      e.trace_cap = cap;
      e.trace_sweeps = b.tr_sweeps + (size_t)(cap + 2) * i;
      e.sched = h->sched.empty() ? nullptr : b.sched;
      e.sched_len = (int)h->sched.size();
      e.ndone = ndone;
      e.stagnation_guard = mode == 2 && pdt == DASHSVD_BF16;
      e.decline = &b.state[i].j1_decline;
      EigArgs &f = ea[(size_t)(mode + 2) * count + i];
      f = e;
      f.decline = nullptr;
      f.run_if = &b.state[i].j1_decline;
    }
  HIPCHK(hipMemcpyAsync(eargs, ea.data(), sizeof(EigArgs) * ea.size(), hipMemcpyHostToDevice, st));
  // ONESIDED: one-sided Jacobi on the Cholesky factor (l <= 128; two-sided
  // where it declines); the batched form has no Cholesky-QR blocks
  const bool onesided = h->opt.eig_method == DASHSVD_EIG_ONESIDED && l <= 128;
  auto beig = [&](int mode) -> hipError_t {
    const EigArgs *a1 = eargs + (size_t)(mode - 1) * count;
    if (!onesided) return launch_eig_batched(a1, count, l, st);
    const hipError_t e = launch_eig1s_batched(a1, count, l, st);
    return e == hipSuccess ? launch_eig_batched(a1 + 3 * (size_t)count, count, l, st) : e;
  };
  const int64_t nIM = (int64_t)itM.size(), nIN = (int64_t)itN.size();

  // Panels of the passes: BF16 (or the form's type) until a matrix's PVE
  // ratio reaches a plateau above tol (the stagnation guard of the single
  // form), then FP32 for the whole batch: Q = C W of the last block is formed
  // again in FP32 and the pass is captured again.
  void *Qc = b.Q, *Yc = b.Y;
  int pc = pdt;
  // one eigSVD block of every matrix on C (rows of M^T): Gram, eig, Q = C W,
  // then Y = M Q; gate: skip the matrices stopped before this pass
  auto block = [&](int mode, int gate) -> hipError_t {
    hipError_t e = launch_bgram(itN_d, nIN, ioffN_d, count, l, b.C, ld, cdt, bpart, b.G, (int64_t)ll, b.state,
                                gate, st);
    if (e == hipSuccess) e = beig(mode);
    if (e == hipSuccess)
      e = launch_brescale(itN_d, nIN, l, b.C, nullptr, ld, cdt, b.W, (int64_t)ll, l, l, Qc, ld, pc, b.state,
                          gate, st);
    if (e == hipSuccess)
      e = launch_spmm(m, rpA, colA, valA, vdt, Qc, ld, pc, Yc, ld, pc, ld, b.planM.n_chunks, b.planM.order,
                      b.planM.n_long, b.planM.longs, b.planM.partial, T, vm, nullptr, 0, nullptr, nullptr, st,
                      gate ? rowmatM : nullptr, b.state, n);
    return e;
  };
  // sketch: C = M^T Omega, eigSVD, Y = M Q
  HIPCHK(plan_spmm(b.planT, n, b.rpT, b.colT, b.valT, vdt, b.Y, ld, pdt, b.C, ld, cdt, ld, T, vm, nullptr, 0, nullptr,
                   nullptr, st));
  HIPCHK(block(1, 0));
  // one power pass of every running matrix, captured once and replayed
  auto pass = [&]() -> hipError_t {
    hipError_t e = launch_bsnap(b.state, count, 1, st);
    if (e == hipSuccess)
      e = launch_spmm(n, b.rpT, b.colT, b.valT, vdt, Yc, ld, pc, b.C, ld, cdt, ld, b.planT.n_chunks,
                      b.planT.order, b.planT.n_long, b.planT.longs, b.planT.partial, T, vm, Qc, ld, &b.state->alpha,
                      nullptr, st, rowmatN, b.state, m);
    if (e == hipSuccess) e = block(2, 1);
    return e;
  };
  // check_interval passes are captured as one graph and launched at once
  // (all p_max of them, one launch, when check_interval >= p_max); the host
  // reads the stop counters between launches.  A shorter last chunk is
  // captured again.
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int captured = 0;  // passes in the captured graph
  auto capture = [&](int npass) -> dashsvd_status {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    captured = 0;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t ec = hipSuccess;
    for (int c = 0; c < npass && ec == hipSuccess; ++c) ec = pass();
    hipError_t ee = hipStreamEndCapture(st, &graph);
    if (ec != hipSuccess || ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      graph = nullptr;
      return fail(h, DASHSVD_ERR_HIP, std::string("pass capture: ") + hipGetErrorString(ec != hipSuccess ? ec : ee));
    }
    hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(graph);
      graph = nullptr;
      return fail(h, DASHSVD_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
    }
    captured = npass;
    return DASHSVD_OK;
  };
  const int every = h->opt.check_interval > 0 ? std::min(h->opt.check_interval, std::max(pmax, 1)) : 1;
  if (pmax > 0) {
    dashsvd_status sc = capture(std::min(every, pmax));
    if (sc != DASHSVD_OK) return sc;
  }
  int launched = 0;
  int promoted = 0;
  int graph_launches = 0;
  HIPCHK(hipStreamSynchronize(st));
  const double t_loop0 = now_ms();
  hipError_t eloop = hipSuccess;
  dashsvd_status sloop = DASHSVD_OK;
  while (launched < pmax && eloop == hipSuccess && sloop == DASHSVD_OK) {
    const int chunk = (pmax - launched) < every ? (pmax - launched) : every;
    if (chunk != captured) sloop = capture(chunk);
    if (sloop != DASHSVD_OK) break;
    eloop = hipGraphLaunch(exec, st);
    ++graph_launches;
    launched += chunk;
    if (eloop == hipSuccess && tol > 0.0 && launched < pmax) {
      int32_t nd[2] = {0, 0};
      eloop = hipMemcpyAsync(nd, ndone, 8, hipMemcpyDeviceToHost, st);
      if (eloop == hipSuccess) eloop = hipStreamSynchronize(st);
      if (eloop != hipSuccess || nd[0] >= count) break;
      if (nd[1] > 0 && pc == DASHSVD_BF16) {
        Qc = b.Q32;
        Yc = b.Y32;
        pc = cdt;
        promoted = 1;
        eloop = launch_brescale(itN_d, nIN, l, b.C, nullptr, ld, cdt, b.W, (int64_t)ll, l, l, Qc, ld, pc, b.state,
                                1, st);
        if (eloop == hipSuccess)
          eloop = launch_spmm(m, rpA, colA, valA, vdt, Qc, ld, pc, Yc, ld, pc, ld, b.planM.n_chunks,
                              b.planM.order, b.planM.n_long, b.planM.longs, b.planM.partial, T, vm, nullptr, 0,
                              nullptr, nullptr, st, rowmatM, b.state, n);
        if (eloop == hipSuccess) sloop = capture(std::min(every, pmax - launched));
      }
    }
  }
  if (eloop == hipSuccess) eloop = hipStreamSynchronize(st);
  const double t_loop1 = now_ms();
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (sloop != DASHSVD_OK) return sloop;
  HIPCHK(eloop);
  // final Rayleigh-Ritz of every matrix: B = M Q, eigSVD(B), U = B W(:,1:k),
  // V = Q Vs(:,1:k), signs
  HIPCHK(launch_bsnap(b.state, count, 0, st));
  HIPCHK(plan_spmm(b.planM, m, rpA, colA, valA, vdt, Qc, ld, pc, b.B, ld, cdt, ld, T, vm, nullptr, 0, nullptr, nullptr,
                   st));
  HIPCHK(launch_bgram(itM_d, nIM, ioffM_d, count, l, b.B, ld, cdt, bpart, b.G, (int64_t)ll, b.state, 0, st));
  HIPCHK(beig(3));
  HIPCHK(launch_brescale(itM_d, nIM, l, b.B, nullptr, ld, cdt, b.W, (int64_t)ll, l, k, b.Uo, k, cdt, b.state, 0,
                         st));
  HIPCHK(launch_brescale(itN_d, nIN, l, Qc, nullptr, ld, pc, b.Vs, (int64_t)ll, l, k, b.Vo, k, cdt, b.state, 0,
                         st));
  HIPCHK(launch_bsign(offN, offM, count, k, b.Vo, b.Uo, k, cdt, st));
  // aggregate info
  std::vector<SolverState> hs(count);
  HIPCHK(hipMemcpyAsync(hs.data(), b.state, sizeof(SolverState) * (size_t)count, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  auto &bo = h->bat;
  std::memset(&bo.info, 0, sizeof(bo.info));
  bo.info.converged = 1;
  for (int i = 0; i < count; ++i) {
    bo.info.passes = std::max(bo.info.passes, hs[i].pass);
    bo.info.converged &= hs[i].converged;
    bo.info.rank_deficient |= hs[i].deficient;
    bo.info.eig_calls += hs[i].eig_calls;
    bo.info.eig_sweeps += hs[i].eig_sweeps;
  }
  bo.info.l = l;
  bo.info.graph_launches = graph_launches;
  bo.info.time_loop_ms = t_loop1 - t_loop0;
  bo.info.long_row_used = T;
  bo.info.lane_vectors_used = vm;
  bo.info.slab_kib_used = (int32_t)(bslab_b >> 10);
  bo.info.promoted = promoted;
  bo.have = true;
  bo.count = count;
  bo.k = k;
  bo.l = l;
  bo.cap = cap;
  bo.out_dt = cdt;
  bo.m.assign(count, 0);
  bo.n.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    bo.m[i] = As[i].m;
    bo.n[i] = As[i].n;
  }
  bo.row_off = roff;
  bo.col_off = coff;
  bo.Uo = b.Uo;
  bo.Vo = b.Vo;
  bo.S = b.S;
  bo.state = b.state;
  bo.tr_alpha = b.tr_alpha;
  bo.tr_ratio = b.tr_ratio;
  bo.tr_sweeps = b.tr_sweeps;
  dashsvd_status s = DASHSVD_OK;
  if (tol > 0.0 && !bo.info.converged) s = DASHSVD_NOT_CONVERGED;
  else if (bo.info.rank_deficient) s = DASHSVD_RANK_DEFICIENT;
  bo.info.status = s;
  return s;
}

// Arguments of a batched run (as dashsvd_run for each matrix, plus the
// batched form's own requirements).
// Largest stacked index (rows, columns, nonzeros) of a sub-batch: the 32-bit
// indices of the stacked operator, its transposition and its plans.
constexpr int64_t kStackMax = (int64_t)INT32_MAX - 1;
static int64_t batch_limit(const dashsvd_handle *h) {
  const int64_t o = h->opt.batch_nnz_max;
  return o > 0 && o < kStackMax ? o : kStackMax;
}

static dashsvd_status check_batch(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k, int32_t p,
                                  double tol) {
  if (!As || count < 1) return fail(h, DASHSVD_ERR_INVALID_ARG, "empty batch");
  if (h->opt.shift_policy == DASHSVD_SHIFT_LEARNED)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "the batched form takes the PAPER, NONE, FIXED or SCHEDULE policy");
  if (h->opt.omega) return fail(h, DASHSVD_ERR_INVALID_ARG, "the batched form draws its own Omega");
  for (int i = 0; i < count; ++i) {
    dashsvd_status s = check_args(h, &As[i], k, p, tol);
    if (s != DASHSVD_OK) {
      h->err = "matrix " + std::to_string(i) + ": " + h->err;
      return s;
    }
    if (As[i].m < As[i].n)
      return fail(h, DASHSVD_ERR_INVALID_ARG, "batched form: matrix " + std::to_string(i) + " has m < n");
    if (As[i].value_dtype != As[0].value_dtype || (As[i].on_device != 0) != (As[0].on_device != 0))
      return fail(h, DASHSVD_ERR_INVALID_ARG, "batched form: mixed value types or memory spaces");
  }
  if (k + p > kBMaxL) return fail(h, DASHSVD_ERR_INVALID_ARG, "batched form: k + oversampling exceeds 64");
  const int64_t lim = batch_limit(h);
  for (int i = 0; i < count; ++i)
    if (As[i].nnz > lim || As[i].m > kStackMax || As[i].n > kStackMax)
      return fail(h, DASHSVD_ERR_INVALID_ARG, "batched form: matrix " + std::to_string(i) + " has " +
                                                  std::to_string(As[i].nnz) + " nonzeros, above the sub-batch "
                                                  "limit of " + std::to_string(lim));
  return DASHSVD_OK;
}

// Consecutive groups of members (first, count), each within the sub-batch
// limit of nonzeros and the 32-bit limit of the stacked rows and columns.
static std::vector<std::pair<int32_t, int32_t>> batch_groups(const dashsvd_handle *h, const dashsvd_csr *As,
                                                             int32_t count) {
  const int64_t lim = batch_limit(h);
  std::vector<std::pair<int32_t, int32_t>> g;
  int64_t z = 0, r = 0, c = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (g.empty() || z + As[i].nnz > lim || r + As[i].m > kStackMax || c + As[i].n > kStackMax) {
      g.push_back({i, 0});
      z = r = c = 0;
    }
    g.back().second += 1;
    z += As[i].nnz;
    r += As[i].m;
    c += As[i].n;
  }
  return g;
}

// A run of several sub-batches: each group runs in the arena, then its
// members' results are copied to the handle's own result buffers, which the
// batched getters then read.
static dashsvd_status run_sub_batches(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k,
                                      int32_t p, double tol,
                                      const std::vector<std::pair<int32_t, int32_t>> &groups) {
  const int prec = h->opt.precision;
  const int cdt = prec == DASHSVD_PREC_FP64 ? DASHSVD_F64 : DASHSVD_F32;
  const size_t os = dsz(cdt);
  const int l = k + p;
  const int cap = h->opt.p_max > 0 ? h->opt.p_max : 1;
  std::vector<int64_t> roff(count + 1, 0), coff(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    roff[i + 1] = roff[i] + As[i].m;
    coff[i + 1] = coff[i] + As[i].n;
  }
  // result layout: U, V, S, states, traces
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  const size_t oU = carve(os * (size_t)roff[count] * k), oV = carve(os * (size_t)coff[count] * k);
  const size_t oS = carve(8 * (size_t)l * count), oSt = carve(sizeof(SolverState) * (size_t)count);
  const size_t oA = carve(8 * (size_t)cap * count), oR = carve(8 * (size_t)cap * count);
  const size_t oW = carve(4 * (size_t)(cap + 2) * count);
  if (off > h->ball.cap) {
    if (h->ball.base) {
      (void)hipStreamSynchronize(h->stg);
      (void)hipFree(h->ball.base);
      h->ball.base = nullptr;
      h->ball.cap = 0;
    }
    HIPCHK(hipMalloc(&h->ball.base, off));
    h->ball.cap = off;
  }
  char *base = (char *)h->ball.base;
  hipStream_t st = h->stg;
  dashsvd_info agg;
  std::memset(&agg, 0, sizeof(agg));
  agg.converged = 1;
  for (const auto &g : groups) {
    const int32_t g0 = g.first, gn = g.second;
    dashsvd_status s = run_batched_impl(h, As + g0, gn, k, p, tol, false, nullptr, g0);
    if (s < 0) return s;
    auto &bo = h->bat;
    const int64_t mr = roff[g0 + gn] - roff[g0], nc = coff[g0 + gn] - coff[g0];
    HIPCHK(hipMemcpyAsync(base + oU + os * (size_t)roff[g0] * k, bo.Uo, os * (size_t)mr * k,
                          hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(base + oV + os * (size_t)coff[g0] * k, bo.Vo, os * (size_t)nc * k,
                          hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(base + oS + 8 * (size_t)l * g0, bo.S, 8 * (size_t)l * gn, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(base + oSt + sizeof(SolverState) * (size_t)g0, bo.state, sizeof(SolverState) * (size_t)gn,
                          hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(base + oA + 8 * (size_t)cap * g0, bo.tr_alpha, 8 * (size_t)cap * gn,
                          hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(base + oR + 8 * (size_t)cap * g0, bo.tr_ratio, 8 * (size_t)cap * gn,
                          hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(base + oW + 4 * (size_t)(cap + 2) * g0, bo.tr_sweeps, 4 * (size_t)(cap + 2) * gn,
                          hipMemcpyDeviceToDevice, st));
    const dashsvd_info &gi = bo.info;
    agg.passes = std::max(agg.passes, gi.passes);
    agg.converged &= gi.converged;
    agg.rank_deficient |= gi.rank_deficient;
    agg.eig_calls += gi.eig_calls;
    agg.eig_sweeps += gi.eig_sweeps;
    agg.time_loop_ms += gi.time_loop_ms;
    agg.promoted |= gi.promoted;
    agg.graph_launches += gi.graph_launches;
    agg.long_row_used = gi.long_row_used;
    agg.lane_vectors_used = gi.lane_vectors_used;
    agg.slab_kib_used = gi.slab_kib_used;
  }
  HIPCHK(hipStreamSynchronize(st));
  auto &bo = h->bat;
  agg.l = l;
  bo.info = agg;
  bo.have = true;
  bo.count = count;
  bo.m.assign(count, 0);
  bo.n.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    bo.m[i] = As[i].m;
    bo.n[i] = As[i].n;
  }
  bo.row_off = roff;
  bo.col_off = coff;
  bo.Uo = base + oU;
  bo.Vo = base + oV;
  bo.S = (double *)(base + oS);
  bo.state = (SolverState *)(base + oSt);
  bo.tr_alpha = (double *)(base + oA);
  bo.tr_ratio = (double *)(base + oR);
  bo.tr_sweeps = (int32_t *)(base + oW);
  dashsvd_status s = DASHSVD_OK;
  if (tol > 0.0 && !agg.converged) s = DASHSVD_NOT_CONVERGED;
  else if (agg.rank_deficient) s = DASHSVD_RANK_DEFICIENT;
  bo.info.status = s;
  return s;
}

dashsvd_status dashsvd_run_batched(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k, int32_t p,
                                   double tol) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  h->err.clear();
  {
    dashsvd_status s = check_batch(h, As, count, k, p, tol);
    if (s != DASHSVD_OK) return s;
  }
  if (h->opt.pve_mode == DASHSVD_PVE_NOSURR)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "pve_mode NOSURR is for single solves");
  if (!h->stg) {
    HIPCHK(hipStreamCreateWithFlags(&h->stg, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&h->ev_b0, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_b1, hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(h->ev_b0, h->st));
  HIPCHK(hipStreamWaitEvent(h->stg, h->ev_b0, 0));
  const double t0 = now_ms();
  const auto groups = batch_groups(h, As, count);
  dashsvd_status s = groups.size() == 1 ? run_batched_impl(h, As, count, k, p, tol, false, nullptr)
                                        : run_sub_batches(h, As, count, k, p, tol, groups);
  (void)hipStreamSynchronize(h->stg);
  h->bat.info.time_total_ms = now_ms() - t0;
  h->bat.info.status = s;
  h->bat.info.sub_batches = (int32_t)groups.size();
  return s;
}

dashsvd_status dashsvd_autotune(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k, int32_t p,
                                const char *db_path, int32_t *best) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  h->err.clear();
  if (!As || count < 1) return fail(h, DASHSVD_ERR_INVALID_ARG, "empty input");
  const dashsvd_options saved = h->opt;
  const std::vector<double> saved_sched = h->sched;
  const auto saved_tune = h->tune;
  const int ld = (int)round_up(k + p, 8);
  int64_t rows = 0, nnz = 0;
  for (int i = 0; i < count; ++i) {
    const bool wide = As[i].m < As[i].n;
    rows += wide ? As[i].n : As[i].m;
    nnz += As[i].nnz;
  }
  const std::string key = tune_key(saved.precision, ld, rows, nnz, count > 1);
  // start from the defaults (or the options that fix a knob)
  TuneVal cur;
  cur.T = saved.long_row > 0 ? saved.long_row : (nnz >= DASHSVD_REORDER_MIN_NNZ ? kDefaultLongRowLarge : kDefaultLongRow);
  cur.vm = saved.lane_vectors > 0 ? saved.lane_vectors : 1;
  cur.slab_kib = saved.slab_kib > 0 ? saved.slab_kib : 0;
  cur.reorder = saved.reorder != DASHSVD_REORDER_AUTO ? saved.reorder
                                                       : (nnz >= DASHSVD_REORDER_MIN_NNZ ? 1 : -1);
  dashsvd_status s = DASHSVD_OK;
  // the fastest of three short runs of configuration v (milliseconds)
  auto time_of = [&](const TuneVal &v) -> double {
    h->opt = saved;
    h->sched = saved_sched;
    h->tune.clear();
    h->opt.long_row = v.T;
    h->opt.lane_vectors = v.vm;
    h->opt.slab_kib = v.slab_kib;
    h->opt.reorder = v.reorder;
    h->opt.p_max = 2;
    h->opt.timing = count == 1 ? DASHSVD_TIMING_SPMM : 0;
    h->opt.shift_policy = saved.shift_policy == DASHSVD_SHIFT_LEARNED ? DASHSVD_SHIFT_PAPER : saved.shift_policy;
    double t = 0.0;
    for (int rep = 0; rep < 3 && s >= 0; ++rep) {
      double tr = 0.0;
      if (count == 1) {
        s = dashsvd_run(h, As, k, p, 0.0);
        tr = h->info.kt_ms[DASHSVD_KT_SPMM] + h->info.kt_ms[DASHSVD_KT_SPMM_T];
      } else {
        s = dashsvd_run_batched(h, As, count, k, p, 0.0);
        tr = h->bat.info.time_loop_ms;
      }
      if (rep == 0 || tr < t) t = tr;
    }
    return t;
  };
  double best_t = time_of(cur);
  auto knob = [&](int TuneVal::*field, std::initializer_list<int> cands, bool fixed) {
    if (fixed) return;
    for (int c : cands) {
      if (s < 0) return;
      if (c == cur.*field) continue;
      TuneVal v = cur;
      v.*field = c;
      const double t = time_of(v);
      if (s >= 0 && t < best_t) {
        best_t = t;
        cur = v;
      }
    }
  };
  knob(&TuneVal::T, {32, 64, 128, 256, 512, 768, 1024}, saved.long_row > 0);
  knob(&TuneVal::vm, {1, 2}, saved.lane_vectors > 0);
  knob(&TuneVal::slab_kib, {0, 2048}, saved.slab_kib > 0);
  knob(&TuneVal::reorder, {1, -1}, count > 1 || saved.reorder != DASHSVD_REORDER_AUTO);
  const std::string err = h->err;
  h->opt = saved;
  h->sched = saved_sched;
  h->tune = saved_tune;
  h->have = false;
  h->bat.have = false;
  if (s < 0) {
    h->err = err;
    return s;
  }
  if (count > 1) cur.reorder = 0;  // the batched form has no degree order
  h->tune.emplace_back(key, cur);
  if (db_path) {
    FILE *f = std::fopen(db_path, "a");
    if (!f) return fail(h, DASHSVD_ERR_INVALID_ARG, std::string("cannot append to ") + db_path);
    std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), cur.T, cur.vm, cur.slab_kib, cur.reorder);
    std::fclose(f);
  }
  if (best) *best = cur.T;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_get_USV_batched(dashsvd_handle *h, int32_t idx, void *U, int64_t ldu, double *S, void *V,
                                       int64_t ldv, int32_t dtype, int32_t on_device) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  auto &bo = h->bat;
  if (!bo.have) return fail(h, DASHSVD_ERR_STATE, "no batched results: run_batched first");
  if (idx < 0 || idx >= bo.count) return fail(h, DASHSVD_ERR_INVALID_ARG, "matrix index");
  if (dtype != DASHSVD_F32 && dtype != DASHSVD_F64) return fail(h, DASHSVD_ERR_INVALID_ARG, "dtype");
  if ((U && ldu < bo.k) || (V && ldv < bo.k)) return fail(h, DASHSVD_ERR_INVALID_ARG, "leading dimension");
  hipStream_t st = h->stg;
  const size_t es = dsz(dtype), os = dsz(bo.out_dt);
  struct Item {
    void *dst;
    int64_t ldd;
    const void *src;
    int64_t rows;
  } items[2] = {{U, ldu, (const char *)bo.Uo + os * (size_t)bo.row_off[idx] * bo.k, bo.m[idx]},
                {V, ldv, (const char *)bo.Vo + os * (size_t)bo.col_off[idx] * bo.k, bo.n[idx]}};
  for (auto &it : items) {
    if (!it.dst) continue;
    if (on_device) {
      HIPCHK(launch_copy2d(it.src, bo.k, bo.out_dt, it.dst, it.ldd, dtype, it.rows, bo.k, st));
    } else {
      void *tmp = nullptr;
      HIPCHK(hipMalloc(&tmp, es * (size_t)it.rows * bo.k + 16));
      hipError_t e = launch_copy2d(it.src, bo.k, bo.out_dt, tmp, bo.k, dtype, it.rows, bo.k, st);
      if (e == hipSuccess)
        e = hipMemcpy2DAsync(it.dst, es * it.ldd, tmp, es * bo.k, es * bo.k, it.rows, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      (void)hipFree(tmp);
      HIPCHK(e);
    }
  }
  if (S)
    HIPCHK(hipMemcpyAsync(S, bo.S + (size_t)bo.l * idx, 8 * (size_t)bo.k,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_get_info_batched(dashsvd_handle *h, int32_t idx, dashsvd_info *out) {
  if (!h || !out) return DASHSVD_ERR_INVALID_ARG;
  auto &bo = h->bat;
  if (!bo.have) return fail(h, DASHSVD_ERR_STATE, "no batched results: run_batched first");
  if (idx < 0) {
    *out = bo.info;
    return DASHSVD_OK;
  }
  if (idx >= bo.count) return fail(h, DASHSVD_ERR_INVALID_ARG, "matrix index");
  hipStream_t st = h->stg;
  SolverState s;
  HIPCHK(hipMemcpyAsync(&s, bo.state + idx, sizeof(s), hipMemcpyDeviceToHost, st));
  std::memset(out, 0, sizeof(*out));
  const int ntr = bo.cap < DASHSVD_MAX_TRACE ? bo.cap : DASHSVD_MAX_TRACE;
  HIPCHK(hipMemcpyAsync(out->alpha_used, bo.tr_alpha + (size_t)bo.cap * idx, 8 * (size_t)ntr,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(out->ratio, bo.tr_ratio + (size_t)bo.cap * idx, 8 * (size_t)ntr, hipMemcpyDeviceToHost,
                        st));
  const int nsw = bo.cap + 2 < DASHSVD_MAX_TRACE + 2 ? bo.cap + 2 : DASHSVD_MAX_TRACE + 2;
  HIPCHK(hipMemcpyAsync(out->sweeps_per_call, bo.tr_sweeps + (size_t)(bo.cap + 2) * idx, 4 * (size_t)nsw,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  out->passes = s.pass;
  out->converged = s.converged;
  out->rank_deficient = s.deficient;
  out->l = bo.l;
  out->final_alpha = s.alpha;
  out->eig_calls = s.eig_calls;
  out->eig_sweeps = s.eig_sweeps;
  out->status = bo.info.status;
  return DASHSVD_OK;
}

// ===================================================================== learned shift
// The MLP of the learned shift policy (kernels in k_mlp.hip): parameters,
// gradients and Adam moments live in one device allocation of the handle.
static dashsvd_status mlp_buffers(dashsvd_handle *h, int B) {
  auto &M = h->mlp;
  if (B <= M.buf_batch) return DASHSVD_OK;
  if (M.buf) (void)hipFree(M.buf);
  M.buf = nullptr;
  M.buf_batch = 0;
  const size_t n = (size_t)B * (M.D + 4 * M.H + 6) + 4;
  if (hipMalloc(&M.buf, 4 * n) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, DASHSVD_ERR_OOM, "MLP batch buffers");
  }
  M.buf_batch = B;
  return DASHSVD_OK;
}

struct MlpBufs {
  float *X, *T, *A1, *A2, *O, *dO, *dA2, *dA1, *loss;
};
static MlpBufs mlp_view(dashsvd_handle *h, int B) {
  auto &M = h->mlp;
  MlpBufs v;
  v.X = M.buf;
  v.T = v.X + (size_t)B * M.D;
  v.A1 = v.T + 2 * (size_t)B;
  v.A2 = v.A1 + (size_t)B * M.H;
  v.O = v.A2 + (size_t)B * M.H;
  v.dO = v.O + 2 * (size_t)B;
  v.dA2 = v.dO + 2 * (size_t)B;
  v.dA1 = v.dA2 + (size_t)B * M.H;
  v.loss = v.dA1 + (size_t)B * M.H;
  return v;
}

dashsvd_status dashsvd_mlp_init(dashsvd_handle *h, int32_t l, uint64_t seed, double c_max) {
  if (!h) return DASHSVD_ERR_INVALID_ARG;
  h->err.clear();
  if (l < 2 || l > DASHSVD_MAX_L) return fail(h, DASHSVD_ERR_INVALID_ARG, "l");
  if (!(c_max > 0.5 && c_max < 1.0)) return fail(h, DASHSVD_ERR_INVALID_ARG, "c_max must be in (0.5, 1)");
  auto &M = h->mlp;
  if (M.P) (void)hipFree(M.P);
  M = dashsvd_handle::Mlp();
  M.l = l;
  M.D = 3 * l + 3;
  M.H = kMlpH;
  M.cmax = c_max;
  M.np = mlp_num_params(M.D, M.H);
  void *p = nullptr;
  if (hipMalloc(&p, 4 * 4 * (size_t)M.np) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, DASHSVD_ERR_OOM, "MLP parameters");
  }
  M.P = (float *)p;
  M.G = M.P + M.np;
  M.m = M.G + M.np;
  M.v = M.m + M.np;
  // He-uniform weights from a splitmix64 stream, zero biases, a small output
  // layer
  std::vector<float> host((size_t)M.np, 0.0f);
  uint64_t z = seed;
  auto uni = [&]() {
    z += 0x9E3779B97F4A7C15ULL;
    uint64_t x = z;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
    x ^= x >> 31;
    return (double)(x >> 11) * 0x1.0p-53 * 2.0 - 1.0;
  };
  size_t o = 0;
  const double r1 = std::sqrt(6.0 / M.D), r2 = std::sqrt(6.0 / M.H);
  for (int64_t i = 0; i < (int64_t)M.H * M.D; ++i) host[o++] = (float)(r1 * uni());
  o += M.H;
  for (int64_t i = 0; i < (int64_t)M.H * M.H; ++i) host[o++] = (float)(r2 * uni());
  o += M.H;
  for (int64_t i = 0; i < 2 * (int64_t)M.H; ++i) host[o++] = (float)(0.1 * r2 * uni());
  HIPCHK(hipMemcpy(M.P, host.data(), 4 * (size_t)M.np, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(M.m, 0, 4 * 2 * (size_t)M.np));
  M.ok = true;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_mlp_num_params(dashsvd_handle *h, int64_t *n) {
  if (!h || !n) return DASHSVD_ERR_INVALID_ARG;
  if (!h->mlp.ok) return fail(h, DASHSVD_ERR_STATE, "no MLP: dashsvd_mlp_init first");
  *n = h->mlp.np;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_mlp_set_params(dashsvd_handle *h, const float *params, int64_t n) {
  if (!h || !params) return DASHSVD_ERR_INVALID_ARG;
  if (!h->mlp.ok) return fail(h, DASHSVD_ERR_STATE, "no MLP: dashsvd_mlp_init first");
  if (n != h->mlp.np) return fail(h, DASHSVD_ERR_INVALID_ARG, "parameter count");
  HIPCHK(hipMemcpy(h->mlp.P, params, 4 * (size_t)n, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(h->mlp.m, 0, 4 * 2 * (size_t)n));
  h->mlp.step = 0;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_mlp_get_params(dashsvd_handle *h, float *params, int64_t n) {
  if (!h || !params) return DASHSVD_ERR_INVALID_ARG;
  if (!h->mlp.ok) return fail(h, DASHSVD_ERR_STATE, "no MLP: dashsvd_mlp_init first");
  if (n != h->mlp.np) return fail(h, DASHSVD_ERR_INVALID_ARG, "parameter count");
  HIPCHK(hipMemcpy(params, h->mlp.P, 4 * (size_t)n, hipMemcpyDeviceToHost));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_mlp_forward(dashsvd_handle *h, const float *X, int32_t batch, float *out) {
  if (!h || !X || !out || batch < 1) return DASHSVD_ERR_INVALID_ARG;
  if (!h->mlp.ok) return fail(h, DASHSVD_ERR_STATE, "no MLP: dashsvd_mlp_init first");
  auto &M = h->mlp;
  dashsvd_status s = mlp_buffers(h, batch);
  if (s != DASHSVD_OK) return s;
  MlpBufs v = mlp_view(h, batch);
  HIPCHK(hipMemcpy(v.X, X, 4 * (size_t)batch * M.D, hipMemcpyHostToDevice));
  HIPCHK(mlp_forward({M.D, M.H}, M.P, v.X, batch, v.A1, v.A2, v.O, nullptr));
  std::vector<float> o(2 * (size_t)batch);
  HIPCHK(hipMemcpy(o.data(), v.O, 4 * o.size(), hipMemcpyDeviceToHost));
  for (int b = 0; b < batch; ++b) {
    const double sg = 1.0 / (1.0 + std::exp(-(double)o[2 * b]));
    out[2 * b] = (float)(0.5 + (M.cmax - 0.5) * sg);
    out[2 * b + 1] = o[2 * b + 1];
  }
  return DASHSVD_OK;
}

static dashsvd_status mlp_grad_impl(dashsvd_handle *h, const float *X, const float *Y, int32_t batch,
                                    float *loss) {
  auto &M = h->mlp;
  dashsvd_status s = mlp_buffers(h, batch);
  if (s != DASHSVD_OK) return s;
  MlpBufs v = mlp_view(h, batch);
  HIPCHK(hipMemcpy(v.X, X, 4 * (size_t)batch * M.D, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(v.T, Y, 4 * 2 * (size_t)batch, hipMemcpyHostToDevice));
  HIPCHK(mlp_backward({M.D, M.H}, M.P, v.X, v.T, batch, (float)M.cmax, kMlpLambda, v.A1, v.A2, v.O, v.dO, v.dA2,
                      v.dA1, M.G, v.loss, nullptr));
  if (loss) HIPCHK(hipMemcpy(loss, v.loss, 4, hipMemcpyDeviceToHost));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_mlp_grad(dashsvd_handle *h, const float *X, const float *Y, int32_t batch, float *grad,
                                float *loss) {
  if (!h || !X || !Y || batch < 1) return DASHSVD_ERR_INVALID_ARG;
  if (!h->mlp.ok) return fail(h, DASHSVD_ERR_STATE, "no MLP: dashsvd_mlp_init first");
  dashsvd_status s = mlp_grad_impl(h, X, Y, batch, loss);
  if (s != DASHSVD_OK) return s;
  if (grad) HIPCHK(hipMemcpy(grad, h->mlp.G, 4 * (size_t)h->mlp.np, hipMemcpyDeviceToHost));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_mlp_train_step(dashsvd_handle *h, const float *X, const float *Y, int32_t batch, float lr,
                                      float *loss) {
  if (!h || !X || !Y || batch < 1 || !(lr > 0.0f)) return DASHSVD_ERR_INVALID_ARG;
  if (!h->mlp.ok) return fail(h, DASHSVD_ERR_STATE, "no MLP: dashsvd_mlp_init first");
  dashsvd_status s = mlp_grad_impl(h, X, Y, batch, loss);
  if (s != DASHSVD_OK) return s;
  auto &M = h->mlp;
  M.step += 1;
  HIPCHK(mlp_adam(M.P, M.G, M.m, M.v, M.np, lr, M.step, nullptr));
  HIPCHK(hipDeviceSynchronize());
  return DASHSVD_OK;
}

dashsvd_status dashsvd_learned_features(dashsvd_handle *h, float *feat, int32_t n) {
  if (!h || !feat) return DASHSVD_ERR_INVALID_ARG;
  if (!h->have) return fail(h, DASHSVD_ERR_STATE, "no results: run first");
  const int l = h->l;
  if (n != 3 * l + 3) return fail(h, DASHSVD_ERR_INVALID_ARG, "feature count must be 3 l + 3");
  if (h->info.passes < 2 || h->trace_cap < 2) return fail(h, DASHSVD_ERR_STATE, "features need two passes");
  std::vector<double> s((size_t)2 * l);
  HIPCHK(hipMemcpyAsync(s.data(), h->trace_s, 8 * s.size(), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  const double a1 = h->info.alpha_used[0], a2 = h->info.alpha_used[1];
  const double e11 = s[0] + a1, e21 = s[l] + a2;
  for (int i = 0; i < l; ++i) {
    const double e1 = s[i] + a1, e2 = s[l + i] + a2;
    feat[i] = e11 > 0.0 ? (float)(e1 / e11) : 0.0f;
    feat[l + i] = e21 > 0.0 ? (float)(e2 / e21) : 0.0f;
    feat[2 * l + i] = e1 > 0.0 ? (float)(e2 / e1) : 0.0f;
  }
  const int64_t Mm = h->m > h->n ? h->m : h->n, Mn = h->m > h->n ? h->n : h->m;
  const int64_t nnz = h->ev_ctx.nnz;
  feat[3 * l] = (float)std::log((double)Mm);
  feat[3 * l + 1] = (float)std::log((double)Mn);
  feat[3 * l + 2] = (float)std::log((double)(nnz > 0 ? nnz : 1) / (double)Mm);
  return DASHSVD_OK;
}

dashsvd_status dashsvd_get_info(dashsvd_handle *h, dashsvd_info *out) {
  if (!h || !out) return DASHSVD_ERR_INVALID_ARG;
  *out = h->info;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_get_trace(dashsvd_handle *h, double *s_hat, int32_t max_passes) {
  if (!h || !s_hat) return DASHSVD_ERR_INVALID_ARG;
  if (!h->have) return fail(h, DASHSVD_ERR_STATE, "no results: run first");
  int np = h->info.passes < max_passes ? h->info.passes : max_passes;
  if (np > h->trace_cap) np = h->trace_cap;
  if (np > 0) {
    HIPCHK(hipMemcpyAsync(s_hat, h->trace_s, 8 * (size_t)np * h->l, hipMemcpyDeviceToHost, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
  }
  return DASHSVD_OK;
}

// ------------------------------------------------------------------ kernel-level entries
dashsvd_status dashsvd_k_gaussian(uint64_t seed, int64_t rows, int64_t cols, void *out, int64_t ld, int32_t dtype,
                                  void *stream) {
  dashsvd_handle *h = nullptr;
  if (rows < 0 || cols < 0 || ld < cols || !out || dtype < 0 || dtype > 2)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "gaussian arguments");
  HIPCHK(launch_gaussian(seed, rows, cols, out, ld, dtype, (hipStream_t)stream));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_philox_raw(uint64_t seed, int64_t nwords, uint64_t *out, void *stream) {
  dashsvd_handle *h = nullptr;
  if (nwords < 0 || !out) return fail(h, DASHSVD_ERR_INVALID_ARG, "philox arguments");
  HIPCHK(launch_philox_raw(seed, nwords, out, (hipStream_t)stream));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_sort_index(int64_t n, const uint32_t *keys_in, uint32_t *keys_out, int32_t *idx_out,
                                    int32_t bits, int32_t descending, void *stream) {
  dashsvd_handle *h = nullptr;
  if (n < 0 || n > INT32_MAX || bits < 1 || bits > 32 || (n > 0 && (!keys_in || !keys_out || !idx_out)))
    return fail(h, DASHSVD_ERR_INVALID_ARG, "sort arguments");
  if (n == 0) return DASHSVD_OK;
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = sort_ws_bytes(n, (unsigned)bits, 4);
  void *ws = nullptr;
  if (hipMalloc(&ws, bytes) != hipSuccess) return fail(h, DASHSVD_ERR_OOM, "sort workspace");
  hipError_t e = sort_keys_index(n, keys_in, keys_out, idx_out, (unsigned)bits, descending != 0, ws, bytes, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(ws);
  HIPCHK(e);
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_transpose(int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                                   const void *val, int32_t dtype, int64_t *rowT, int32_t *colT, void *valT,
                                   void *stream) {
  dashsvd_handle *h = nullptr;
  if (m < 1 || n < 1 || nnz < 0 || nnz > INT32_MAX || (dtype != 0 && dtype != 1))
    return fail(h, DASHSVD_ERR_INVALID_ARG, "transpose arguments");
  hipStream_t st = (hipStream_t)stream;
  const size_t tws_bytes = transpose_ws_bytes(n, nnz);
  size_t bytes[3] = {4 * (size_t)(nnz + 1), 64, tws_bytes};
  void *ptr[3] = {};
  for (int i = 0; i < 3; ++i) {
    if (hipMalloc(&ptr[i], bytes[i]) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipFree(ptr[j]);
      return fail(h, DASHSVD_ERR_OOM, "transpose workspace");
    }
  }
  int32_t *rowidx = (int32_t *)ptr[0], *flags = (int32_t *)ptr[1];
  dashsvd_status res = DASHSVD_OK;
  int32_t hc[4] = {0, 0, 0, 0};
  hipError_t e = hipMemsetAsync(flags, 0, 64, st);
  if (e == hipSuccess) e = launch_validate(m, n, nnz, row_ptr, col, val, dtype, rowidx, flags, st);
  if (e == hipSuccess) e = hipMemcpyAsync(hc, flags, 16, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess && (hc[0] & 1)) res = DASHSVD_ERR_BAD_CSR;
  else if (e == hipSuccess && (hc[0] & 2)) res = DASHSVD_ERR_NONFINITE;
  if (e == hipSuccess && res == DASHSVD_OK) {
    e = launch_transpose(n, nnz, col, rowidx, val, dtype, rowT, colT, valT, ptr[2], tws_bytes, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
  }
  for (int i = 0; i < 3; ++i) (void)hipFree(ptr[i]);
  if (e != hipSuccess) return fail(h, DASHSVD_ERR_HIP, hipGetErrorString(e));
  if (res != DASHSVD_OK) return fail(h, res, "invalid CSR");
  return DASHSVD_OK;
}

}  // extern "C"

// Scratch of dashsvd_k_spmm_static (32 MiB per device; see below).
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {

// Plan and product of the kernel-level SpMM entries over a workspace at
// `base` (measured by spmm_ws_bytes): the row-split plan, a host read of its
// two sizes, then the product.  Synchronises the stream before returning.
struct SpmmCall {
  int64_t rows, cols, nnz;
  const int64_t *row_ptr;
  const int32_t *col;
  const void *val;
  const void *X;
  int64_t ldx;
  int32_t xdtype;
  void *Y;
  int64_t ldy;
  int32_t ydtype;
  int32_t l;
  const void *Q;
  int64_t ldq;
  const double *alpha;
  int32_t long_row;
  hipStream_t st;
};

dashsvd_status spmm_call_check(const SpmmCall &c) {
  dashsvd_handle *h = nullptr;
  const int ld = (int)round_up(c.l, 8);
  if (c.rows < 1 || c.l < 1 || c.l > DASHSVD_MAX_L || c.ldx % 8 || c.ldy % 8 || c.ldx < ld || c.ldy < ld ||
      (c.alpha && (!c.Q || c.ldq % 8 || c.ldq < ld)))
    return fail(h, DASHSVD_ERR_INVALID_ARG, "spmm arguments (leading dimensions must be multiples of 8 >= l)");
  return DASHSVD_OK;
}

// Lays the plan out in `a` (a measuring arena takes no memory).
void spmm_layout(const SpmmCall &c, Arena &a, Plan &pl, int64_t **scan_tmp) {
  const int ld = (int)round_up(c.l, 8);
  const size_t accsz = c.xdtype == DASHSVD_F64 ? 8 : 4;
  const int32_t T = c.long_row > 0 ? c.long_row : kDefaultLongRow;
  const size_t xsz = c.xdtype == DASHSVD_F64 ? 8 : (c.xdtype == DASHSVD_BF16 ? 2 : 4);
  plan_alloc(nullptr, a, pl, c.rows, c.nnz, T, ld, accsz, c.cols, c.ldx * (int64_t)xsz, 0);
  *scan_tmp = (int64_t *)a.take(8 * scan_tmp_elems(c.rows + 1));
}

size_t spmm_ws_bytes(const SpmmCall &c) {
  Arena a;
  a.reset(true);
  Plan pl;
  int64_t *scan_tmp = nullptr;
  spmm_layout(c, a, pl, &scan_tmp);
  return a.used;
}

// The plan's atomic long-row counter must start at zero; every other word of
// the workspace is written before it is read.
hipError_t spmm_run_on(const SpmmCall &c, char *base, size_t cap) {
  const int ld = (int)round_up(c.l, 8);
  const int vdt = c.xdtype == DASHSVD_F64 ? DASHSVD_F64 : DASHSVD_F32;
  const int32_t T = c.long_row > 0 ? c.long_row : kDefaultLongRow;
  Arena a;
  a.base = base;
  a.cap = cap;
  a.reset(false);
  Plan pl;
  int64_t *scan_tmp = nullptr;
  spmm_layout(c, a, pl, &scan_tmp);
  ZeroRanges z{};
  z.add(pl.nlong, 16);
  z.add(pl.slab_cnt, 8 * (size_t)(kMaxSlabs + 1));
  hipError_t e = launch_zero_ranges(z, c.st);
  if (e == hipSuccess) e = plan_build(pl, c.row_ptr, c.col, T, scan_tmp, c.st);
  int64_t tot = 0;
  int32_t nl = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&tot, pl.off + c.rows, 8, hipMemcpyDeviceToHost, c.st);
  if (e == hipSuccess) e = hipMemcpyAsync(&nl, pl.nlong, 4, hipMemcpyDeviceToHost, c.st);
  if (e == hipSuccess) e = hipStreamSynchronize(c.st);
  if (e == hipSuccess)
    e = launch_spmm(c.rows, c.row_ptr, c.col, c.val, vdt, c.X, c.ldx, c.xdtype, c.Y, c.ldy, c.ydtype, ld, tot,
                    pl.order, nl, pl.longs, pl.partial, T, 1, c.Q, c.ldq, c.alpha, nullptr, c.st, nullptr, nullptr,
                    c.cols);
  if (e == hipSuccess) e = hipStreamSynchronize(c.st);
  return e;
}

// Scratch of dashsvd_k_spmm_static: the plan and long-row partials of one
// call.  Every device holds its own copy for the life of the process.  In
// host code the array's name is not a device address: the kernels get the
// address hipGetSymbolAddress returns for the current device, resolved once
// per device and kept in g_scratch_dev.
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxScratchDevices] = {};

hipError_t static_scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

dashsvd_status dashsvd_k_spmm(int64_t rows, int64_t cols, int64_t nnz, const int64_t *row_ptr, const int32_t *col,
                              const void *val, const void *X, int64_t ldx, int32_t xdtype, void *Y, int64_t ldy,
                              int32_t ydtype, int32_t l, const void *Q, int64_t ldq, const double *alpha,
                              int32_t long_row, void *stream) {
  dashsvd_handle *h = nullptr;
  const SpmmCall c{rows, cols, nnz, row_ptr, col, val, X, ldx, xdtype, Y, ldy, ydtype, l, Q, ldq, alpha,
                   long_row, (hipStream_t)stream};
  dashsvd_status s = spmm_call_check(c);
  if (s != DASHSVD_OK) return s;
  const size_t bytes = spmm_ws_bytes(c) + 256;
  void *base = nullptr;
  if (hipMalloc(&base, bytes) != hipSuccess) return fail(h, DASHSVD_ERR_OOM, "spmm workspace");
  hipError_t e = hipMemsetAsync(base, 0, bytes, c.st);
  if (e == hipSuccess) e = spmm_run_on(c, (char *)base, bytes);
  (void)hipFree(base);
  if (e != hipSuccess) return fail(h, DASHSVD_ERR_HIP, hipGetErrorString(e));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_spmm_static(int64_t rows, int64_t cols, int64_t nnz, const int64_t *row_ptr,
                                     const int32_t *col, const void *val, const void *X, int64_t ldx,
                                     int32_t xdtype, void *Y, int64_t ldy, int32_t ydtype, int32_t l,
                                     const void *Q, int64_t ldq, const double *alpha, int32_t long_row,
                                     void *stream) {
  dashsvd_handle *h = nullptr;
  const SpmmCall c{rows, cols, nnz, row_ptr, col, val, X, ldx, xdtype, Y, ldy, ydtype, l, Q, ldq, alpha,
                   long_row, (hipStream_t)stream};
  dashsvd_status s = spmm_call_check(c);
  if (s != DASHSVD_OK) return s;
  const size_t bytes = spmm_ws_bytes(c);
  if (bytes > kStaticScratchBytes)
    return fail(h, DASHSVD_ERR_INVALID_ARG,
                "k_spmm_static: this call's plan needs " + std::to_string(bytes) +
                    " bytes of scratch, the static scratch holds " + std::to_string(kStaticScratchBytes) +
                    " (a larger long_row needs fewer partial rows; dashsvd_k_spmm has no limit)");
  void *base = nullptr;
  hipError_t e = static_scratch_address(&base);
  if (e != hipSuccess) return fail(h, DASHSVD_ERR_HIP, std::string("static scratch: ") + hipGetErrorString(e));
  e = spmm_run_on(c, (char *)base, kStaticScratchBytes);
  if (e != hipSuccess) return fail(h, DASHSVD_ERR_HIP, hipGetErrorString(e));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_gram(int64_t r, int32_t l, const void *C, int64_t ldc, int32_t cdtype, double *G,
                              void *stream) {
  dashsvd_handle *h = nullptr;
  if (r < 1 || l < 1 || l > DASHSVD_MAX_L || ldc < l || (cdtype != 0 && cdtype != 1))
    return fail(h, DASHSVD_ERR_INVALID_ARG, "gram arguments");
  hipStream_t st = (hipStream_t)stream;
  const int nb = gram_blocks(r, l);
  double *part = nullptr;
  HIPCHK(hipMalloc(&part, 8 * gram_partial_elems(nb, l)));
  hipError_t e = launch_gram(r, l, C, ldc, cdtype, part, nb, G, nullptr, st, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(part);
  HIPCHK(e);
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_eig_prof(int32_t l, const double *G, double *S, double *Vs, double *W,
                                  int32_t *sweeps, long long *prof, void *stream);
dashsvd_status dashsvd_k_eig(int32_t l, const double *G, double *S, double *Vs, double *W, int32_t *sweeps,
                             void *stream) {
  return dashsvd_k_eig_prof(l, G, S, Vs, W, sweeps, nullptr, stream);
}

// As dashsvd_k_eig, with an optional device array of 6 int64 step-profile
// counters (phase-A cycles, phase-B cycles, 100 MHz ticks, steps) added to.
dashsvd_status dashsvd_k_eig_prof(int32_t l, const double *G, double *S, double *Vs, double *W,
                                  int32_t *sweeps, long long *prof, void *stream) {
  dashsvd_handle *h = nullptr;
  if (l < 1 || l > DASHSVD_MAX_L || !G || !S || !W) return fail(h, DASHSVD_ERR_INVALID_ARG, "eig arguments");
  EigArgs ea;
  std::memset(&ea, 0, sizeof(ea));
  ea.l = l;
  ea.k = 0;
  ea.skip = 0x1.0p-53;
  ea.G = G;
  ea.S = S;
  ea.Vs = Vs;
  ea.W = W;
  ea.sweeps = sweeps;
  ea.prof = prof;
  ea.mode = 0;
  HIPCHK(launch_eig(ea, (hipStream_t)stream));
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_eig_onesided(int32_t l, const double *G, double *S, double *Vs, double *W, double skip,
                                      int32_t *sweeps, int32_t *accepted, long long *prof, void *stream) {
  dashsvd_handle *h = nullptr;
  if (l < 1 || l > 128 || !G || !S || !W || !accepted || !(skip >= 0.0) || !(skip < 1.0))
    return fail(h, DASHSVD_ERR_INVALID_ARG, "one-sided eig arguments (l <= 128, 0 <= skip < 1)");
  hipStream_t st = (hipStream_t)stream;
  int32_t *flag = nullptr;
  HIPCHK(hipMalloc(&flag, sizeof(int32_t)));
  EigArgs ea;
  std::memset(&ea, 0, sizeof(ea));
  ea.l = l;
  ea.skip = skip;
  ea.G = G;
  ea.S = S;
  ea.Vs = Vs;
  ea.W = W;
  ea.sweeps = sweeps;
  ea.prof = prof;
  ea.decline = flag;
  int32_t declined = 1;
  hipError_t e = launch_eig1s(ea, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&declined, flag, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(flag);
  HIPCHK(e);
  *accepted = declined ? 0 : 1;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_eig_tridiag(int32_t l, const double *G, double *S, double *Vs, double *W,
                                     int32_t *accepted, long long *prof, void *stream) {
  dashsvd_handle *h = nullptr;
  if (l < 1 || l > kTriMaxL || !G || !S || !W || !Vs || !accepted)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "tridiagonal eig arguments (l <= 160, Vs required)");
  hipStream_t st = (hipStream_t)stream;
  // the decline flag, then the workspace
  void *mem = nullptr;
  HIPCHK(hipMalloc(&mem, 256 + kTriWsBytes));
  EigArgs ea;
  std::memset(&ea, 0, sizeof(ea));
  ea.l = l;
  ea.G = G;
  ea.S = S;
  ea.Vs = Vs;
  ea.W = W;
  ea.decline = (int32_t *)mem;
  ea.tri_ws = (double *)((char *)mem + 256);
  ea.prof = prof;
  int32_t declined = 1;
  hipError_t e = launch_eigtri(ea, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&declined, mem, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(mem);
  HIPCHK(e);
  *accepted = declined ? 0 : 1;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_cholqr(int32_t l, const double *G, double *S, double *W, int32_t *accepted,
                                void *stream) {
  dashsvd_handle *h = nullptr;
  if (l < 1 || l > DASHSVD_MAX_L || !G || !S || !W || !accepted)
    return fail(h, DASHSVD_ERR_INVALID_ARG, "cholqr arguments");
  hipStream_t st = (hipStream_t)stream;
  SolverState *state = nullptr;
  HIPCHK(hipMalloc(&state, sizeof(SolverState)));
  EigArgs ea;
  std::memset(&ea, 0, sizeof(ea));
  ea.l = l;
  ea.G = G;
  ea.S = S;
  ea.W = W;
  ea.state = state;
  ea.mode = 1;
  int32_t fallback = 1;
  hipError_t e = hipMemsetAsync(state, 0, sizeof(SolverState), st);
  if (e == hipSuccess) e = launch_cholqr(ea, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&fallback, &state->cq_fallback, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(state);
  HIPCHK(e);
  *accepted = fallback ? 0 : 1;
  return DASHSVD_OK;
}

dashsvd_status dashsvd_k_rescale(int64_t r, int32_t l, const void *C, int64_t ldc, int32_t cdtype, const double *W,
                                 int64_t ldw, int32_t c, void *Out, int64_t ldo, int32_t odtype, void *stream) {
  dashsvd_handle *h = nullptr;
  if (r < 1 || l < 1 || l > DASHSVD_MAX_L || c < 1 || c > DASHSVD_MAX_L || ldc < l || ldw < c || ldo < c ||
      ldc % 8 || ((uintptr_t)C & 15))
    return fail(h, DASHSVD_ERR_INVALID_ARG, "rescale arguments (ldc: multiple of 8, C 16-byte aligned)");
  HIPCHK(launch_rescale(r, l, C, ldc, cdtype, W, ldw, c, Out, ldo, odtype, nullptr, (hipStream_t)stream));
  return DASHSVD_OK;
}

}  // extern "C"
