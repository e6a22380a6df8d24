/*
 * dashsvd.h -- C ABI of the MI355X (gfx950) dashSVD library.
 *
 * The library computes a rank-k truncated SVD  A ~ U diag(S) V^T  of a sparse
 * CSR matrix A (m x n) with randomized, dynamically shifted power iteration
 * and the per-vector-error (PVE) accuracy control of Feng, Yu, Xie and Tang,
 * "Faster Randomized SVD with Dynamic Shifts" (dashSVD):
 *   - Alg. 5 (dashSVD with PVE accuracy control) is the driver; with
 *     tol == 0 it runs exactly p_max passes, which is Alg. 4;
 *   - Alg. 3 (eigSVD) orthonormalises each block: Gram matrix, symmetric
 *     eigendecomposition, rescale, descending order;
 *   - Sec. 3.1: a matrix with m < n is processed through A^T and U, V are
 *     exchanged on output.
 * Every step runs in the library's own HIP kernels on one GPU.  No call
 * throws; every call returns a dashsvd_status.
 *
 * Threading: a handle must be used by one host thread at a time.  Calls are
 * ordered on the HIP stream given in the options (the null stream if none).
 */
#ifndef DASHSVD_H
#define DASHSVD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  Negative: error, the handle stays valid and reusable.
 * Positive: warning, results are valid. */
typedef int32_t dashsvd_status;
#define DASHSVD_OK 0
#define DASHSVD_NOT_CONVERGED 1   /* p_max passes ran without meeting tol (results valid) */
#define DASHSVD_RANK_DEFICIENT 2  /* some eigSVD column had S <= S_max*sqrt(l*eps) and was zeroed */
#define DASHSVD_ERR_INVALID_ARG -1
#define DASHSVD_ERR_BAD_CSR -2    /* row_ptr not monotone / wrong ends, column out of range or not strictly increasing */
#define DASHSVD_ERR_NONFINITE -3  /* a stored value is NaN or Inf */
#define DASHSVD_ERR_OOM -4
#define DASHSVD_ERR_HIP -5        /* a HIP runtime call failed; see dashsvd_last_error */
#define DASHSVD_ERR_STATE -6      /* call out of order (e.g. get_USV before a successful run) */

/* Element types. */
#define DASHSVD_F32 0
#define DASHSVD_F64 1
#define DASHSVD_BF16 2

/* Precision forms.
 *   FP32: panels Omega, Q, Y, C in FP32 with FP32 SpMM accumulation; the
 *         Gram matrix accumulates in FP64 and the l x l eigenproblem is FP64.
 *   FP64: everything in FP64.
 *   BF16_PANELS: Omega, Q, Y stored in BF16 (round to nearest even), SpMM
 *         accumulates FP32, C = A^T Y - alpha Q kept FP32; Gram, eig and the
 *         final Rayleigh-Ritz step in FP64 / FP32 as in FP32 mode. */
#define DASHSVD_PREC_FP32 0
#define DASHSVD_PREC_FP64 1
#define DASHSVD_PREC_BF16_PANELS 2

/* Shift policies.
 *   PAPER:    Alg. 5 step 6: if S_l > alpha then alpha = (S_l + alpha)/2.
 *   NONE:     alpha = 0 throughout (Alg. 1 with eigSVD orthonormalisation).
 *   FIXED:    the rule applied once after the first pass, then frozen.
 *   SCHEDULE: after pass j, alpha = max(alpha, c_j * (S_l + alpha)) with
 *             caller multipliers c_j (c = 0.5 reproduces PAPER); dropped for
 *             the rest of the run (c = 0.5) once the PVE ratio grows or
 *             S_{k+1} + alpha shrinks between passes.
 *   LEARNED:  as SCHEDULE, with the multipliers proposed on the device by the
 *             handle's MLP from the first two passes (see dashsvd_mlp_*). */
#define DASHSVD_SHIFT_PAPER 0
#define DASHSVD_SHIFT_NONE 1
#define DASHSVD_SHIFT_FIXED 2
#define DASHSVD_SHIFT_SCHEDULE 3
#define DASHSVD_SHIFT_LEARNED 4

/* Readings of the PVE check (Alg. 5 step 5 with eq. (19)), and the check
 * without the surrogate.
 *   R2 (default): E_i = S_i + alpha with the alpha that produced S_i, for
 *       both the current and the previous pass.
 *   R1: the literal step order, where the stored previous shift is the one
 *       after its update.
 *   NOSURR: the accuracy control that Sec. 4.3 (Table 3) compares the
 *       surrogate against: after every pass, the singular values of
 *       B = A Q (Alg. 3 on B) and eq. (18) on their squares, E' = 0 before
 *       the first pass.  The shift rule is unchanged.  Costs a Gram of an
 *       m x l block and an l x l eigensolve per pass; FP32 and FP64 panels
 *       only (BF16 panels: DASHSVD_ERR_INVALID_ARG), single solves only. */
#define DASHSVD_PVE_R2 0
#define DASHSVD_PVE_R1 1
#define DASHSVD_PVE_NOSURR 2

/* The eigensolver of eigSVD (Alg. 3 steps 1-4) for the sketch, pass and
 * final blocks.
 *   AUTO (default): TRIDIAG in the FP32 and BF16 forms, CHOLQR in the FP64
 *       form.
 *   JACOBI: two-sided Jacobi on G for every block.
 *   ONESIDED: for l <= 128, one-sided Jacobi on the Cholesky factor of G
 *       (rotations J orthogonalise the columns of R^T; R^T J = V diag(S)
 *       gives the eigenvectors V and S = sqrt(eig G) together) for every
 *       block; where the factorisation meets a non-positive pivot (G
 *       singular to working precision) the call goes to the two-sided
 *       solver, as do all calls above 128.
 *   TRIDIAG: in the FP32 and BF16 forms, every block by the tridiagonal
 *       eigensolver (Householder reduction, multisection eigenvalues,
 *       twisted-factorisation eigenvectors, back-transformation: normwise
 *       accurate like the paper's LAPACK eig); where eigenvalues lie within
 *       2^-30 ||G|| of each other the call goes to the two-sided solver, as
 *       do calls without eigenvector output and the FP64 form (whose Jacobi
 *       keeps relative accuracy).
 *   CHOLQR: the sketch and the early pass blocks by Cholesky-QR: W = R^-1
 *       from G = C^T C = R^T R, so that Q = C W is orthonormal with the span
 *       of eigSVD's Q, and S from the eigenvalues of G (Householder
 *       tridiagonalisation and Sturm-count bisection, FP64).  The passes use
 *       only S and span(Q), which both bases share.  Two-sided Jacobi from
 *       the first pass whose PVE ratio is within 100 tol, for the last two
 *       pass blocks, where G is not safely positive definite (lambda_min <=
 *       2^-32 lambda_max, or a failed factorisation) and for the final step. */
#define DASHSVD_EIG_AUTO 0
#define DASHSVD_EIG_JACOBI 1
#define DASHSVD_EIG_ONESIDED 2
#define DASHSVD_EIG_TRIDIAG 3
#define DASHSVD_EIG_CHOLQR 4

#define DASHSVD_MAX_L 160     /* largest supported l = k + oversampling */
#define DASHSVD_MAX_TRACE 256 /* passes recorded in dashsvd_info */

/* A sparse matrix in CSR form.  Owned by the caller; must stay valid until
 * dashsvd_run returns.  row_ptr has m+1 int64 entries with row_ptr[0] = 0
 * and row_ptr[m] = nnz; col_idx has nnz int32 entries, strictly increasing
 * within each row and in [0, n); values has nnz entries of value_dtype
 * (DASHSVD_F32 or DASHSVD_F64).  on_device = 1 means the three pointers are
 * device memory of the current GPU, 0 means host memory (copied in). */
typedef struct {
  int64_t m, n, nnz;
  const int64_t *row_ptr;
  const int32_t *col_idx;
  const void *values;
  int32_t value_dtype;
  int32_t on_device;
} dashsvd_csr;

typedef struct {
  int32_t precision;      /* DASHSVD_PREC_* (default FP32) */
  int32_t shift_policy;   /* DASHSVD_SHIFT_* (default PAPER) */
  int32_t pve_mode;       /* DASHSVD_PVE_* (default R2) */
  int32_t p_max;          /* pass cap; < 0 selects 64 */
  uint64_t seed;          /* key of the Philox4x64-10 stream for Omega */
  void *hip_stream;       /* hipStream_t, NULL = null stream */
  int32_t long_row;       /* SpMM rows longer than this are split into chunks of this many
                             nonzeros; <= 0 selects the tuning database's value for the
                             shape, else 1024 (768 with BF16 panels) from
                             DASHSVD_REORDER_MIN_NNZ nonzeros and 128 below */
  int32_t check_interval; /* passes launched between host reads of the done flag; <= 0: 1 */
  const double *schedule; /* SHIFT_SCHEDULE multipliers, host, p_max + 1 entries (index = pass) */
  const void *omega;      /* optional caller-provided Omega (rows = max(m,n), l columns,
                             row-major, leading dimension l); NULL = draw from seed */
  int32_t omega_dtype;    /* DASHSVD_F32 / DASHSVD_F64 */
  int32_t omega_on_device;
  int32_t timing;         /* DASHSVD_TIMING_ALL (1): time each kernel group with HIP events
                             on its stream (results in dashsvd_info.kt_ms / kt_count);
                             DASHSVD_TIMING_SPMM (2): only the two SpMM groups, so that
                             the events barely slow the run; 0: none */
  const char *tuning_db;  /* optional path of a tuning database written by dashsvd_autotune;
                             runs with long_row <= 0 take the SpMM chunk length stored for
                             their shape bucket (else the built-in default).  Read when the
                             options are set. */
  int32_t eig_method;     /* DASHSVD_EIG_* (default AUTO): how the sketch and the power passes
                             orthonormalise their block */
  int32_t reorder;        /* DASHSVD_REORDER_*: solve P_r A P_c^T with rows and columns
                             by non-increasing nonzero count (memory locality of the
                             products); U and V are returned in the caller's order.
                             AUTO (0): the tuning database's choice for the shape,
                             else on from DASHSVD_REORDER_MIN_NNZ nonzeros */
  int32_t slab_kib;       /* > 0: the SpMM cuts the long rows also at column-slab
                             boundaries and runs their chunks slab by slab, each slab
                             covering about this many KiB of gathered panel rows (one
                             slab at a time in every XCD's L2); <= 0 (default): the
                             tuning database's value for the shape, else no slabs
                             (chunks in row order) */
  int64_t batch_nnz_max;  /* batched form: the members are run in consecutive groups
                             (sub-batches) of at most this many nonzeros in total
                             (and 2^31 - 1 rows, columns and nonzeros, the limit of the
                             stacked operator's 32-bit indices); <= 0 (default):
                             2^31 - 1.  A member larger than the limit is an error. */
  int32_t lane_vectors;   /* SpMM: 16-byte panel vectors per lane, 1 (a row over ld / V
                             lanes) or 2 (half as many lanes, twice the gathers in
                             flight per lane; used where the row splits evenly); <= 0
                             (default): the tuning database's value, else 1 */
  int32_t dense_head;     /* DASHSVD_HEAD_*: with the degree order, the leading rows of M and
                             of M^T that hold at least max(long_row + 1, columns / 16)
                             nonzeros each (at most 128; none if fewer than 16) are
                             multiplied as a dense block on the matrix cores instead of
                             by the row-split SpMM.  AUTO (0, default): on where the degree
                             order is on (l rounded up to 8 at most 160); OFF (-1) */
} dashsvd_options;

#define DASHSVD_HEAD_AUTO 0
#define DASHSVD_HEAD_OFF (-1)

#define DASHSVD_REORDER_AUTO 0
#define DASHSVD_REORDER_ON 1
#define DASHSVD_REORDER_OFF (-1)
#define DASHSVD_REORDER_MIN_NNZ (1 << 22)

#define DASHSVD_TIMING_ALL 1
#define DASHSVD_TIMING_SPMM 2

/* Kernel groups timed when options.timing is set (index into kt_ms / kt_count). */
#define DASHSVD_KT_SPMM 0        /* M times a panel: Z = M C (FP32/FP64 forms) or Y = M Q (BF16 form) */
#define DASHSVD_KT_SPMM_T 1      /* M^T times a panel: X = M^T Z, or C = M^T Y - alpha Q (BF16 form) */
#define DASHSVD_KT_GRAM 2        /* Gram partials + reduction (every eigSVD) */
#define DASHSVD_KT_EIG 3         /* Jacobi eigSVD + tail */
#define DASHSVD_KT_RESCALE 4     /* C+ = (X - alpha C) W, or Q = C W (BF16 form) */
#define DASHSVD_KT_TRANSPOSE 5   /* validation + CSR(A^T) build */
#define DASHSVD_KT_SKETCH 6      /* Omega + M^T Omega */
#define DASHSVD_KT_FINAL 7       /* B = M Q, its eigSVD, U, V, signs */
#define DASHSVD_KT_CHOLQR 8      /* Cholesky-QR + eigenvalue blocks (eig_method AUTO) */
#define DASHSVD_KT_CHECK 9       /* pve_mode NOSURR: Gram of B, its eigenvalues, eq. (18) */
#define DASHSVD_KT_GROUPS 10

typedef struct {
  int32_t passes;          /* N_p: shifted power passes executed */
  int32_t converged;       /* 1 if the PVE check stopped the loop */
  int32_t rank_deficient;  /* 1 if some eigSVD zeroed a column */
  int32_t status;          /* status of the last run */
  int32_t l;               /* k + oversampling */
  int32_t learned_fallback;/* 1 if a schedule/learned run fell back to the paper rule */
  double final_alpha;      /* shift after the last pass */
  double alpha_used[DASHSVD_MAX_TRACE]; /* shift used in pass j (index j-1) */
  double ratio[DASHSVD_MAX_TRACE];      /* PVE ratio of pass j */
  double time_total_ms;    /* host wall time of dashsvd_run */
  double time_setup_ms;    /* validation, CSR(A^T), SpMM plans, Omega */
  double time_loop_ms;     /* sketch + power passes */
  double time_final_ms;    /* final Rayleigh-Ritz and sign normalisation */
  int64_t long_chunks_A;   /* SpMM chunk tasks of the row-split plan, A side */
  int64_t long_chunks_AT;  /* same for A^T */
  double kt_ms[DASHSVD_KT_GROUPS];     /* summed HIP-event time per kernel group (timing = 1) */
  int32_t kt_count[DASHSVD_KT_GROUPS]; /* launches counted per group (passes after the stop
                                          excluded) */
  int32_t eig_calls;       /* eigSVD eigenproblems solved in the run */
  int32_t eig_sweeps;      /* Jacobi sweeps summed over them (Cholesky-QR calls count 0) */
  int32_t sweeps_per_call[DASHSVD_MAX_TRACE + 2]; /* sweeps of eigSVD call c: the sketch (c = 0),
                                                     the passes, then the final step */
  int32_t long_row_used;   /* SpMM chunk length of the run (option, tuning database or default) */
  int32_t learned_n;       /* LEARNED policy: pass count predicted after pass 2 (0 if none) */
  int32_t promoted;        /* BF16 panels: 1 if the stagnation guard switched the remaining
                              passes to FP32 panels (the PVE ratio stayed above tol and above
                              0.8 x its previous value for two passes) */
  int32_t cholqr_calls;    /* eig_calls solved by Cholesky-QR (eig_method AUTO) */
  int32_t sub_batches;     /* batched form: groups of members run one after the other (1 when
                              the batch fits the limit of option batch_nnz_max) */
  int32_t graph_launches;  /* batched form: launches of the captured pass graph (each holds
                              check_interval passes; summed over the sub-batches) */
  int32_t lane_vectors_used; /* SpMM lane vectors of the run (option, tuning database or 1) */
  int32_t slab_kib_used;   /* SpMM column-slab KiB of the run (0: none) */
  int32_t reordered;       /* 1 if the run iterated the degree-ordered operator */
  int32_t head_rows;       /* rows of M multiplied as a dense head (option dense_head; 0: none) */
  int32_t head_rows_t;     /* the same for M^T */
} dashsvd_info;

typedef struct dashsvd_handle dashsvd_handle;

/* Create a handle.  opt may be NULL (all defaults).  The options are copied. */
dashsvd_status dashsvd_create(dashsvd_handle **h, const dashsvd_options *opt);
/* Release a handle and its device workspace.  NULL is ignored. */
void dashsvd_destroy(dashsvd_handle *h);

/* Replace the options of an existing handle (workspace kept). */
dashsvd_status dashsvd_set_options(dashsvd_handle *h, const dashsvd_options *opt);

/* Alg. 5 (Alg. 4 when tol == 0): rank k, oversampling p (l = k + p),
 * tolerance tol of the PVE check.  Requires 1 <= k, 1 <= p (the check reads
 * S_{k+1}), k + p <= min(m, n), k + p <= DASHSVD_MAX_L, tol >= 0.  Returns
 * OK, NOT_CONVERGED (tol > 0 and p_max passes ran), RANK_DEFICIENT, or an
 * error.  Results stay in the handle until the next run or destroy. */
dashsvd_status dashsvd_run(dashsvd_handle *h, const dashsvd_csr *A, int32_t k, int32_t p,
                           double tol);

/* Copy the last run's results: U (m x k, row-major, leading dimension ldu),
 * S (k, descending), V (n x k, leading dimension ldv), each in dtype
 * (DASHSVD_F32 or DASHSVD_F64; S always double).  on_device selects device
 * or host destination pointers.  Any pointer may be NULL to skip it.  Signs:
 * the entry of largest magnitude of each V column is positive (lowest row on
 * ties), U columns flipped alike.  Synchronises the stream. */
dashsvd_status dashsvd_get_USV(dashsvd_handle *h, void *U, int64_t ldu, double *S, void *V,
                               int64_t ldv, int32_t dtype, int32_t on_device);

dashsvd_status dashsvd_get_info(dashsvd_handle *h, dashsvd_info *out);

/* Accuracy of the last run (Sec. 4 metrics), computed on the device:
 *   eps_pve   = max_{i<k} |sigma_i^2 - ||A^T u_i||^2| / sigma_{k+1}^2,
 *   eps_sigma = max_{i<k} |sigma_i - S_i| / sigma_i,
 * with u_i the computed left singular vectors, S the computed values and
 * sigma_ref (host, n_ref >= k + 1 doubles, descending, sigma_ref[k] > 0)
 * reference singular values of A.  A must be the matrix of the last run
 * (same sizes; device arrays still valid).  A^T U is formed with the
 * library's SpMM in the run's compute type and its squared column norms in
 * FP64.  Either output pointer may be NULL.  Synchronises the stream; the
 * panels of the last run are overwritten, its results (U, S, V) are not. */
dashsvd_status dashsvd_evaluate(dashsvd_handle *h, const dashsvd_csr *A, const double *sigma_ref,
                                int32_t n_ref, double *eps_pve, double *eps_sigma);

/* All four error metrics of Sec. 4 for the last run, on the device. */
typedef struct {
  double eps_pve;    /* max_{i<k} |sigma_i^2 - ||A^T u_i||^2| / sigma_{k+1}^2 */
  double eps_sigma;  /* max_{i<k} |sigma_i - S_i| / sigma_i */
  double eps_res;    /* max_{i<k} ||A^T u_i - S_i v_i||_2 / sigma_i */
  double eps_spec;   /* (||A - U diag(S) V^T||_2 - sigma_{k+1}) / sigma_{k+1} */
  double spec_norm;  /* the estimate of ||A - U diag(S) V^T||_2 used (a lower bound) */
  int32_t lanczos_steps;  /* Lanczos steps taken for spec_norm */
  int32_t pad;
} dashsvd_metrics;

/* As dashsvd_evaluate, plus eps_res and eps_spec (Sec. 4).  eps_res forms
 * A^T U with the library's SpMM and the column norms of A^T U - V diag(S) in
 * FP64.  ||A - U diag(S) V^T||_2 is the square root of the largest
 * eigenvalue of E^T E (E = A - U S V^T), estimated by the Lanczos process
 * with full reorthogonalisation (two rounds of Gram-Schmidt per step)
 * started from the Gaussian vector of the Philox stream keyed by seed
 * (Omega's generator, one column), with the products by A and A^T in the
 * run's compute type and the vectors in FP64.  The estimate never exceeds
 * the norm and grows with the steps; it stops after max_steps steps (at
 * most n), at an invariant subspace, or when it has changed by at most
 * 1e-14 (FP64 runs; 1e-9 otherwise) relative over 5 steps.  Allocates
 * FP64 buffers of (m + n) k + n max(k, max_steps + 1) doubles for the call
 * and frees them.  Synchronises the stream; errors as dashsvd_evaluate. */
dashsvd_status dashsvd_evaluate_all(dashsvd_handle *h, const dashsvd_csr *A, const double *sigma_ref,
                                    int32_t n_ref, int32_t max_steps, uint64_t seed,
                                    dashsvd_metrics *out);

/* Per-pass S (the l singular values of each pass's block C, descending):
 * writes min(passes, max_passes) rows of l doubles to host memory. */
dashsvd_status dashsvd_get_trace(dashsvd_handle *h, double *s_hat, int32_t max_passes);

/* Batched form: count independent matrices, each solved by Alg. 5 (Alg. 4
 * when tol == 0) with the handle's options, the same k and oversampling p,
 * and its own shift, PVE check, stopping pass and traces.  Matrix i draws
 * Omega from the Philox stream keyed (seed + i, 0).  Requirements: every
 * matrix as for dashsvd_run, plus m >= n, k + p <= 64, the same value dtype
 * and memory space for all, and stacked sizes (sum of rows, columns and
 * nonzeros) below 2^31.  The matrices advance pass-synchronously: each step
 * of a pass is one launch over the whole batch, and one pass is captured as
 * a HIP graph and replayed.  Policies PAPER, NONE, FIXED and SCHEDULE.
 * Returns OK, NOT_CONVERGED (some matrix reached p_max with tol > 0),
 * RANK_DEFICIENT or an error.  Results stay in the handle until the next
 * run of either form.  The arrays of all matrices must stay valid until
 * the call returns (it synchronises). */
dashsvd_status dashsvd_run_batched(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k,
                                   int32_t p, double tol);
/* Results of matrix idx of the last batched run, as dashsvd_get_USV. */
dashsvd_status dashsvd_get_USV_batched(dashsvd_handle *h, int32_t idx, void *U, int64_t ldu, double *S,
                                       void *V, int64_t ldv, int32_t dtype, int32_t on_device);
/* Per-matrix info of the last batched run (passes, convergence, alpha and
 * ratio traces, sweeps); idx < 0 gives the batch summary (maximum passes,
 * all converged, total eig calls and sweeps, wall time). */
dashsvd_status dashsvd_get_info_batched(dashsvd_handle *h, int32_t idx, dashsvd_info *out);

/* Autotuner of the SpMM work split and layout: times short runs (2 passes,
 * tol 0, 3 repetitions, the fastest kept) of the given matrix (count == 1,
 * dashsvd_run) or batch (count > 1, dashsvd_run_batched), by the SpMM kernel
 * time (single matrix) or the pass-loop time (batch), over four knobs in
 * turn, each at the best values found so far for the others (a coordinate
 * search): the long-row chunk length (32 ... 1024 nonzeros: from row
 * splitting towards an even split of the nonzeros), the lane vectors per
 * row (1 or 2), the column slabs (none or 2 MiB) and, for a single matrix,
 * the degree order (on or off; its setup is not in the timed SpMM time, so
 * this knob compares the products only).  Knobs that the handle's options
 * fix (long_row, lane_vectors, slab_kib > 0, reorder ON / OFF) keep the
 * option's value.  Appends "key chunk_length lanes slab_kib reorder" to the
 * text file db_path (if not NULL) and to the handle's table, and returns the
 * chunk length in *best.  The key is the shape bucket: precision, l rounded
 * up to 8, log2 of the rows and of the mean nonzeros per row of the
 * operator, and the form (single / batched).  Runs whose options leave a
 * knob at its default take its value from the table.  The handle's other
 * options are left unchanged; the results of the tuning runs are
 * discarded. */
dashsvd_status dashsvd_autotune(dashsvd_handle *h, const dashsvd_csr *As, int32_t count, int32_t k,
                                int32_t p, const char *db_path, int32_t *best);

/* ---------------------------------------------------------------------
 * Learned shift (policy DASHSVD_SHIFT_LEARNED).  The paper's rule sets the
 * shift of Alg. 5 step 6 from S_l; this policy lets an MLP propose the
 * multiplier c in alpha_j = c E_l(j-1) for passes 3, 4, ... (E = S + the
 * shift that produced S) from the E of passes 1 and 2, with the PVE check of
 * step 5 still deciding termination and a guard that returns to c = 1/2 once
 * E_{k+1} decreases or the PVE ratio increases.
 *   features (3 l + 3): E_i(1)/E_1(1), E_i(2)/E_1(2), E_i(2)/E_i(1) for
 *     i < l, then log m, log n, log(nnz/m) of the operator (m >= n);
 *   network: relu(W1 x + b1) -> relu(W2 . + b2) -> W3 . + b3, hidden width
 *     128, FP32; outputs o: c = 1/2 + (c_max - 1/2) sigmoid(o_0), log N = o_1;
 *   loss: mean of (c - c*)^2 + 0.1 (o_1 - log N*)^2.
 * Inference runs inside the eigensolver of pass 2.  All buffers of these
 * calls are host memory; the parameters stay on the device in the handle.
 * ------------------------------------------------------------------- */
/* New MLP for blocks of l = k + oversampling columns; weights He-uniform from
 * seed, Adam state cleared.  c_max in (0.5, 1). */
dashsvd_status dashsvd_mlp_init(dashsvd_handle *h, int32_t l, uint64_t seed, double c_max);
dashsvd_status dashsvd_mlp_num_params(dashsvd_handle *h, int64_t *n);
/* Parameters as one FP32 vector: W1 (128 x D), b1, W2 (128 x 128), b2,
 * W3 (2 x 128), b3, row-major; set also clears the Adam state. */
dashsvd_status dashsvd_mlp_set_params(dashsvd_handle *h, const float *params, int64_t n);
dashsvd_status dashsvd_mlp_get_params(dashsvd_handle *h, float *params, int64_t n);
/* out (batch x 2) = (c, log N) for features X (batch x D). */
dashsvd_status dashsvd_mlp_forward(dashsvd_handle *h, const float *X, int32_t batch, float *out);
/* Gradient of the loss (same layout as the parameters) and the loss, for
 * targets Y (batch x 2: c*, log N*). */
dashsvd_status dashsvd_mlp_grad(dashsvd_handle *h, const float *X, const float *Y, int32_t batch,
                                float *grad, float *loss);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) of learning rate lr on a batch. */
dashsvd_status dashsvd_mlp_train_step(dashsvd_handle *h, const float *X, const float *Y,
                                      int32_t batch, float lr, float *loss);
/* Features of the last dashsvd_run (it must have run two passes), exactly as
 * the LEARNED policy forms them; n = 3 l + 3. */
dashsvd_status dashsvd_learned_features(dashsvd_handle *h, float *feat, int32_t n);

/* Device bytes a run with these arguments needs (workspace of the handle),
 * under the default options with the given precision.  Host only: no HIP
 * call is made. */
dashsvd_status dashsvd_workspace_size(const dashsvd_csr *A, int32_t k, int32_t p,
                                      int32_t precision, size_t *bytes);
/* The same for dashsvd_run_batched over the count matrices As. */
dashsvd_status dashsvd_workspace_size_batched(const dashsvd_csr *As, int32_t count, int32_t k,
                                              int32_t p, int32_t precision, size_t *bytes);
/* The same under the options of handle h (its precision, degree order,
 * caller Omega, schedule, tuning database ...): batched = 0 sizes
 * dashsvd_run on As[0], batched = 1 sizes dashsvd_run_batched on the count
 * matrices.  Host only. */
dashsvd_status dashsvd_handle_workspace_size(const dashsvd_handle *h, const dashsvd_csr *As,
                                             int32_t count, int32_t batched, int32_t k, int32_t p,
                                             size_t *bytes);

/* Caller-owned workspace (for instance a torch allocation), used in place of
 * the arena the handle would allocate itself: every device buffer of
 * dashsvd_run, dashsvd_run_batched and dashsvd_evaluate is carved out of
 * [dev_ptr, dev_ptr + bytes).  dev_ptr must be device memory of the current
 * GPU, 256-byte aligned; it stays owned by the caller, who must keep it
 * valid, and not use it, until the handle is destroyed or given another
 * workspace.  A run that needs more than bytes (dashsvd_handle_workspace_size)
 * fails with DASHSVD_ERR_OOM and allocates nothing.  dev_ptr = NULL returns
 * the handle to its own arena, allocated on the next run.  The call waits
 * for the handle's queued work and discards the results of earlier runs,
 * which lived in the old workspace. */
dashsvd_status dashsvd_set_workspace(dashsvd_handle *h, void *dev_ptr, size_t bytes);

const char *dashsvd_status_string(dashsvd_status s);
/* Detail of the last error on this handle (or of the last failed create when
 * h is NULL).  Valid until the next call on the handle. */
const char *dashsvd_last_error(const dashsvd_handle *h);

/* ---------------------------------------------------------------------
 * Kernel-level entry points.  They run one step of the path on device
 * buffers the caller owns, on the given stream, and return after the work
 * is queued (no synchronisation).  They exist so each step can be checked
 * alone; the solver calls the same kernels.
 * ------------------------------------------------------------------- */

/* Alg. 5 step 1 (randn): out[i*ld + j] for i < rows, j < cols, element
 * e = i*cols + j from Philox4x64-10 keyed (seed, 0), counter (b+1, 0, 0, 0)
 * for block b, raw words 2t, 2t+1 -> Box-Muller pair t = e/2.  dtype F32,
 * F64 or BF16 (rounded to nearest even from FP64). */
dashsvd_status dashsvd_k_gaussian(uint64_t seed, int64_t rows, int64_t cols, void *out,
                                  int64_t ld, int32_t dtype, void *stream);

/* Raw Philox words: out[w] = word w of the stream keyed (seed, 0). */
dashsvd_status dashsvd_k_philox_raw(uint64_t seed, int64_t nwords, uint64_t *out, void *stream);

/* The library's stable LSD radix sort (used for CSR(A^T) and the degree
 * order): keys_out = keys_in sorted on their low `bits` bits (1..32),
 * ascending, or descending when descending != 0 (non-increasing keys); equal
 * keys keep their input order, and idx_out[p] is the input position of
 * keys_out[p].  All pointers device memory, n entries each.  Synchronises
 * the stream. */
dashsvd_status dashsvd_k_sort_index(int64_t n, const uint32_t *keys_in, uint32_t *keys_out, int32_t *idx_out,
                                    int32_t bits, int32_t descending, void *stream);

/* CSR of A^T (the transposed operand of Alg. 5 steps 2 and 4): rows of A^T
 * list their columns in increasing order.  All pointers are device memory;
 * rowT has n+1 entries, colT/valT nnz.  values dtype as given (F32/F64).
 * Validates A first (status BAD_CSR / NONFINITE).  Synchronises the stream. */
dashsvd_status dashsvd_k_transpose(int64_t m, int64_t n, int64_t nnz, const int64_t *row_ptr,
                                   const int32_t *col, const void *val, int32_t dtype,
                                   int64_t *rowT, int32_t *colT, void *valT, void *stream);

/* Y = A X or, with alpha != NULL, Y = A X - (*alpha) Q (the shifted block of
 * Alg. 5 step 4), with the library's row-split + long-row-chunk SpMM.
 * A: CSR rows x cols on device, values F32 (panel types F32/BF16) or F64
 * (F64 panels).  X: cols x ldx, Y: rows x ldy, Q: rows x ldq; the first l
 * columns are used.  xdtype / ydtype: element types of X/Q and Y.  cols <= 0
 * means the rows of X are not given: the gathers then use plain loads
 * instead of range-checked buffer loads (the path panels of 2 GB and more
 * take; same results).  long_row <= 0 selects the default.  Synchronises
 * the stream (plan sizing). */
dashsvd_status dashsvd_k_spmm(int64_t rows, int64_t cols, int64_t nnz, const int64_t *row_ptr,
                              const int32_t *col, const void *val, const void *X, int64_t ldx,
                              int32_t xdtype, void *Y, int64_t ldy, int32_t ydtype, int32_t l,
                              const void *Q, int64_t ldq, const double *alpha, int32_t long_row,
                              void *stream);

/* dashsvd_k_spmm without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture that builds around it, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, kernels
 * and results (bit for bit) as dashsvd_k_spmm; the row-split plan and the
 * partial rows of long-row chunks live in a static device array of 32 MiB
 * (33554432 bytes) that each device holds until the process ends.  The plan
 * takes about 16 bytes per row plus, for each of the 2 * nnz / long_row + 1
 * chunks it may hold, 16 + ld * 4 bytes (ld * 8 with F64 panels; ld = l
 * rounded up to 8) and 24 bytes per nnz / long_row + 1 long rows.  A call
 * whose plan needs more than the array fails with DASHSVD_ERR_INVALID_ARG and
 * a message giving the size, before any work is queued; a larger long_row
 * needs less.  All calls on one device share the array, which keeps the last
 * call's contents: calls that overlap on one device (several host threads or
 * streams) race and give wrong results.  Each call synchronises the stream
 * before returning, so calls made one after another from one thread are
 * safe. */
dashsvd_status dashsvd_k_spmm_static(int64_t rows, int64_t cols, int64_t nnz, const int64_t *row_ptr,
                                     const int32_t *col, const void *val, const void *X, int64_t ldx,
                                     int32_t xdtype, void *Y, int64_t ldy, int32_t ydtype, int32_t l,
                                     const void *Q, int64_t ldq, const double *alpha, int32_t long_row,
                                     void *stream);

/* G (l x l, FP64, row-major, full symmetric) = C^T C for C r x l (ldc),
 * C dtype F32 or F64; FP64 accumulation (Alg. 3 step 1). */
dashsvd_status dashsvd_k_gram(int64_t r, int32_t l, const void *C, int64_t ldc, int32_t cdtype,
                              double *G, void *stream);

/* Symmetric eigendecomposition of G (l x l FP64, device) by the library's
 * Jacobi kernel: S (l, descending sqrt of the clamped eigenvalues), Vs
 * (l x l, column i = eigenvector of S_i), W = Vs diag(1/S) with zeroed
 * columns where S <= S_max*sqrt(l*eps) (Alg. 3 steps 1-4).  sweeps
 * (optional, device int) receives the sweep count. */
dashsvd_status dashsvd_k_eig(int32_t l, const double *G, double *S, double *Vs, double *W,
                             int32_t *sweeps, void *stream);
/* dashsvd_k_eig with a step profile: prof (device, 6 int64) accumulates, as
 * seen by thread 0, the cycles of the rotation phase and of the update
 * phase, the 100 MHz wall-clock ticks, the number of Jacobi steps, and the
 * cycles of thread 0's own rotation work and V update. */
dashsvd_status dashsvd_k_eig_prof(int32_t l, const double *G, double *S, double *Vs, double *W,
                                  int32_t *sweeps, long long *prof, void *stream);

/* The eigensolver of dashsvd_k_eig by one-sided Jacobi (eig_method ONESIDED,
 * Alg. 3 steps 1-4): the Cholesky factorisation G = R^T R, then Hestenes
 * rotations orthogonalise the columns of R^T; R^T J = Vs diag(S).  Same
 * outputs and ordering as dashsvd_k_eig; skip is the relative rotation
 * threshold (2^-53 in the FP64 form, 2^-23 in the FP32 and BF16 forms;
 * raised to l 2^-53, the rounding level of the dot products).  l <= 128.
 * *accepted (host) is 0 when G is not positive definite to working
 * precision (a non-positive or non-finite Cholesky pivot); then nothing
 * is written.  *sweeps (device, optional): sweeps that rotated (a last one
 * without rotations confirms convergence).  prof (device, optional, 6
 * int64) accumulates, as seen by thread 0, the cycles of the dot products
 * with their reduction, of the rotation parameters, of the column updates,
 * of the column exchange with its barrier, the number of steps and the
 * cycles of the Cholesky phase.  Synchronises the stream. */
dashsvd_status dashsvd_k_eig_onesided(int32_t l, const double *G, double *S, double *Vs, double *W, double skip,
                                      int32_t *sweeps, int32_t *accepted, long long *prof, void *stream);

/* The eigensolver of dashsvd_k_eig by tridiagonalisation (eig_method
 * TRIDIAG, Alg. 3 steps 1-4): Householder reduction G = H T H^T in one
 * workgroup, then one wave per eigenvalue: multisection on Sturm counts,
 * the eigenvector of T from its twisted factorisation, V = H z.  Same
 * outputs and ordering as dashsvd_k_eig; Vs is required (W holds the
 * reflectors before the result).  l <= 160.  *accepted (host) is 0 when two
 * eigenvalues lie within 2^-30 ||G|| of each other, or G is zero or has a
 * non-finite entry; then S, Vs and W hold no result.  prof (device,
 * optional, 8 int64): cycles of the reduction, then, as seen by the first
 * wave of the eigenvalue kernel, of the multisection, the isolation check,
 * the factorisations with the twist and z, the back-transformation, the
 * cycles of the last workgroup's W and tail, and, summed over the steps of
 * the reduction as seen by its first thread, the cycles to the end of the
 * reflector's publication and of the product A22 v.  Allocates a small
 * workspace; synchronises the stream. */
dashsvd_status dashsvd_k_eig_tridiag(int32_t l, const double *G, double *S, double *Vs, double *W,
                                     int32_t *accepted, long long *prof, void *stream);

/* Orthonormalisation of a pass block without eigenvectors (the solver of
 * the sketch and power passes under eig_method AUTO): from G (device, l x l
 * symmetric, FP64, row-major) the Cholesky-QR weights W = R^-1 (device,
 * l x l, upper triangular, zeros below the diagonal; G = R^T R) and S
 * (device, l, descending) = sqrt of the eigenvalues of G, from Householder
 * tridiagonalisation and Sturm-count bisection.  *accepted (host) is 1 when
 * the factorisation completed and lambda_min > 2^-32 lambda_max; when 0,
 * W and S are unspecified (the solver then runs the Jacobi eigSVD).
 * Synchronises the stream. */
dashsvd_status dashsvd_k_cholqr(int32_t l, const double *G, double *S, double *W, int32_t *accepted,
                                void *stream);

/* Out (r x c, ldo, odtype) = C (r x l, ldc, cdtype) * W (l x c, FP64,
 * row-major, leading dimension ldw): the rescale U = C V S^-1 of Alg. 3
 * step 3 and the final products of Alg. 5.  Columns c..ldo-1 of Out are
 * written as zero. */
dashsvd_status dashsvd_k_rescale(int64_t r, int32_t l, const void *C, int64_t ldc, int32_t cdtype,
                                 const double *W, int64_t ldw, int32_t c, void *Out, int64_t ldo,
                                 int32_t odtype, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DASHSVD_H */
