/*
 * dashSVD oracle: a plain, slow, FP64 CPU implementation of what the GPU hot
 * path computes.  TEST INFRASTRUCTURE ONLY: it is called by the tests, by the
 * smoke check and by the CPU-baseline leg of the benchmark, never by the
 * product library.  It shares no code, header or constant table with the HIP
 * sources.
 *
 * Source: Feng, Yu, Xie, Tang, "Faster Randomized SVD with Dynamic Shifts"
 * (dashSVD).  Each function names the passage it follows:
 *   - Alg. 3 (eigSVD): eig of C^T C, S = sqrt(D), U = C V S^{-1}, flip to
 *     descending order.
 *   - Alg. 4 / Alg. 5 (dashSVD for m >= n): sketch A^T Omega, shifted power
 *     passes eigSVD(A^T (A Q) - alpha Q), the dynamic shift rule and the PVE
 *     surrogate check of eq. (19) with the surrogate of Prop. 3, then the
 *     final eigSVD of B = A Q.
 *   - Sec. 3.1 (orientation): a matrix with m < n is handled through A^T.
 *
 * Readings where the paper is silent or ambiguous (listed again in the design
 * notes of the repository):
 *   - randn: Philox4x64-10 (Salmon et al., SC'11) keyed by (seed, 0), counter
 *     (b+1, 0, 0, 0) for block b, words taken in order; Box-Muller on word
 *     pairs (see orc_gaussian).
 *   - PVE check: reading R2 (default) pairs each singular value estimate with
 *     the shift that produced it; reading R1 is the literal step order, in
 *     which the previous shift is stored after its update.
 *   - eigSVD on a rank-deficient block: eigenvalues are clamped at 0 and
 *     columns with S <= S_max * sqrt(l * eps) are set to zero and reported.
 *
 * All arithmetic is FP64.  OpenMP parallelises only loops whose iterations
 * are independent, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11).  Round: two 64x64->128 multiplies of counter
 * words 0 and 2 by the round multipliers, outputs permuted and xored with
 * the other counter words and the key; the key is bumped by the Weyl
 * constants between rounds. */
static const uint64_t ORC_PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t ORC_PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t ORC_PHILOX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t ORC_PHILOX_W1 = 0xBB67AE8584CAA73BULL;

static void orc_mulhilo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                       uint64_t out[4]) {
  uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += ORC_PHILOX_W0;
      k1 += ORC_PHILOX_W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    orc_mulhilo(ORC_PHILOX_M0, x0, &hi0, &lo0);
    orc_mulhilo(ORC_PHILOX_M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Raw word w of the stream keyed by `seed`: block b = w / 4 uses counter
 * (b + 1, 0, 0, 0); word w is output word w % 4 of that block. */
static uint64_t orc_philox_word(uint64_t seed, uint64_t w) {
  uint64_t ctr[4] = {w / 4 + 1, 0, 0, 0};
  uint64_t key[2] = {seed, 0};
  uint64_t out[4];
  orc_philox4x64_10(ctr, key, out);
  return out[w % 4];
}

void orc_philox_raw(uint64_t seed, int64_t nwords, uint64_t *out) {
  for (int64_t w = 0; w < nwords; ++w) out[w] = orc_philox_word(seed, (uint64_t)w);
}

/* Omega = randn(rows, cols), row-major; element e = i*cols + j.  Pair t = e/2
 * takes raw words (2t, 2t+1):
 *   u1 = ((w0 >> 11) + 1) * 2^-53  in (0, 1]
 *   u2 =  (w1 >> 11)      * 2^-53  in [0, 1)
 *   element 2t   = sqrt(-2 ln u1) * cos(2 pi u2)
 *   element 2t+1 = sqrt(-2 ln u1) * sin(2 pi u2)          (Box-Muller) */
void orc_gaussian(uint64_t seed, int64_t rows, int64_t cols, double *out) {
  const int64_t total = rows * cols;
  const int64_t npairs = (total + 1) / 2;
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < npairs; ++t) {
    uint64_t w0 = orc_philox_word(seed, 2 * (uint64_t)t);
    uint64_t w1 = orc_philox_word(seed, 2 * (uint64_t)t + 1);
    double u1 = (double)((w0 >> 11) + 1) * 0x1.0p-53;
    double u2 = (double)(w1 >> 11) * 0x1.0p-53;
    double r = sqrt(-2.0 * log(u1));
    out[2 * t] = r * cos(two_pi * u2);
    if (2 * t + 1 < total) out[2 * t + 1] = r * sin(two_pi * u2);
  }
}

/* ------------------------------------------------------------------ */
/* Sparse products on a CSR matrix (row_ptr m+1, col nnz, val nnz). */

/* Y (m x l) = A X, X n x l, all row-major with leading dimension l.
 * Row r: Y[r,:] = sum over the stored entries of row r, in storage order. */
void orc_csr_spmm(int64_t m, const int64_t *row_ptr, const int32_t *col,
                  const double *val, const double *X, int64_t l, double *Y) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t r = 0; r < m; ++r) {
    double *y = Y + r * l;
    for (int64_t j = 0; j < l; ++j) y[j] = 0.0;
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      const double a = val[e];
      const double *x = X + (int64_t)col[e] * l;
      for (int64_t j = 0; j < l; ++j) y[j] += a * x[j];
    }
  }
}

/* CSR of A^T by counting sort on the column index: count the entries of each
 * column, prefix-sum the counts, then walk A row by row and append each entry
 * to its column, so each column of A^T lists its rows in increasing order. */
void orc_csr_transpose(int64_t m, int64_t n, const int64_t *row_ptr,
                       const int32_t *col, const double *val, int64_t *rowT,
                       int32_t *colT, double *valT) {
  for (int64_t c = 0; c <= n; ++c) rowT[c] = 0;
  const int64_t nnz = row_ptr[m];
  for (int64_t e = 0; e < nnz; ++e) rowT[col[e] + 1] += 1;
  for (int64_t c = 0; c < n; ++c) rowT[c + 1] += rowT[c];
  int64_t *cursor = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t c = 0; c < n; ++c) cursor[c] = rowT[c];
  for (int64_t r = 0; r < m; ++r) {
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      int64_t pos = cursor[col[e]]++;
      colT[pos] = (int32_t)r;
      valT[pos] = val[e];
    }
  }
  free(cursor);
}

/* ------------------------------------------------------------------ */
/* Dense helpers. */

/* G (l x l) = C^T C for C r x l row-major: upper triangle by definition,
 * lower triangle mirrored. */
void orc_gram(int64_t r, int64_t l, const double *C, double *G) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < l; ++i) {
    for (int64_t j = i; j < l; ++j) {
      double s = 0.0;
      for (int64_t t = 0; t < r; ++t) s += C[t * l + i] * C[t * l + j];
      G[i * l + j] = s;
    }
  }
  for (int64_t i = 0; i < l; ++i)
    for (int64_t j = 0; j < i; ++j) G[i * l + j] = G[j * l + i];
}

/* Out (r x c) = X (r x t) * W (t x c), row-major with given column counts. */
static void orc_matmul(int64_t r, int64_t t, int64_t c, const double *X,
                       int64_t ldx, const double *W, int64_t ldw, double *Out,
                       int64_t ldo) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < r; ++i) {
    for (int64_t j = 0; j < c; ++j) {
      double s = 0.0;
      for (int64_t q = 0; q < t; ++q) s += X[i * ldx + q] * W[q * ldw + j];
      Out[i * ldo + j] = s;
    }
  }
}

/* Symmetric eigenproblem by cyclic-by-row Jacobi (Golub & Van Loan, Matrix
 * Computations, Sec. 8.5: the 2x2 symmetric Schur decomposition and the
 * cyclic sweep).  On return G is overwritten, evals holds the eigenvalues in
 * ascending order (stable in the original index on ties) and V (l x l,
 * row-major) holds the matching eigenvectors as columns.  A rotation is
 * skipped when |g_pq| is below half an ulp of sqrt(|g_pp g_qq|); the sweeps
 * stop when a sweep skips every rotation.  Returns the number of sweeps. */
int orc_jacobi_eig(int64_t l, double *G, double *evals, double *V) {
  for (int64_t i = 0; i < l * l; ++i) V[i] = 0.0;
  for (int64_t i = 0; i < l; ++i) V[i * l + i] = 1.0;
  int sweeps = 0;
  for (; sweeps < 100; ++sweeps) {
    int64_t rotated = 0;
    for (int64_t p = 0; p < l - 1; ++p) {
      for (int64_t q = p + 1; q < l; ++q) {
        const double apq = G[p * l + q];
        const double app = G[p * l + p];
        const double aqq = G[q * l + q];
        if (apq == 0.0) continue;
        if (fabs(apq) <= 1.1102230246251565e-16 * sqrt(fabs(app * aqq))) continue;
        /* symSchur2: tau = (a_qq - a_pp) / (2 a_pq); t = sign(tau) /
         * (|tau| + sqrt(1 + tau^2)); c = 1/sqrt(1+t^2); s = t c. */
        const double tau = (aqq - app) / (2.0 * apq);
        double t;
        if (tau >= 0.0)
          t = 1.0 / (tau + sqrt(1.0 + tau * tau));
        else
          t = -1.0 / (-tau + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = t * c;
        ++rotated;
        /* G <- J^T G J with J = identity except J_pp = J_qq = c,
         * J_pq = s, J_qp = -s. Columns first, then rows. */
        for (int64_t k = 0; k < l; ++k) {
          const double gkp = G[k * l + p], gkq = G[k * l + q];
          G[k * l + p] = c * gkp - s * gkq;
          G[k * l + q] = s * gkp + c * gkq;
        }
        for (int64_t k = 0; k < l; ++k) {
          const double gpk = G[p * l + k], gqk = G[q * l + k];
          G[p * l + k] = c * gpk - s * gqk;
          G[q * l + k] = s * gpk + c * gqk;
        }
        for (int64_t k = 0; k < l; ++k) {
          const double vkp = V[k * l + p], vkq = V[k * l + q];
          V[k * l + p] = c * vkp - s * vkq;
          V[k * l + q] = s * vkp + c * vkq;
        }
      }
    }
    if (rotated == 0) break;
  }
  /* Sort ascending, stable in the index (insertion sort on an index list). */
  int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)l);
  double *d = (double *)malloc(sizeof(double) * (size_t)l);
  double *Vs = (double *)malloc(sizeof(double) * (size_t)(l * l));
  for (int64_t i = 0; i < l; ++i) {
    idx[i] = i;
    d[i] = G[i * l + i];
  }
  for (int64_t i = 1; i < l; ++i) {
    int64_t key = idx[i];
    int64_t j = i - 1;
    while (j >= 0 && d[idx[j]] > d[key]) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = key;
  }
  for (int64_t i = 0; i < l; ++i) {
    evals[i] = d[idx[i]];
    for (int64_t k = 0; k < l; ++k) Vs[k * l + i] = V[k * l + idx[i]];
  }
  memcpy(V, Vs, sizeof(double) * (size_t)(l * l));
  free(idx);
  free(d);
  free(Vs);
  return sweeps + 1;
}

/* Alg. 3 (eigSVD) for C (r x l, r >= l, row-major):
 *   [V, D] = eig(C^T C);  S = sqrt(D);  U = C V S^{-1};
 *   U = fliplr(U), V = fliplr(V), S = rot90(S, 2)   (descending order).
 * Eigenvalues below zero (rounding) are clamped at zero.  The eigenvalues of
 * the Gram matrix carry an absolute rounding error of order l * eps *
 * lambda_max, so an S at most S_max * sqrt(l * eps) cannot be told apart
 * from zero: its U column is set to zero.  U may be NULL when only S
 * and V are wanted.  Returns 1 if some column was zeroed, else 0. */
int orc_eigsvd(int64_t r, int64_t l, const double *C, double *U, double *S,
               double *V) {
  double *G = (double *)malloc(sizeof(double) * (size_t)(l * l));
  double *ev = (double *)malloc(sizeof(double) * (size_t)l);
  double *Va = (double *)malloc(sizeof(double) * (size_t)(l * l));
  orc_gram(r, l, C, G);
  orc_jacobi_eig(l, G, ev, Va);
  /* descending: position i takes ascending entry l-1-i */
  for (int64_t i = 0; i < l; ++i) {
    double lam = ev[l - 1 - i];
    if (lam < 0.0) lam = 0.0;
    S[i] = sqrt(lam);
    for (int64_t k = 0; k < l; ++k) V[k * l + i] = Va[k * l + (l - 1 - i)];
  }
  const double tau = S[0] * sqrt((double)l * 2.220446049250313e-16);
  int deficient = 0;
  if (U) {
    /* W = V diag(1/S), zero column when S <= tau; U = C W */
    double *W = (double *)malloc(sizeof(double) * (size_t)(l * l));
    for (int64_t i = 0; i < l; ++i) {
      const int zero = !(S[i] > tau);
      if (zero) deficient = 1;
      for (int64_t k = 0; k < l; ++k) W[k * l + i] = zero ? 0.0 : V[k * l + i] / S[i];
    }
    orc_matmul(r, l, l, C, l, W, l, U, l);
    free(W);
  } else {
    for (int64_t i = 0; i < l; ++i)
      if (!(S[i] > tau)) deficient = 1;
  }
  free(G);
  free(ev);
  free(Va);
  return deficient;
}

/* ------------------------------------------------------------------ */
/* The accuracy check and the shift rule of Alg. 5. */

/* PVE surrogate check (Alg. 5 step 5 with eq. (19)): with E_i = S_i + a and
 * E'_i = Sprev_i + aprev,
 *     ratio = max_{i<k} |E'_i - E_i| / (S_{k+1} + a).
 * The caller chooses aprev according to the reading (R1: the stored previous
 * shift after its update; R2: the shift that produced Sprev).  Returns the
 * ratio; the pass stops when ratio <= tol. */
double orc_pve_ratio(int64_t k, const double *S, const double *Sprev, double a,
                     double aprev) {
  double worst = 0.0;
  const double denom = S[k] + a;
  for (int64_t i = 0; i < k; ++i) {
    double v = fabs((Sprev[i] + aprev) - (S[i] + a)) / denom;
    if (v > worst || v != v) worst = v;
  }
  return worst;
}

/* Dynamic shift update (Alg. 2 step 5, Alg. 5 step 6): if S_l > alpha then
 * alpha = (S_l + alpha) / 2. */
double orc_shift_update(int64_t l, const double *S, double alpha) {
  if (S[l - 1] > alpha) return 0.5 * (S[l - 1] + alpha);
  return alpha;
}

/* Proposed-multiplier form of the shift rule (the learned shift's policy;
 * our extension of Alg. 5 step 6).  The paper's update alpha <- (S_l +
 * alpha)/2 equals max(alpha, 0.5 * E_l) with E_l = S_l + alpha the surrogate
 * of sigma_l^2 (Prop. 3); a schedule replaces 0.5 by c for the shift set
 * after pass j.  Guard: from the second pass on, once the PVE ratio grows or
 * E_{k+1} shrinks between consecutive passes, *off is set and 0.5 is used
 * for the rest of the run.  Arguments: pass number j (1-based), its ratio
 * and E_{k+1}, the previous pass's ratio and E_{k+1}, E_l, the shift used in
 * pass j, and the proposed multiplier c.  Returns the next shift. */
double orc_schedule_shift(int64_t j, double ratio, double prev_ratio, double ek1,
                          double prev_ek1, double el, double alpha, double c,
                          int32_t *off) {
  if (j >= 2 && (ratio > prev_ratio || ek1 < prev_ek1)) *off = 1;
  const double mult = *off ? 0.5 : c;
  const double cand = mult * el;
  return cand > alpha ? cand : alpha;
}

/* ------------------------------------------------------------------ */
/* dashSVD, Alg. 5 (Alg. 4 when tol == 0). */

enum { ORC_SHIFT_PAPER = 0, ORC_SHIFT_NONE = 1, ORC_SHIFT_FIXED = 2, ORC_SHIFT_SCHEDULE = 3 };
enum { ORC_PVE_R2 = 0, ORC_PVE_R1 = 1, ORC_PVE_NOSURR = 2 };

typedef struct {
  int32_t passes;      /* N_p: passes executed */
  int32_t converged;   /* 1 if the check stopped the loop */
  int32_t deficient;   /* 1 if some eigSVD zeroed a column */
  int32_t trace_cap;   /* capacity of the trace arrays (passes) */
  double *alpha_used;  /* [trace_cap] shift used in pass j */
  double *ratio;       /* [trace_cap] PVE ratio of pass j */
  double *s_hat;       /* [trace_cap * l] S of pass j (may be NULL) */
  double final_alpha;
} orc_info;

/* Inputs:
 *   A: CSR m x n (row_ptr int64, col int32, val double).
 *   k, s: rank and oversampling, l = k + s.
 *   p_max, tol: pass cap and tolerance (tol = 0 runs exactly p_max passes).
 *   omega: optional m x l Gaussian block (row-major) for the m >= n
 *          orientation, or n x l when m < n; if NULL it is drawn from seed.
 *   shift_policy: PAPER (Alg. 5), NONE (alpha = 0), FIXED (set by the rule
 *          after the first pass, then frozen), SCHEDULE (after pass j the
 *          shift becomes max(alpha, sched[j] * (S_l + alpha)), with the
 *          guard described at the update; sched has p_max + 1 entries).
 *   pve_mode: R2 (default) or R1 (readings of the surrogate check), or
 *          NOSURR: the accuracy control without the surrogate that Sec. 4.3
 *          (Table 3) compares against, checking eq. (18) on the computed
 *          singular values themselves: after each pass the singular values
 *          of B = A Q (eigSVD of B, Alg. 3) are formed, E_i = sigma_i(B)^2,
 *          and the pass stops when max_{i<=k} |E'_i - E_i| / E_{k+1} <= tol,
 *          E' being the previous pass's values (zeros before the first
 *          pass, as S' in Alg. 5 step 2).  The shift rule still reads the S
 *          of eigSVD(A^T A Q - alpha Q); the trace's ratio is this ratio.
 * Outputs: U (m x k), S (k), V (n x k), row-major, signs normalised so the
 * entry of largest magnitude in each V column is positive (lowest index on
 * ties).  Q_out (optional) receives the final orthonormal basis Q in the
 * orientation the algorithm ran in (min(m,n) x l).  Returns 0 on success, 1 if not converged (tol > 0), negative on
 * invalid arguments. */
int orc_dashsvd(int64_t m, int64_t n, const int64_t *row_ptr,
                const int32_t *col, const double *val, int64_t k, int64_t s,
                int64_t p_max, double tol, uint64_t seed, const double *omega,
                int32_t shift_policy, int32_t pve_mode, const double *sched,
                double *U_out, double *S_out, double *V_out, double *Q_out,
                orc_info *info) {
  const int64_t l = k + s;
  if (k < 1 || s < 1 || l > (m < n ? m : n) || p_max < 0 || !(tol >= 0.0)) return -1;
  /* Orientation (Sec. 3.1): Alg. 4/5 are written for m >= n; a wide matrix
   * runs on A^T and the roles of U and V are exchanged at the end. */
  const int wide = m < n;
  const int64_t nnz = row_ptr[m];
  int64_t *rT = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t *cT = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  double *vT = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  orc_csr_transpose(m, n, row_ptr, col, val, rT, cT, vT);
  /* M = the m' x n' matrix the algorithm runs on (m' >= n'). */
  const int64_t M_m = wide ? n : m, M_n = wide ? m : n;
  const int64_t *M_rp = wide ? rT : row_ptr;
  const int32_t *M_c = wide ? cT : col;
  const double *M_v = wide ? vT : val;
  const int64_t *T_rp = wide ? row_ptr : rT;
  const int32_t *T_c = wide ? col : cT;
  const double *T_v = wide ? val : vT;

  double *Om = (double *)malloc(sizeof(double) * (size_t)(M_m * l));
  if (omega)
    memcpy(Om, omega, sizeof(double) * (size_t)(M_m * l));
  else
    orc_gaussian(seed, M_m, l, Om);
  double *Q = (double *)malloc(sizeof(double) * (size_t)(M_n * l));
  double *Y = (double *)malloc(sizeof(double) * (size_t)(M_m * l));
  double *Cb = (double *)malloc(sizeof(double) * (size_t)(M_n * l));
  double *Sv = (double *)malloc(sizeof(double) * (size_t)l);
  double *Sp = (double *)calloc((size_t)l, sizeof(double));
  double *Vl = (double *)malloc(sizeof(double) * (size_t)(l * l));
  /* NOSURR: squared singular values of B = A Q, this pass and the last */
  double *Eb = (double *)malloc(sizeof(double) * (size_t)l);
  double *Ebp = (double *)calloc((size_t)l, sizeof(double));
  double *Zb = (double *)malloc(sizeof(double) * (size_t)l);
  int deficient = 0;

  /* Step 2: Q = eigSVD(A^T Omega).U, alpha = alpha' = 0, S' = zeros(l). */
  orc_csr_spmm(M_n, T_rp, T_c, T_v, Om, l, Cb);
  deficient |= orc_eigsvd(M_n, l, Cb, Q, Sv, Vl);
  double alpha = 0.0, alpha_prev = 0.0;
  double prev_ratio = 0.0, prev_ek1 = 0.0;
  int32_t sched_off = 0;
  int32_t passes = 0, converged = 0;

  for (int64_t j = 1; j <= p_max; ++j) {
    /* Step 4: [Q, S] = eigSVD(A^T (A Q) - alpha Q). */
    orc_csr_spmm(M_m, M_rp, M_c, M_v, Q, l, Y);
    orc_csr_spmm(M_n, T_rp, T_c, T_v, Y, l, Cb);
    for (int64_t i = 0; i < M_n * l; ++i) Cb[i] -= alpha * Q[i];
    deficient |= orc_eigsvd(M_n, l, Cb, Q, Sv, Vl);
    passes = (int32_t)j;
    /* Step 5: the PVE surrogate check, or eq. (18) on sigma(A Q). */
    const double a_used = alpha;
    double ratio;
    if (pve_mode == ORC_PVE_NOSURR) {
      double *Vb = (double *)malloc(sizeof(double) * (size_t)(l * l));
      orc_csr_spmm(M_m, M_rp, M_c, M_v, Q, l, Y);
      orc_eigsvd(M_m, l, Y, NULL, Zb, Vb);
      free(Vb);
      for (int64_t i = 0; i < l; ++i) Eb[i] = Zb[i] * Zb[i];
      ratio = orc_pve_ratio(k, Eb, Ebp, 0.0, 0.0);
      memcpy(Ebp, Eb, sizeof(double) * (size_t)l);
    } else {
      ratio = orc_pve_ratio(k, Sv, Sp, a_used, alpha_prev);
    }
    if (info && j - 1 < info->trace_cap) {
      if (info->alpha_used) info->alpha_used[j - 1] = a_used;
      if (info->ratio) info->ratio[j - 1] = ratio;
      if (info->s_hat) memcpy(info->s_hat + (j - 1) * l, Sv, sizeof(double) * (size_t)l);
    }
    if (tol > 0.0 && ratio <= tol) {
      converged = 1;
      break;
    }
    /* Step 6: the shift rule. */
    if (shift_policy == ORC_SHIFT_PAPER) {
      alpha = orc_shift_update(l, Sv, alpha);
    } else if (shift_policy == ORC_SHIFT_FIXED) {
      if (j == 1) alpha = orc_shift_update(l, Sv, alpha);
    } else if (shift_policy == ORC_SHIFT_SCHEDULE) {
      /* schedule sched[j] for the shift set after pass j (0.5 without one) */
      const double El = Sv[l - 1] + a_used;
      const double Ek1 = Sv[k] + a_used;
      alpha = orc_schedule_shift(j, ratio, prev_ratio, Ek1, prev_ek1, El, alpha,
                                 sched ? sched[j] : 0.5, &sched_off);
      prev_ek1 = Ek1;
    }
    prev_ratio = ratio;
    /* Step 7: S' = S and alpha' per the reading. */
    memcpy(Sp, Sv, sizeof(double) * (size_t)l);
    alpha_prev = (pve_mode == ORC_PVE_R1) ? alpha : a_used;
  }

  if (Q_out) memcpy(Q_out, Q, sizeof(double) * (size_t)(M_n * l));
  /* Steps 9-11: B = A Q; [U, S, V] = eigSVD(B); keep k; V = Q V(:, 1:k). */
  orc_csr_spmm(M_m, M_rp, M_c, M_v, Q, l, Y);
  double *Ub = (double *)malloc(sizeof(double) * (size_t)(M_m * l));
  deficient |= orc_eigsvd(M_m, l, Y, Ub, Sv, Vl);
  double *Vk = (double *)malloc(sizeof(double) * (size_t)(M_n * k));
  orc_matmul(M_n, l, k, Q, l, Vl, l, Vk, k);
  /* Sign normalisation on output: largest-magnitude entry of each column of
   * the right factor positive (lowest index on ties), same flip on U. */
  for (int64_t c = 0; c < k; ++c) {
    int64_t best = 0;
    double bv = -1.0;
    for (int64_t i = 0; i < M_n; ++i) {
      double a = fabs(Vk[i * k + c]);
      if (a > bv) { bv = a; best = i; }
    }
    double sg = Vk[best * k + c] < 0.0 ? -1.0 : 1.0;
    for (int64_t i = 0; i < M_n; ++i) Vk[i * k + c] *= sg;
    for (int64_t i = 0; i < M_m; ++i) Ub[i * l + c] *= sg;
  }
  /* Outputs in the caller's orientation. */
  for (int64_t c = 0; c < k; ++c) S_out[c] = Sv[c];
  if (!wide) {
    for (int64_t i = 0; i < m; ++i)
      for (int64_t c = 0; c < k; ++c) U_out[i * k + c] = Ub[i * l + c];
    memcpy(V_out, Vk, sizeof(double) * (size_t)(n * k));
  } else {
    /* algorithm ran on A^T: its left factor (n x k) is V, its right (m x k) is U */
    for (int64_t i = 0; i < n; ++i)
      for (int64_t c = 0; c < k; ++c) V_out[i * k + c] = Ub[i * l + c];
    memcpy(U_out, Vk, sizeof(double) * (size_t)(m * k));
  }
  if (info) {
    info->passes = passes;
    info->converged = converged;
    info->deficient = deficient;
    info->final_alpha = alpha;
  }
  free(rT); free(cT); free(vT); free(Om); free(Q); free(Y); free(Cb);
  free(Sv); free(Sp); free(Vl); free(Ub); free(Vk); free(Eb); free(Ebp); free(Zb);
  if (tol > 0.0 && !converged) return 1;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Error metrics (Sec. 4): with exact sigma_1..sigma_{k+1},
 *   eps_PVE   = max_i |sigma_i^2 - ||A^T u_i||^2| / sigma_{k+1}^2
 *   eps_sigma = max_i |sigma_i - s_i| / sigma_i
 * (u_i^T A A^T u_i = sigma_i^2 for the exact left vectors). */
void orc_metrics(int64_t m, int64_t n, const int64_t *row_ptr,
                 const int32_t *col, const double *val, int64_t k,
                 const double *U, const double *S, const double *sigma_ref,
                 double *eps_pve, double *eps_sigma) {
  /* ||A^T u_i||^2 = sum over columns c of (sum_r A[r,c] U[r,i])^2 */
  double *Z = (double *)calloc((size_t)(n * k), sizeof(double));
  for (int64_t r = 0; r < m; ++r)
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
      for (int64_t i = 0; i < k; ++i) Z[(int64_t)col[e] * k + i] += val[e] * U[r * k + i];
  double pve = 0.0, es = 0.0;
  const double sk1 = sigma_ref[k] * sigma_ref[k];
  for (int64_t i = 0; i < k; ++i) {
    double nrm = 0.0;
    for (int64_t c = 0; c < n; ++c) nrm += Z[c * k + i] * Z[c * k + i];
    double v = fabs(sigma_ref[i] * sigma_ref[i] - nrm) / sk1;
    if (v > pve) pve = v;
    double w = fabs(sigma_ref[i] - S[i]) / sigma_ref[i];
    if (w > es) es = w;
  }
  free(Z);
  *eps_pve = pve;
  *eps_sigma = es;
}

/* The other two error metrics of Sec. 4, for a computed triplet (U m x k,
 * S k, V n x k, row-major) against the exact sigma_1..sigma_{k+1}:
 *   eps_res  = max_{i<=k} ||A^T u_i - s_i v_i||_2 / sigma_i,
 *   eps_spec = (||A - U diag(S) V^T||_2 - sigma_{k+1}) / sigma_{k+1}
 * (||A - A_k||_2 = sigma_{k+1}).  The spectral norm of E = A - U S V^T is
 * the square root of the largest eigenvalue of E^T E, estimated by the
 * Lanczos process with full reorthogonalisation (Golub & Van Loan,
 * Sec. 10.1; every new vector is orthogonalised twice against all earlier
 * ones) started from a Gaussian vector of the Philox stream keyed by
 * `seed`.  The largest eigenvalue of the tridiagonal T_j (by orc_jacobi_eig)
 * is a lower bound of ||E||_2^2 that does not decrease with j; the process
 * stops after `steps` steps (at most n), at an invariant subspace, or once
 * the estimate has changed by at most 1e-14 relative over 5 steps.  Outputs
 * the two metrics, ||E||_2 and the steps taken. */
static void orc_apply_ete(int64_t m, int64_t n, const int64_t *rp, const int32_t *c,
                          const double *v, const int64_t *rpT, const int32_t *cT,
                          const double *vT, int64_t k, const double *U, const double *S,
                          const double *V, const double *x, double *y, double *z,
                          double *tk) {
  /* y = A x - U (S .* (V^T x)) */
  orc_csr_spmm(m, rp, c, v, x, 1, y);
  for (int64_t i = 0; i < k; ++i) {
    double d = 0.0;
    for (int64_t r = 0; r < n; ++r) d += V[r * k + i] * x[r];
    tk[i] = S[i] * d;
  }
  for (int64_t r = 0; r < m; ++r) {
    double d = 0.0;
    for (int64_t i = 0; i < k; ++i) d += U[r * k + i] * tk[i];
    y[r] -= d;
  }
  /* z = A^T y - V (S .* (U^T y)) */
  orc_csr_spmm(n, rpT, cT, vT, y, 1, z);
  for (int64_t i = 0; i < k; ++i) {
    double d = 0.0;
    for (int64_t r = 0; r < m; ++r) d += U[r * k + i] * y[r];
    tk[i] = S[i] * d;
  }
  for (int64_t r = 0; r < n; ++r) {
    double d = 0.0;
    for (int64_t i = 0; i < k; ++i) d += V[r * k + i] * tk[i];
    z[r] -= d;
  }
}

static double orc_tridiag_max_eig(int64_t j, const double *al, const double *be) {
  double *T = (double *)calloc((size_t)(j * j), sizeof(double));
  double *ev = (double *)malloc(sizeof(double) * (size_t)j);
  double *Vt = (double *)malloc(sizeof(double) * (size_t)(j * j));
  for (int64_t i = 0; i < j; ++i) {
    T[i * j + i] = al[i];
    if (i + 1 < j) T[i * j + i + 1] = T[(i + 1) * j + i] = be[i];
  }
  orc_jacobi_eig(j, T, ev, Vt);
  const double lam = ev[j - 1];
  free(T); free(ev); free(Vt);
  return lam;
}

void orc_residual_metrics(int64_t m, int64_t n, const int64_t *row_ptr,
                          const int32_t *col, const double *val, int64_t k,
                          const double *U, const double *S, const double *V,
                          const double *sigma_ref, int64_t steps, uint64_t seed,
                          double *eps_res, double *eps_spec, double *enorm,
                          int64_t *steps_taken) {
  const int64_t nnz = row_ptr[m];
  int64_t *rT = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int32_t *cT = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  double *vT = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  orc_csr_transpose(m, n, row_ptr, col, val, rT, cT, vT);
  /* eps_res: Z = A^T U (n x k), then the column norms of Z - V diag(S) */
  double *Z = (double *)malloc(sizeof(double) * (size_t)(n * k));
  orc_csr_spmm(n, rT, cT, vT, U, k, Z);
  double res = 0.0;
  for (int64_t i = 0; i < k; ++i) {
    double s2 = 0.0;
    for (int64_t r = 0; r < n; ++r) {
      const double d = Z[r * k + i] - S[i] * V[r * k + i];
      s2 += d * d;
    }
    const double e = sqrt(s2) / sigma_ref[i];
    if (e > res || e != e) res = e;
  }
  free(Z);
  /* ||E||_2 by Lanczos on E^T E */
  if (steps > n) steps = n;
  if (steps < 1) steps = 1;
  double *Qv = (double *)malloc(sizeof(double) * (size_t)((steps + 1) * n));
  double *al = (double *)malloc(sizeof(double) * (size_t)steps);
  double *be = (double *)malloc(sizeof(double) * (size_t)steps);
  double *y = (double *)malloc(sizeof(double) * (size_t)m);
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  double *tk = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
  orc_gaussian(seed, n, 1, Qv);
  double nrm = 0.0;
  for (int64_t r = 0; r < n; ++r) nrm += Qv[r] * Qv[r];
  nrm = sqrt(nrm);
  for (int64_t r = 0; r < n; ++r) Qv[r] /= nrm;
  double lam = 0.0, lam_old = -1.0;
  int64_t j = 0;
  for (; j < steps; ++j) {
    const double *q = Qv + j * n;
    orc_apply_ete(m, n, row_ptr, col, val, rT, cT, vT, k, U, S, V, q, y, w, tk);
    double a = 0.0;
    for (int64_t r = 0; r < n; ++r) a += q[r] * w[r];
    al[j] = a;
    for (int pass = 0; pass < 2; ++pass) {
      for (int64_t i = 0; i <= j; ++i) {
        const double *qi = Qv + i * n;
        double d = 0.0;
        for (int64_t r = 0; r < n; ++r) d += qi[r] * w[r];
        for (int64_t r = 0; r < n; ++r) w[r] -= d * qi[r];
      }
    }
    double b = 0.0;
    for (int64_t r = 0; r < n; ++r) b += w[r] * w[r];
    b = sqrt(b);
    be[j] = b;
    const int last = j + 1 == steps || !(b > 1e-14 * fabs(a));
    if (last || (j + 1) % 5 == 0) {
      lam = orc_tridiag_max_eig(j + 1, al, be);
      if (last || fabs(lam - lam_old) <= 1e-14 * lam) {
        ++j;
        break;
      }
      lam_old = lam;
    }
    double *qn = Qv + (j + 1) * n;
    for (int64_t r = 0; r < n; ++r) qn[r] = w[r] / b;
  }
  const double en = sqrt(lam > 0.0 ? lam : 0.0);
  *eps_res = res;
  *enorm = en;
  *eps_spec = (en - sigma_ref[k]) / sigma_ref[k];
  *steps_taken = j;
  free(Qv); free(al); free(be); free(y); free(w); free(tk);
  free(rT); free(cT); free(vT);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
