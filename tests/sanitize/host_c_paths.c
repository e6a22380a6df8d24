/* Sanitizer harness (ASan + UBSan, host code only) for the plain C parts:
 * the oracle (dashsvd_oracle.c) and the power-law sampler (zipf_gen.c).
 * Builds small inputs, runs every oracle entry the tests use and the
 * sampler, and exits 0; any out-of-bounds access, use after free or
 * undefined behaviour aborts with the sanitizer's report.  Built and run by
 * tests/test_sanitize_host.py. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t passes, converged, deficient, trace_cap;
  double *alpha_used, *ratio, *s_hat;
  double final_alpha;
} orc_info;

int orc_dashsvd(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, int64_t k,
                int64_t s, int64_t p_max, double tol, uint64_t seed, const double *omega, int32_t shift_policy,
                int32_t pve_mode, const double *sched, double *U_out, double *S_out, double *V_out, double *Q_out,
                orc_info *info);
void orc_metrics(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, int64_t k,
                 const double *U, const double *S, const double *sigma_ref, double *eps_pve, double *eps_sigma);
void orc_residual_metrics(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                          int64_t k, const double *U, const double *S, const double *V, const double *sigma_ref,
                          int64_t steps, uint64_t seed, double *eps_res, double *eps_spec, double *enorm,
                          int64_t *steps_taken);
void zipf_fill(int64_t m, int64_t n, const int64_t *row_ptr, const double *cdf, const double *logw, uint64_t seed,
               int32_t *col, float *val);

/* m x n CSR with the given row degrees drawn by the sampler (Zipf-like
 * column law), returned in FP64. */
static void make_csr(int64_t m, int64_t n, const int64_t *deg, int64_t **rp, int32_t **col, double **val) {
  *rp = malloc(sizeof(int64_t) * (size_t)(m + 1));
  (*rp)[0] = 0;
  for (int64_t r = 0; r < m; ++r) (*rp)[r + 1] = (*rp)[r] + deg[r];
  const int64_t nnz = (*rp)[m];
  double *w = malloc(sizeof(double) * (size_t)n), *cdf = malloc(sizeof(double) * (size_t)n),
         *logw = malloc(sizeof(double) * (size_t)n);
  double tot = 0.0;
  for (int64_t j = 0; j < n; ++j) tot += (w[j] = pow((double)((j * 7919) % n + 1), -1.1));
  double acc = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    acc += w[j] / tot;
    cdf[j] = acc;
    logw[j] = log(w[j]);
  }
  cdf[n - 1] = 1.0;
  *col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  float *vf = malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
  zipf_fill(m, n, *rp, cdf, logw, 77, *col, vf);
  *val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  for (int64_t i = 0; i < nnz; ++i) (*val)[i] = vf[i];
  free(w); free(cdf); free(logw); free(vf);
}

static int run_case(int64_t m, int64_t n, int64_t k, int64_t s, int32_t pve_mode, int32_t policy) {
  int64_t *deg = malloc(sizeof(int64_t) * (size_t)m);
  for (int64_t r = 0; r < m; ++r) deg[r] = r == 0 ? n : 1 + (r * 13) % (n / 3 + 1);  /* one full row */
  int64_t *rp;
  int32_t *col;
  double *val;
  make_csr(m, n, deg, &rp, &col, &val);
  const int64_t l = k + s, mn = m < n ? m : n, P = 6;
  double *U = malloc(sizeof(double) * (size_t)(m * k)), *S = malloc(sizeof(double) * (size_t)k),
         *V = malloc(sizeof(double) * (size_t)(n * k)), *Q = malloc(sizeof(double) * (size_t)(mn * l));
  double *a = malloc(sizeof(double) * P), *r = malloc(sizeof(double) * P), *sh = malloc(sizeof(double) * P * l);
  double *sched = malloc(sizeof(double) * (P + 1));
  for (int i = 0; i <= P; ++i) sched[i] = 0.7;
  orc_info info = {0, 0, 0, (int32_t)P, a, r, sh, 0.0};
  int st = orc_dashsvd(m, n, rp, col, val, k, s, P, 1e-3, 5, NULL, policy, pve_mode, sched, U, S, V, Q, &info);
  if (st < 0) return 1;
  double *sig = malloc(sizeof(double) * (size_t)(k + 1));
  for (int64_t i = 0; i <= k; ++i) sig[i] = 1.0 + (double)(k - i);
  double pve, es, er, esp, en;
  int64_t steps;
  orc_metrics(m, n, rp, col, val, k, U, S, sig, &pve, &es);
  orc_residual_metrics(m, n, rp, col, val, k, U, S, V, sig, 40, 3, &er, &esp, &en, &steps);
  printf("case %lld x %lld k %lld: passes %d pve %.3g res %.3g spec %.3g steps %lld\n", (long long)m,
         (long long)n, (long long)k, info.passes, pve, er, esp, (long long)steps);
  free(deg); free(rp); free(col); free(val); free(U); free(S); free(V); free(Q); free(a); free(r); free(sh);
  free(sched); free(sig);
  return 0;
}

int main(void) {
  int bad = 0;
  bad |= run_case(300, 120, 8, 4, 0, 0);   /* tall, surrogate check (R2), paper rule */
  bad |= run_case(90, 260, 6, 5, 1, 2);    /* wide, R1, fixed shift */
  bad |= run_case(200, 150, 10, 6, 2, 3);  /* no surrogate, schedule */
  bad |= run_case(40, 40, 3, 2, 0, 1);     /* square, no shift */
  return bad;
}
