// Orthonormalisation of a power-pass block without its eigenvectors.
//
// eigSVD (Alg. 3) of a block C gives Q = C V S^-1 and the singular values S.
// Inside the passes of Alg. 5 only two things of it are used: the values S
// (PVE check of step 5, shift rule of step 6) and the span of Q.  The next
// block is (M^T M - alpha I) Q, and another orthonormal basis Q' = Q X of
// the same span (X orthogonal) gives the next block times X: the same
// singular values and the same span again.  Eigenvectors are needed only by
// the final Rayleigh-Ritz step (steps 9-11), which keeps the Jacobi solver.
// So a pass block is orthonormalised from its Gram matrix G = C^T C (FP64)
// by two workgroups:
//   - workgroup 0: the Cholesky factorisation G = L L^T (right-looking, one
//     column per step) and X = L^-1 (one row per step); W = X^T = R^-1 with
//     R = L^T, so Q = C W has Q^T Q = I (Cholesky-QR);
//   - workgroup 1: the eigenvalues of G: Householder reduction to a
//     symmetric tridiagonal T (Golub & Van Loan Sec. 8.3.1), then every
//     eigenvalue by multisection of the Gershgorin interval with Sturm
//     counts (Sec. 8.4.1); S = sqrt(max(lambda, 0)) in descending order.
// The workgroup that finishes second accepts the call when the
// factorisation completed and lambda_min > 2^-32 lambda_max (then the
// Cholesky-QR basis is as orthonormal as the eigSVD one: both lose
// orthogonality as kappa(G) times the rounding of G), runs the pass tail,
// and otherwise flags the call for the Jacobi eigensolver launched after
// it on the same stream.
#include <cmath>

#include "common.h"
#include "pass_tail.h"

namespace dsv {

namespace {

constexpr int kCqThreads = 1024;
constexpr int kCqWaves = kCqThreads / kWave;
constexpr int kCqMaxL = 160;
constexpr int kSeg = 8;   // lanes per dot product
constexpr int kSect = 2;  // evaluation points per eigenvalue and multisection step
// steps to shrink an interval by 2^-53: each step divides it by kSect + 1
constexpr int kSectSteps = 34;
static_assert(kSect == 2, "kSectSteps is set for kSect = 2");

// row-packed lower triangle: (i, j) with j <= i
__device__ __forceinline__ int pl(int i, int j) { return (i * (i + 1)) / 2 + j; }

// (ii, kk), kk <= ii, of entry t of a row-packed lower triangle
__device__ __forceinline__ void unpack_lower(int t, int &ii, int &kk) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (((i + 1) * (i + 2)) / 2 <= t) ++i;
  while ((i * (i + 1)) / 2 > t) --i;
  ii = i;
  kk = t - (i * (i + 1)) / 2;
}

__device__ __forceinline__ double seg_sum(double x) {
  x += __shfl_xor(x, 1, kSeg);
  x += __shfl_xor(x, 2, kSeg);
  x += __shfl_xor(x, 4, kSeg);
  return x;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// hardware reciprocal refined by two Newton steps
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Number of eigenvalues of the tridiagonal (d, off-diagonal squares e2)
// below x: the negative pivots of the LDL^T factorisation of T - x I, a
// pivot of magnitude below kPivMin taken as -kPivMin (T is scaled so that
// its entries are below 1, which keeps e2 / q finite).
__device__ __forceinline__ int sturm_count(const double *d, const double *e2, int n, double x) {
  constexpr double kPivMin = 0x1.0p-1000;
  double q = d[0] - x;
  if (fabs(q) < kPivMin) q = -kPivMin;
  int c = q < 0.0 ? 1 : 0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] * rcp_nr(q);
    if (fabs(q) < kPivMin) q = -kPivMin;
    c += q < 0.0 ? 1 : 0;
  }
  return c;
}

__global__ __launch_bounds__(kCqThreads) void k_cholqr(EigArgs a) {
  SolverState *state = a.state;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int l = a.l;
  const bool handover = a.mode == 2 && !state->done && state->cq_off;
  if (!handover && a.call_idx > 0 && blockIdx.x == 0 && tid == 0) signal_started(&state->eig_started, a.call_idx);
  if (a.mode == 2) {
    // a pass launched after the check already passed: nothing to do
    const int stopped = state->done;
    if (blockIdx.x == 0 && tid == 0) {
      state->skip_rescale = stopped;
      if (stopped) state->cq_fallback = 0;
    }
    if (stopped) return;
    // near the end of the run: the Jacobi eigensolver takes over (and
    // signals its own start)
    if (handover) {
      if (blockIdx.x == 0 && tid == 0) state->cq_fallback = 1;
      return;
    }
  }
  extern __shared__ double A[];  // lower triangle of G, row-packed
  for (int idx = tid; idx < l * l; idx += kCqThreads) {
    const int i = idx / l, j = idx - i * l;
    if (j <= i) A[pl(i, j)] = a.G[idx];
  }
  __syncthreads();

  if (blockIdx.x == 0) {
    // ------------------------------------------------ Cholesky and L^-1
    __shared__ double Ld[kCqMaxL];      // diagonal of L
    __shared__ double lrow[2][kCqMaxL];  // row of L being inverted
    bool ok = true;
    // Step s: column s of L and the update of the trailing entries by
    // column s - 1 (A <- A - L(:, s-1) L(:, s-1)^T).  The pivot is formed
    // by every thread from entries this step does not write, and the new
    // diagonal entry goes to Ld, so the step needs one barrier.
    for (int s = 0; s < l; ++s) {
      const double ls = s > 0 ? A[pl(s, s - 1)] : 0.0;
      const double piv = fma(-ls, ls, A[pl(s, s)]);
      if (!(piv > 0.0) || !(piv < INFINITY)) {
        ok = false;
        break;
      }
      const double sq = sqrt(piv);
      const double inv = 1.0 / sq;
      if (s == 0) {
        for (int i = tid; i < l; i += kCqThreads) {
          if (i == 0)
            Ld[0] = sq;
          else
            A[pl(i, 0)] *= inv;
        }
      } else {
        const int m = l - s, cnt = m * (m + 1) / 2;
        for (int t = tid; t < cnt; t += kCqThreads) {
          int ii, kk;
          unpack_lower(t, ii, kk);
          const int i = s + ii, k = s + kk;
          const double li = A[pl(i, s - 1)], lk = A[pl(k, s - 1)];
          if (kk == 0) {
            if (ii == 0)
              Ld[s] = sq;
            else
              A[pl(i, s)] = fma(-li, lk, A[pl(i, s)]) * inv;
          } else {
            A[pl(i, k)] = fma(-li, lk, A[pl(i, k)]);
          }
        }
      }
      __syncthreads();
    }
    if (ok) {
      // X = L^-1 in place, row by row: X_ii = 1 / L_ii and, for j < i,
      // X_ij = -X_ii sum_{t=j}^{i-1} L_it X_tj (rows t < i are already X);
      // row i of L is read from a copy made during the previous row.
      for (int i = tid; i < l; i += kCqThreads) A[pl(i, i)] = 1.0 / Ld[i];
      if (l > 1 && tid == 0) lrow[1][0] = A[pl(1, 0)];
      __syncthreads();
      const int g = tid / kSeg, q = tid % kSeg;
      for (int i = 1; i < l; ++i) {
        const double *row = lrow[i & 1];
        const double xi = A[pl(i, i)];
        if (i + 1 < l) {
          for (int t = tid; t <= i; t += kCqThreads) lrow[(i + 1) & 1][t] = A[pl(i + 1, t)];
        }
        for (int j = g; j < i; j += kCqThreads / kSeg) {
          double sum = 0.0;
          for (int t = j + q; t < i; t += kSeg) sum = fma(row[t], A[pl(t, j)], sum);
          sum = seg_sum(sum);
          if (q == 0) A[pl(i, j)] = -xi * sum;
        }
        __syncthreads();
      }
      // W = X^T (upper triangular), l x l row-major
      for (int idx = tid; idx < l * l; idx += kCqThreads) {
        const int r = idx / l, c = idx - r * l;
        a.W[idx] = r <= c ? A[pl(c, r)] : 0.0;
      }
    }
    if (tid == 0) state->cq_chol_ok = ok ? 1 : 0;
  } else {
    // ------------------------------------------------ tridiagonal + eigenvalues
    __shared__ double vb[2][kCqMaxL];  // part below the diagonal of the column being reduced
    __shared__ double ush[kCqMaxL];
    __shared__ double dd[kCqMaxL], ee[kCqMaxL];
    __shared__ double part1[kCqWaves], part2[2][kCqWaves];
    // column c below its diagonal into vb[c & 1], and the partial sums of
    // the squares of its entries after the first into part2[c & 1]
    auto column_prep = [&](int c) {
      double sq = 0.0;
      for (int i = tid; i < l - 1 - c; i += kCqThreads) {
        const double x = A[pl(c + 1 + i, c)];
        vb[c & 1][i] = x;
        if (i >= 1) sq = fma(x, x, sq);
      }
      sq = wave_sum(sq);
      if (lane == 0) part2[c & 1][wave] = sq;
    };
    if (l > 2) column_prep(0);
    __syncthreads();
    const int g = tid / kSeg, q = tid % kSeg;
    // Step p: the Householder reflector H = I - beta v v^T that zeroes
    // column p below its subdiagonal, then A22 <- H A22 H on the trailing
    // block (rows and columns p+1..l-1) as A22 - v w^T - w v^T with
    // u = beta A22 v, w = u - (beta/2)(v^T u) v.  Two barriers: after u,
    // after the update (which also extracts the next column).
    for (int p = 0; p + 2 < l; ++p) {
      const int m = l - 1 - p;
      const double *v = vb[p & 1];
      double tail = 0.0;
      for (int w = 0; w < kCqWaves; ++w) tail += part2[p & 1][w];
      const double x0 = v[0];
      if (tail == 0.0) {
        // already reduced: H = I
        if (tid == 0) {
          dd[p] = A[pl(p, p)];
          ee[p] = x0;
        }
        column_prep(p + 1);
        __syncthreads();
        continue;
      }
      const double nrm = sqrt(fma(x0, x0, tail));
      const double alpha = x0 >= 0.0 ? -nrm : nrm;
      const double v0 = x0 - alpha;  // no cancellation: x0 and -alpha share the sign
      const double beta = 2.0 / fma(v0, v0, tail);
      double acc = 0.0;
      for (int ii = g; ii < m; ii += kCqThreads / kSeg) {
        const int i = p + 1 + ii;
        double sum = 0.0;
        for (int kk = q; kk < m; kk += kSeg) {
          const int k = p + 1 + kk;
          const double aik = kk <= ii ? A[pl(i, k)] : A[pl(k, i)];
          sum = fma(aik, kk == 0 ? v0 : v[kk], sum);
        }
        sum = seg_sum(sum);
        if (q == 0) {
          const double u = beta * sum;
          ush[ii] = u;
          acc = fma(ii == 0 ? v0 : v[ii], u, acc);
        }
      }
      acc = wave_sum(acc);
      if (lane == 0) part1[wave] = acc;
      __syncthreads();
      double vu = 0.0;
      for (int w = 0; w < kCqWaves; ++w) vu += part1[w];
      const double K = 0.5 * beta * vu;
      double *vn = vb[(p + 1) & 1];
      double sq = 0.0;
      const int cnt = m * (m + 1) / 2;
      for (int t = tid; t < cnt; t += kCqThreads) {
        int ii, kk;
        unpack_lower(t, ii, kk);
        const int i = p + 1 + ii, k = p + 1 + kk;
        const double vi = ii == 0 ? v0 : v[ii], vk = kk == 0 ? v0 : v[kk];
        const double wi = fma(-K, vi, ush[ii]), wk = fma(-K, vk, ush[kk]);
        const double nv = fma(-wi, vk, fma(-vi, wk, A[pl(i, k)]));
        A[pl(i, k)] = nv;
        if (kk == 0 && ii >= 1) {
          vn[ii - 1] = nv;
          if (ii >= 2) sq = fma(nv, nv, sq);
        }
      }
      sq = wave_sum(sq);
      if (lane == 0) part2[(p + 1) & 1][wave] = sq;
      if (tid == 0) {
        dd[p] = A[pl(p, p)];
        ee[p] = alpha;
      }
      __syncthreads();
    }
    if (tid == 0) {
      if (l >= 2) {
        dd[l - 2] = A[pl(l - 2, l - 2)];
        dd[l - 1] = A[pl(l - 1, l - 1)];
        ee[l - 2] = A[pl(l - 1, l - 2)];
      } else {
        dd[0] = A[0];
      }
    }
    __syncthreads();

    // T scaled by a power of two so that its largest entry lies in [1/2, 1)
    __shared__ double td[kCqMaxL], te2[kCqMaxL];
    double mx = 0.0;
    for (int i = 0; i < l; ++i) mx = fmax(mx, fabs(dd[i]));
    for (int i = 0; i + 1 < l; ++i) mx = fmax(mx, fabs(ee[i]));
    if (!(mx > 0.0) || !(mx < INFINITY)) {
      // nothing to bisect: report zeros (the call then goes to Jacobi)
      for (int i = tid; i < l; i += kCqThreads) a.S[i] = 0.0;
    } else {
      int ex = 0;
      (void)frexp(mx, &ex);
      for (int i = tid; i < l; i += kCqThreads) {
        td[i] = ldexp(dd[i], -ex);
        if (i + 1 < l) {
          const double e = ldexp(ee[i], -ex);
          te2[i] = e * e;
        }
      }
      __syncthreads();
      // Gershgorin interval, widened by 2^-40 of its magnitude (well above
      // the rounding of the Sturm counts)
      double lo = INFINITY, hi = -INFINITY;
      for (int i = 0; i < l; ++i) {
        const double r = (i > 0 ? fabs(ldexp(ee[i - 1], -ex)) : 0.0) + (i + 1 < l ? fabs(ldexp(ee[i], -ex)) : 0.0);
        lo = fmin(lo, td[i] - r);
        hi = fmax(hi, td[i] + r);
      }
      const double wid = fmax(fabs(lo), fabs(hi));
      lo -= 0x1.0p-40 * wid;
      hi += 0x1.0p-40 * wid;
      // eigenvalue r (ascending) by the kSect lanes of group r: each step
      // evaluates the count at kSect interior points of [lo_r, hi_r) and
      // keeps the piece where it passes r; count(lo_r) <= r < count(hi_r)
      const int r = tid / kSect, qq = tid % kSect;
      if (r < l) {
        double lo_r = lo, hi_r = hi;
        for (int it = 0; it < kSectSteps; ++it) {
          const double x = lo_r + (hi_r - lo_r) * ((double)(qq + 1) / (double)(kSect + 1));
          const int c = sturm_count(td, te2, l, x);
          double nhi = hi_r;
          bool found = false;
#pragma unroll
          for (int z = 0; z < kSect; ++z) {
            const int cz = __shfl(c, z, kSect);
            const double xz = __shfl(x, z, kSect);
            if (!found && cz > r) {
              nhi = xz;
              found = true;
            }
          }
          double nlo = lo_r;
#pragma unroll
          for (int z = 0; z < kSect; ++z) {
            const int cz = __shfl(c, z, kSect);
            const double xz = __shfl(x, z, kSect);
            if (cz <= r && xz < nhi) nlo = xz;
          }
          lo_r = nlo;
          hi_r = nhi;
        }
        if (qq == 0) {
          const double lam = ldexp(0.5 * (lo_r + hi_r), ex);
          a.S[l - 1 - r] = sqrt(fmax(lam, 0.0));
        }
      }
    }
  }

  // ---------------------------------------------------- the second workgroup finishes
  __threadfence();
  __syncthreads();
  __shared__ int s_last;
  if (tid == 0) s_last = atomicAdd(&state->cq_arrive, 1);
  __syncthreads();
  if (s_last == 0) return;
  __threadfence();
  __shared__ double Ssh[kCqMaxL];
  __shared__ int s_chol;
  for (int i = tid; i < l; i += kCqThreads) Ssh[i] = a.S[i];
  if (tid == 0) s_chol = state->cq_chol_ok;
  __syncthreads();
  const bool ok = s_chol && Ssh[0] > 0.0 && Ssh[0] < INFINITY && Ssh[l - 1] > 0x1.0p-16 * Ssh[0];
  if (tid == 0) {
    state->cq_arrive = 0;
    state->cq_fallback = ok ? 0 : 1;
  }
  if (!ok) return;
  if (tid == 0) {
    if (a.sweeps) *a.sweeps = 0;
    if (a.trace_sweeps && state->eig_calls < a.trace_cap + 2) a.trace_sweeps[state->eig_calls] = 0;
    state->eig_calls += 1;
    state->cq_calls += 1;
  }
  if (a.mode != 2) return;
  __syncthreads();
  pass_tail(a, state, Ssh);
}

__global__ __launch_bounds__(kWave) void k_wait_started(const int32_t *flag, int32_t expect) {
  // wall clock at 100 MHz: give up after 200 us
  const long long t0 = wall_clock64();
  while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < expect) {
    if (wall_clock64() - t0 > 20000) break;
    __builtin_amdgcn_s_sleep(2);
  }
}

}  // namespace

hipError_t launch_wait_started(const int32_t *flag, int32_t expect, hipStream_t st) {
  hipLaunchKernelGGL(k_wait_started, dim3(1), dim3(kWave), 0, st, flag, expect);
  return hipGetLastError();
}

hipError_t launch_cholqr(const EigArgs &a, hipStream_t st) {
  if (!a.state || a.l < 1 || a.l > kCqMaxL || (a.mode != 1 && a.mode != 2)) return hipErrorInvalidValue;
  const size_t shm = sizeof(double) * (size_t)a.l * (size_t)(a.l + 1) / 2;
  static size_t shm_set = 64 * 1024;
  if (shm > shm_set) {
    const hipError_t e = hipFuncSetAttribute((const void *)k_cholqr, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)shm);
    if (e != hipSuccess) return e;
    shm_set = shm;
  }
  hipLaunchKernelGGL(k_cholqr, dim3(2), dim3(kCqThreads), shm, st, a);
  return hipGetLastError();
}

hipError_t launch_eig_pass(const EigArgs &a, hipStream_t st) {
  const hipError_t e = launch_cholqr(a, st);
  if (e != hipSuccess) return e;
  EigArgs b = a;
  b.run_if = &a.state->cq_fallback;
  return launch_eig(b, st);
}

}  // namespace dsv
