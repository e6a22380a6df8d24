// Eigen-decomposition of the Gram matrix of an eigSVD block (Alg. 3 steps
// 1-4) through a symmetric tridiagonal form, in one workgroup:
//   1. Householder reduction G = H T H^T (Golub & Van Loan Sec. 8.3.1); the
//      reflector vector of step p is kept in row p of the reduced matrix;
//   2. every eigenvalue of T by multisection on Sturm counts (Sec. 8.4.1):
//      eight lanes per eigenvalue evaluate eight points a step, and 17 steps
//      narrow the Gershgorin interval below 2^-53 of its width;
//   3. every eigenvector of T from its twisted factorisation
//      T - lambda I = N_t Delta N_t^T at the twist index t where |gamma_t| is
//      smallest: z_t = 1 and two recurrences outward (one step of inverse
//      iteration from e_t; Dhillon and Parlett, Linear Algebra Appl. 387,
//      2004), normalised;
//   4. V = H Z, the reflectors applied to Z held in registers (eight lanes a
//      column, no barrier: the columns are independent).
// Outputs as the Jacobi kernels: S = sqrt(eig G) descending, W = V diag(1/S)
// with columns zeroed where S <= S_max sqrt(l eps), Vs = V, and the pass
// tail (PVE check, shift rule) for a power-pass block.
//
// Accuracy is normwise (an eigenvalue to about eps ||G||, an eigenvector to
// about eps ||G|| / gap), as with the paper's LAPACK eigensolver; the solver
// uses this kernel for the FP32 and BF16 forms, whose Jacobi threshold is
// 2^-23.  Where two eigenvalues lie within 2^-30 ||G|| of each other their
// vectors would not be orthogonal to that level, and a non-finite G has no
// decomposition: the call then declines (*decline = 1, nothing written) and
// the two-sided Jacobi kernel launched after it on the same stream runs.
// l <= 128 (G in LDS as a square array).  W and Vs serve as scratch for the
// factorisations of step 3 before they receive the results.
#include <cstring>

#include "common.h"
#include "pass_tail.h"

namespace dsv {

namespace {

constexpr int kTT = 1024;          // threads
constexpr int kTWaves = kTT / kWave;
constexpr int kTMaxL = 128;
constexpr int kPts = 8;            // evaluation points per eigenvalue and step
constexpr int kSectSteps = 17;     // 9^17 > 2^53
constexpr double kPivMin = 0x1.0p-1000;

__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// sum over the eight lanes of an aligned group
__device__ __forceinline__ double sum8(double x) {
  x += __shfl_xor(x, 1, 8);
  x += __shfl_xor(x, 2, 8);
  x += __shfl_xor(x, 4, 8);
  return x;
}

// Number of eigenvalues of the tridiagonal (d, off-diagonal squares e2) below
// x: the negative pivots of the LDL^T factorisation of T - x I, a pivot of
// magnitude below kPivMin taken as -kPivMin (T is scaled so that its entries
// are below 1).
__device__ __forceinline__ int sturm_count(const double *d, const double *e2, int n, double x) {
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

__device__ __forceinline__ double guard(double q) { return fabs(q) < kPivMin ? -kPivMin : q; }

__global__ __launch_bounds__(kTT) void k_eigtri(EigArgs a) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  if ((a.run_if && *a.run_if == 0) || (a.skip_if && *a.skip_if)) {
    if (tid == 0 && a.decline) *a.decline = 0;
    return;
  }
  SolverState *state = a.state;
  if (state && a.call_idx > 0 && tid == 0) signal_started(&state->eig_started, a.call_idx);
  if (state && a.mode == 2) {
    const int stopped = state->done;
    __syncthreads();
    if (tid == 0) state->skip_rescale = stopped;
    if (stopped) {
      if (tid == 0 && a.decline) *a.decline = 0;
      return;
    }
  }
  const int l = a.l;
  extern __shared__ double A[];  // l x l, row-major
  __shared__ double vv[kTMaxL], uu[kTMaxL], dd[kTMaxL], ee[kTMaxL], bet[kTMaxL];
  __shared__ double td[kTMaxL], te[kTMaxL], te2[kTMaxL], lam[kTMaxL], znrm[kTMaxL];
  __shared__ double Ssh[kTMaxL];
  __shared__ int twist[kTMaxL];
  __shared__ double part[2][kTWaves];
  __shared__ int s_bad;
  int pc = 0;  // partial-sum buffer in use (double-buffered: one barrier a sum)
  auto block_sum = [&](double x) __attribute__((always_inline)) -> double {
    x = wave_sum(x);
    if (lane == 0) part[pc][wave] = x;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kTWaves; ++w) s += part[pc][w];
    pc ^= 1;
    return s;
  };

  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int idx = tid; idx < l * l; idx += kTT) {
    const double g = a.G[idx];
    A[idx] = g;
    if (!(fabs(g) < INFINITY)) s_bad = 1;
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0 && a.decline) *a.decline = 1;
    return;
  }

  // ------------------------------------------------------------ 1. Householder
  // Step p: x = A(p+1:, p) (read as row p), v = x - alpha e_1, beta = 2 / v^T v,
  // u = beta A22 v, w = u - (beta/2)(v^T u) v, A22 -= v w^T + w v^T.  v goes to
  // row p (A(p, p+1:)), beta to bet[p], the diagonal and alpha to dd, ee.
  const int gseg = tid / 8, qseg = tid % 8;
  const int ty = tid / 32, tx = tid % 32;
  for (int p = 0; p + 2 < l; ++p) {
    const int m = l - 1 - p;
    double *rowp = A + (size_t)p * l + p + 1;  // x, then v
    double sq = 0.0;
    for (int i = 1 + tid; i < m; i += kTT) sq = fma(rowp[i], rowp[i], sq);
    const double tail = block_sum(sq);
    const double x0 = rowp[0];
    if (tail == 0.0) {
      // already reduced: H = I
      if (tid == 0) {
        dd[p] = A[(size_t)p * l + p];
        ee[p] = x0;
        bet[p] = 0.0;
      }
      continue;
    }
    const double nrm = sqrt(fma(x0, x0, tail));
    const double alpha = x0 >= 0.0 ? -nrm : nrm;
    const double v0 = x0 - alpha;  // no cancellation: x0 and -alpha share the sign
    const double beta = 2.0 / fma(v0, v0, tail);
    for (int i = tid; i < m; i += kTT) vv[i] = i == 0 ? v0 : rowp[i];
    __syncthreads();
    if (tid == 0) {
      dd[p] = A[(size_t)p * l + p];
      ee[p] = alpha;
      bet[p] = beta;
      rowp[0] = v0;
    }
    // u = beta A22 v, one row per 8-lane group; v^T u for K
    double acc = 0.0;
    for (int ii = gseg; ii < m; ii += kTT / 8) {
      const double *ar = A + (size_t)(p + 1 + ii) * l + p + 1;
      double s = 0.0;
      for (int kk = qseg; kk < m; kk += 8) s = fma(ar[kk], vv[kk], s);
      s = sum8(s) * beta;
      if (qseg == 0) {
        uu[ii] = s;
        acc = fma(vv[ii], s, acc);
      }
    }
    const double K = 0.5 * beta * block_sum(acc);
    // A22 -= v w^T + w v^T, w = u - K v; a 32 x 32 thread grid over the block
    for (int ii = ty; ii < m; ii += kTT / 32) {
      const double vi = vv[ii], wi = fma(-K, vi, uu[ii]);
      double *ar = A + (size_t)(p + 1 + ii) * l + p + 1;
      for (int kk = tx; kk < m; kk += 32) {
        const double vk = vv[kk], wk = fma(-K, vk, uu[kk]);
        ar[kk] = fma(-vi, wk, fma(-wi, vk, ar[kk]));
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (l >= 2) {
      dd[l - 2] = A[(size_t)(l - 2) * l + l - 2];
      dd[l - 1] = A[(size_t)(l - 1) * l + l - 1];
      ee[l - 2] = A[(size_t)(l - 1) * l + l - 2];
      bet[l - 2] = 0.0;
    } else {
      dd[0] = A[0];
    }
    if (l >= 1) bet[l - 1] = 0.0;
  }
  __syncthreads();

  // ------------------------------------------------------------ 2. eigenvalues
  // T scaled by a power of two so that its largest entry lies in [1/2, 1)
  double mx = 0.0;
  for (int i = 0; i < l; ++i) mx = fmax(mx, fabs(dd[i]));
  for (int i = 0; i + 1 < l; ++i) mx = fmax(mx, fabs(ee[i]));
  int ex = 0;
  if (mx > 0.0) (void)frexp(mx, &ex);
  for (int i = tid; i < l; i += kTT) {
    td[i] = ldexp(dd[i], -ex);
    if (i + 1 < l) {
      te[i] = ldexp(ee[i], -ex);
      te2[i] = te[i] * te[i];
    }
  }
  __syncthreads();
  {
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < l; ++i) {
      const double r = (i > 0 ? fabs(te[i - 1]) : 0.0) + (i + 1 < l ? fabs(te[i]) : 0.0);
      lo = fmin(lo, td[i] - r);
      hi = fmax(hi, td[i] + r);
    }
    const double wid = fmax(fmax(fabs(lo), fabs(hi)), 0x1.0p-900);
    lo -= 0x1.0p-40 * wid;
    hi += 0x1.0p-40 * wid;
    // eigenvalue r (ascending) by the kPts lanes of group r: each step
    // evaluates the count at kPts interior points of [lo_r, hi_r) and keeps
    // the piece where it passes r; count(lo_r) <= r < count(hi_r)
    const int r = tid / kPts, qq = tid % kPts;
    if (r < l) {
      double lo_r = lo, hi_r = hi;
      for (int it = 0; it < kSectSteps; ++it) {
        const double x = lo_r + (hi_r - lo_r) * ((double)(qq + 1) / (double)(kPts + 1));
        const int c = sturm_count(td, te2, l, x);
        double nhi = hi_r, nlo = lo_r;
        bool found = false;
#pragma unroll
        for (int z = 0; z < kPts; ++z) {
          const int cz = __shfl(c, z, kPts);
          const double xz = __shfl(x, z, kPts);
          if (!found && cz > r) {
            nhi = xz;
            found = true;
          }
        }
#pragma unroll
        for (int z = 0; z < kPts; ++z) {
          const int cz = __shfl(c, z, kPts);
          const double xz = __shfl(x, z, kPts);
          if (cz <= r && xz < nhi) nlo = xz;
        }
        lo_r = nlo;
        hi_r = nhi;
      }
      if (qq == 0) lam[r] = 0.5 * (lo_r + hi_r);
    }
  }
  __syncthreads();
  // clusters: eigenvalues within 2^-30 of the largest magnitude of each other
  {
    const double big = fmax(fabs(lam[0]), fabs(lam[l - 1]));
    for (int r = tid; r + 1 < l; r += kTT)
      if (!(lam[r + 1] - lam[r] > 0x1.0p-30 * big)) s_bad = 1;
  }
  __syncthreads();
  if (s_bad) {
    if (tid == 0 && a.decline) *a.decline = 1;
    return;
  }
  if (tid == 0 && a.decline) *a.decline = 0;

  // ------------------------------------------------------------ 3. eigenvectors of T
  // lane r: D- backward into Wk, D+ forward into Vk with gamma_i = D+_i +
  // D-_i - (d_i - lambda), then z outward from the twist t, written over the
  // factor it consumed (rows < t in Vk, rows > t in Wk; z_t = 1 implied).
  double *Wk = a.W, *Vk = a.Vs;
  if (tid < l) {
    const int r = tid;
    const double lm = lam[r];
    double q = guard(td[l - 1] - lm);
    Wk[(size_t)(l - 1) * l + r] = q;
    for (int i = l - 2; i >= 0; --i) {
      q = guard((td[i] - lm) - te2[i] * rcp_nr(q));
      Wk[(size_t)i * l + r] = q;
    }
    double dp = guard(td[0] - lm);
    Vk[r] = dp;
    double best = fabs(Wk[r]);  // gamma_0 = D-_0
    int t = 0;
    // (unrolled so that the loads of D- are issued ahead of the D+ chain)
#pragma unroll 4
    for (int i = 1; i < l; ++i) {
      dp = guard((td[i] - lm) - te2[i - 1] * rcp_nr(dp));
      Vk[(size_t)i * l + r] = dp;
      const double gm = fabs(dp + Wk[(size_t)i * l + r] - (td[i] - lm));
      if (gm < best) {
        best = gm;
        t = i;
      }
    }
    double nz = 1.0, z = 1.0;
#pragma unroll 4
    for (int i = t - 1; i >= 0; --i) {
      z = -(te[i] * rcp_nr(Vk[(size_t)i * l + r])) * z;
      Vk[(size_t)i * l + r] = z;
      nz = fma(z, z, nz);
    }
    z = 1.0;
#pragma unroll 4
    for (int i = t + 1; i < l; ++i) {
      z = -(te[i - 1] * rcp_nr(Wk[(size_t)i * l + r])) * z;
      Wk[(size_t)i * l + r] = z;
      nz = fma(z, z, nz);
    }
    twist[r] = t;
    znrm[r] = sqrt(nz);
  }
  __syncthreads();

  // ------------------------------------------------------------ 4. V = H Z
  // column j over the 8 lanes of group j: lane g holds rows g + 8 s
  constexpr int kRows = kTMaxL / 8;
  const int j = tid / 8, g8 = tid % 8;
  double vcol[kRows];
  const bool colj = j < l;
  {
    const int tj = colj ? twist[j] : 0;
    const double inv = colj ? 1.0 / znrm[j] : 0.0;
#pragma unroll
    for (int s = 0; s < kRows; ++s) {
      const int i = g8 + 8 * s;
      double z = 0.0;
      if (colj && i < l) z = i == tj ? 1.0 : (i < tj ? Vk[(size_t)i * l + j] : Wk[(size_t)i * l + j]);
      vcol[s] = z * inv;
    }
  }
  __syncthreads();  // every column is in registers before W and Vs are written
  for (int p = l - 3; p >= 0; --p) {
    const double b = bet[p];
    if (b == 0.0) continue;  // uniform
    const double *vp = A + (size_t)p * l;  // v_p(i) = A(p, i), i > p
    double s = 0.0;
#pragma unroll
    for (int s_ = 0; s_ < kRows; ++s_) {
      const int i = g8 + 8 * s_;
      if (i > p && i < l) s = fma(vp[i], vcol[s_], s);
    }
    const double w = sum8(s) * b;
#pragma unroll
    for (int s_ = 0; s_ < kRows; ++s_) {
      const int i = g8 + 8 * s_;
      if (i > p && i < l) vcol[s_] = fma(-vp[i], w, vcol[s_]);
    }
  }

  // ------------------------------------------------------------ tail
  // eigenvalue j (ascending) has rank l - 1 - j in the descending order
  for (int r = tid; r < l; r += kTT) Ssh[l - 1 - r] = sqrt(fmax(ldexp(lam[r], ex), 0.0));
  __syncthreads();
  const double tau = Ssh[0] * sqrt((double)l * 2.220446049250313e-16);
  for (int i = tid; i < l; i += kTT) a.S[i] = Ssh[i];
  if (colj) {
    const int rk = l - 1 - j;
    const double sv = Ssh[rk];
    const double iv = sv > tau ? 1.0 / sv : 0.0;
#pragma unroll
    for (int s_ = 0; s_ < kRows; ++s_) {
      const int i = g8 + 8 * s_;
      if (i < l) {
        a.W[(size_t)i * l + rk] = vcol[s_] * iv;
        a.Vs[(size_t)i * l + rk] = vcol[s_];
      }
    }
  }
  if (a.sweeps && tid == 0) *a.sweeps = 0;
  if (!state) return;
  if (tid == 0) {
    if (a.trace_sweeps && state->eig_calls < a.trace_cap + 2) a.trace_sweeps[state->eig_calls] = 0;
    state->eig_calls += 1;
  }
  if (tid == 0 && !(Ssh[l - 1] > tau)) state->deficient = 1;
  if (a.mode != 2) return;
  __syncthreads();
  pass_tail(a, state, Ssh);
}

}  // namespace

hipError_t launch_eigtri(const EigArgs &a, hipStream_t st) {
  if (a.l < 1 || a.l > kTMaxL || !a.Vs || !a.W || !a.S) return hipErrorInvalidValue;
  const size_t shm = sizeof(double) * (size_t)a.l * (size_t)a.l;
  static size_t shm_set = 64 * 1024;
  if (shm > shm_set) {
    const hipError_t e =
        hipFuncSetAttribute((const void *)k_eigtri, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    shm_set = shm;
  }
  hipLaunchKernelGGL(k_eigtri, dim3(1), dim3(kTT), shm, st, a);
  return hipGetLastError();
}

}  // namespace dsv
