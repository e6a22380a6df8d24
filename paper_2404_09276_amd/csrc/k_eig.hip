// Small symmetric eigenproblem of eigSVD (Alg. 3 steps 1-4) and the per-pass
// tail of Alg. 5 (steps 5-7: PVE check and shift update), in one workgroup.
//
// Method: parallel cyclic Jacobi in FP64 with the odd-even ordering (Luk and
// Park): on even steps the index pairs are (2g, 2g+1), on odd steps
// (2g+1, 2g+2); every rotation is followed by a swap of the two indices, so
// after L steps each pair of original indices has met once (one sweep), as
// in an odd-even transposition network.  Each rotation is the 2x2 symmetric
// Schur decomposition (Golub & Van Loan Sec. 8.5), skipped when the
// off-diagonal entry is below 2^-53 sqrt(|a_pp a_qq|); the sweeps stop when
// no entry is above that threshold.
//
// Data placement (one workgroup of 1024 threads):
//   - G lives in LDS as a packed upper triangle (L(L+1)/2 doubles, L = l
//     rounded up to a multiple of 4 with decoupled zero rows/columns);
//   - the eigenvector matrix V lives in registers: each lane owns four
//     consecutive columns of some rows, so even-step rotations stay in the
//     lane and odd steps exchange one value with the neighbouring lane;
//   - the rotation parameters of a step are published in LDS.
// A step is: rotations (one thread per pair) | barrier | 2x2 block updates
// of G (one thread per block pair) and the V update | barrier.
//
// Tail: S = sqrt(max(lambda, 0)) in descending order (ties by original
// index, descending), W = V diag(1/S) with columns zeroed where S <=
// S_max sqrt(l eps), then for a power pass the PVE ratio of eq. (19) with the
// surrogate E = S + alpha (Prop. 3) and the shift rule.
#include "common.h"

namespace dsv {

namespace {

constexpr int kEigThreads = 1024;
constexpr int kMaxLP = 160;           // padded size L (multiple of 4)
constexpr int kMaxPairs = kMaxLP / 2;
constexpr int kMaxNR = 10;            // register row slots per lane (L=160: 40 lanes/row, 1 row/wave)
constexpr int kMaxItems = 4;          // block items per thread per parity

__device__ __forceinline__ int pk(int i, int j, int L) {  // i <= j
  return i * L - ((i * (i - 1)) >> 1) + (j - i);
}
__device__ __forceinline__ int sk(int i, int j, int L) { return i <= j ? pk(i, j, L) : pk(j, i, L); }

// Group g of a parity: members (first, size).
__device__ __forceinline__ void group_of(int parity, int g, int P, int &first, int &size) {
  if (!parity) {
    first = 2 * g;
    size = 2;
  } else if (g == 0) {
    first = 0;
    size = 1;
  } else if (g == P) {
    first = 2 * P - 1;
    size = 1;
  } else {
    first = 2 * g - 1;
    size = 2;
  }
}
// rotation slot of a size-2 group
__device__ __forceinline__ int slot_of(int parity, int g) { return parity ? g - 1 : g; }

// Reciprocal and reciprocal square root from the hardware approximations
// refined by two Newton steps (relative error near 1 ulp); the rotation only
// needs c^2 + s^2 = 1 to rounding, not correctly rounded quotients.
__device__ __forceinline__ double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double frsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

template <int MAXNR>
__global__ __launch_bounds__(kEigThreads) void k_eig(EigArgs a) {
  SolverState *state = a.state;
  if (state && a.mode == 2) {
    // a pass launched after the check already passed: nothing to do, and
    // its rescale must not run either
    const int stopped = state->done;
    __syncthreads();
    if (threadIdx.x == 0) state->skip_rescale = stopped;
    if (stopped) return;
  }
  extern __shared__ double G[];  // packed upper, L(L+1)/2
  __shared__ double2 rot_cs[kMaxPairs];  // (c, s) of each pair's rotation
  __shared__ double2 rot_tf[kMaxPairs];  // (t = s/c, 1 if rotated else 0)
  __shared__ int label[kMaxLP];
  __shared__ int rank_of[kMaxLP];
  __shared__ double Ssh[kMaxLP];
  __shared__ int s_flag;
  __shared__ int s_sweeps;
  __shared__ uint16_t items[2][kMaxItems * kEigThreads];

  const int l = a.l;
  const double kSkip = a.skip;  // rotation / convergence threshold (relative)
  const int L = (l + 3) & ~3;
  const int P = L / 2;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  for (int idx = tid; idx < L * L; idx += kEigThreads) {
    const int i = idx / L, j = idx - i * L;
    if (i <= j) G[pk(i, j, L)] = (i < l && j < l) ? a.G[(int64_t)i * l + j] : 0.0;
  }
  for (int p = tid; p < L; p += kEigThreads) label[p] = p;

  // block items of both parities, decoded once into LDS: pairs of groups
  // (gb <= ga) enumerated row by row of the packed upper triangle (gb outer,
  // ga inner), so neighbouring lanes touch neighbouring LDS words; packed as
  // ga << 8 | gb (0xffff = none)
  for (int par = 0; par < 2; ++par) {
    const int ng = par ? P + 1 : P;
    const int nitems = ng * (ng + 1) / 2;
    for (int t = tid; t < kMaxItems * kEigThreads; t += kEigThreads) {
      uint16_t code = 0xffff;
      if (t < nitems) {
        int gb = 0, rem = t;
        while (rem >= ng - gb) {
          rem -= ng - gb;
          ++gb;
        }
        code = (uint16_t)(((gb + rem) << 8) | gb);
      }
      items[par][t] = code;
    }
  }

  // V in registers: lane column block cl owns columns 4cl..4cl+3 of its rows
  const int LPR = L / 4;             // lanes per row
  const int RPW = kWave / LPR;       // rows per wave
  const int sub = lane / LPR, cl = lane - sub * LPR;
  const bool active = sub < RPW;
  const int row_stride = (kEigThreads / kWave) * RPW;
  const int NR = (L + row_stride - 1) / row_stride;
  double v[MAXNR][4];
#pragma unroll
  for (int it = 0; it < MAXNR; ++it) {
    const int row = wave * RPW + sub + it * row_stride;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[it][j] = (active && row < L && row == 4 * cl + j) ? 1.0 : 0.0;
  }
  if (tid == 0) s_sweeps = 0;
  __syncthreads();

  for (int sweep = 0; sweep < 60; ++sweep) {
    // convergence test before the sweep: any entry above the skip threshold?
    if (tid == 0) s_flag = 0;
    __syncthreads();
    for (int idx = tid; idx < L * L; idx += kEigThreads) {
      const int i = idx / L, j = idx - i * L;
      if (i < j) {
        const double apq = G[pk(i, j, L)];
        if (apq != 0.0 && !(apq * apq <= kSkip * kSkip * fabs(G[pk(i, i, L)] * G[pk(j, j, L)]))) s_flag = 1;
      }
    }
    __syncthreads();
    if (!s_flag) break;
    if (tid == 0) s_sweeps = sweep + 1;
    for (int step = 0; step < L; ++step) {
      const int par = step & 1;
      const int npairs = par ? P - 1 : P;
      long long c0 = 0, w0 = 0;
      if (a.prof && tid == 0) {
        c0 = clock64();
        w0 = wall_clock64();
      }
      // phase A: rotation of each pair (and the index swap that follows it)
      if (tid < npairs) {
        const int p = par ? 2 * tid + 1 : 2 * tid, q = p + 1;
        const double app = G[pk(p, p, L)], aqq = G[pk(q, q, L)], apq = G[pk(p, q, L)];
        const int lp = label[p], lq = label[q];
        double c = 1.0, s = 0.0, t = 0.0, rot = 0.0;
        if (apq != 0.0 && !(fabs(apq) * fabs(apq) <= kSkip * kSkip * fabs(app * aqq))) {
          const double tau = (aqq - app) * 0.5 * frcp(apq);
          const double w = fma(tau, tau, 1.0);
          const double r = w * frsqrt(w);  // sqrt(1 + tau^2)
          t = tau >= 0.0 ? frcp(tau + r) : -frcp(r - tau);
          c = frsqrt(fma(t, t, 1.0));
          s = t * c;
          rot = 1.0;
        }
        rot_cs[tid] = make_double2(c, s);
        rot_tf[tid] = make_double2(t, rot);
        label[p] = lq;
        label[q] = lp;
      }
      __syncthreads();
      long long c1 = 0;
      if (a.prof && tid == 0) c1 = clock64();
      // phase B: 2x2 blocks of G, B <- Ma^T B Mb with M = J P (rotation then
      // swap): M = [[s, c], [c, -s]] when rotated, [[0, 1], [1, 0]] when not
      for (int s_ = 0; s_ < kMaxItems; ++s_) {
        const uint16_t code = items[par][tid + s_ * kEigThreads];
        if (code == 0xffff) break;
        const int ga = code >> 8, gb = code & 0xff;
        int fa, na, fb, nb;
        group_of(par, ga, P, fa, na);
        group_of(par, gb, P, fb, nb);
        int sa = slot_of(par, ga), sb = slot_of(par, gb);
        sa = sa < 0 ? 0 : (sa >= npairs ? npairs - 1 : sa);
        sb = sb < 0 ? 0 : (sb >= npairs ? npairs - 1 : sb);
        if (ga == gb) {
          if (na == 2) {
            const int p = fa, q = fa + 1;
            const double2 tf = rot_tf[sa];
            const double app = G[pk(p, p, L)], aqq = G[pk(q, q, L)], apq = G[pk(p, q, L)];
            if (tf.y != 0.0) {
              G[pk(p, p, L)] = fma(tf.x, apq, aqq);  // swapped
              G[pk(q, q, L)] = fma(-tf.x, apq, app);
              G[pk(p, q, L)] = 0.0;
            } else {
              G[pk(p, p, L)] = aqq;
              G[pk(q, q, L)] = app;
            }
          }
          continue;
        }
        // off-diagonal block: rows of ga (larger indices), columns of gb;
        // all loads issued before any use.  M = [[s, c], [c, -s]] for both the
        // rotated case and the plain swap (c = 1, s = 0); a single-index group
        // has M = [1].
        const double2 csa = rot_cs[sa], csb = rot_cs[sb];
        const int i00 = pk(fb, fa, L);
        const int i01 = nb == 2 ? pk(fb + 1, fa, L) : i00;
        const int i10 = na == 2 ? pk(fb, fa + 1, L) : i00;
        const int i11 = (na == 2 && nb == 2) ? pk(fb + 1, fa + 1, L) : i00;
        const double g00 = G[i00], g01 = G[i01], g10 = G[i10], g11 = G[i11];
        const double ma00 = na == 2 ? csa.y : 1.0, ma01 = na == 2 ? csa.x : 0.0;
        const double ma10 = na == 2 ? csa.x : 0.0, ma11 = na == 2 ? -csa.y : 1.0;
        const double mb00 = nb == 2 ? csb.y : 1.0, mb01 = nb == 2 ? csb.x : 0.0;
        const double mb10 = nb == 2 ? csb.x : 0.0, mb11 = nb == 2 ? -csb.y : 1.0;
        const double b01 = nb == 2 ? g01 : 0.0;
        const double b10 = na == 2 ? g10 : 0.0;
        const double b11 = (na == 2 && nb == 2) ? g11 : 0.0;
        // T = B Mb ; B' = Ma^T T
        const double t00 = g00 * mb00 + b01 * mb10, t01 = g00 * mb01 + b01 * mb11;
        const double t10 = b10 * mb00 + b11 * mb10, t11 = b10 * mb01 + b11 * mb11;
        G[i00] = ma00 * t00 + ma10 * t10;
        if (nb == 2) G[i01] = ma00 * t01 + ma10 * t11;
        if (na == 2) G[i10] = ma01 * t00 + ma11 * t10;
        if (na == 2 && nb == 2) G[i11] = ma01 * t01 + ma11 * t11;
      }
      long long cmid = 0;
      if (a.prof && tid == 0) cmid = clock64();
      // V <- V M (column pairs of this parity); waves that hold no row skip
      if (wave * RPW < L) {
        // Parameters (8 per lane):
        //   even: pair (p0, p0+1) -> e[0..3], pair (p0+2, p0+3) -> e[4..7]
        //   odd : pair (p0-1, p0) -> e[0] = M01, e[1] = M11 (second member here)
        //         pair (p0+1, p0+2) -> e[2..5]
        //         pair (p0+3, p0+4) -> e[6] = M00, e[7] = M10 (first member here)
        double e[8];
        auto mp = [&](int sl, double &m00, double &m01, double &m10, double &m11) {
          const int slc = sl < 0 ? 0 : (sl >= npairs ? npairs - 1 : sl);
          const double2 cs = rot_cs[slc];
          const bool in = sl >= 0 && sl < npairs;
          m00 = in ? cs.y : 1.0;
          m01 = in ? cs.x : 0.0;
          m10 = in ? cs.x : 0.0;
          m11 = in ? -cs.y : 1.0;
        };
        if (!par) {
          mp(2 * cl, e[0], e[1], e[2], e[3]);
          mp(2 * cl + 1, e[4], e[5], e[6], e[7]);
        } else {
          double d0, d1;
          mp(2 * cl - 1, d0, e[0], d1, e[1]);
          mp(2 * cl, e[2], e[3], e[4], e[5]);
          mp(2 * cl + 1, e[6], d0, e[7], d1);
        }
        const bool first = cl == 0, last = cl == LPR - 1;
#pragma unroll
        for (int it = 0; it < MAXNR; ++it) {
          if (it < NR) {
            const double v0 = v[it][0], v1 = v[it][1], v2 = v[it][2], v3 = v[it][3];
            if (!par) {
              v[it][0] = v0 * e[0] + v1 * e[2];
              v[it][1] = v0 * e[1] + v1 * e[3];
              v[it][2] = v2 * e[4] + v3 * e[6];
              v[it][3] = v2 * e[5] + v3 * e[7];
            } else {
              const double nxt0 = __shfl_down(v0, 1, 64);
              const double prv3 = __shfl_up(v3, 1, 64);
              v[it][0] = first ? v0 : prv3 * e[0] + v0 * e[1];
              v[it][1] = v1 * e[2] + v2 * e[4];
              v[it][2] = v1 * e[3] + v2 * e[5];
              v[it][3] = last ? v3 : v3 * e[6] + nxt0 * e[7];
            }
          }
        }
      }
      __syncthreads();
      if (a.prof && tid == 0) {
        // step profile (thread 0): cycles of phase A, cycles of phase B,
        // wall-clock ticks (100 MHz), steps, G-update cycles, V-update cycles
        const long long c2 = clock64();
        a.prof[0] += c1 - c0;
        a.prof[1] += c2 - c1;
        a.prof[2] += wall_clock64() - w0;
        a.prof[3] += 1;
        a.prof[4] += cmid - c1;
        a.prof[5] += c2 - cmid;
      }
    }
  }

  // ---------------------------------------------------------------- tail
  // rank the real positions by eigenvalue, descending; ties by label, descending
  for (int p = tid; p < L; p += kEigThreads) {
    int rk = -1;
    if (label[p] < l) {
      const double lp = G[pk(p, p, L)];
      rk = 0;
      for (int q = 0; q < L; ++q) {
        if (label[q] >= l || q == p) continue;
        const double lq = G[pk(q, q, L)];
        rk += (lq > lp) || (lq == lp && label[q] > label[p]);
      }
      const double lam = lp > 0.0 ? lp : 0.0;
      Ssh[rk] = sqrt(lam);
    }
    rank_of[p] = rk;
  }
  __syncthreads();
  const double tau = Ssh[0] * sqrt((double)l * 2.220446049250313e-16);
  for (int i = tid; i < l; i += kEigThreads) a.S[i] = Ssh[i];
#pragma unroll
  for (int it = 0; it < MAXNR; ++it) {
    const int row = wave * RPW + sub + it * row_stride;
    if (it < NR && active && row < l) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = 4 * cl + j;
        const int rk = rank_of[p];
        if (rk >= 0) {
          const double sv = Ssh[rk];
          a.W[(int64_t)row * l + rk] = sv > tau ? v[it][j] / sv : 0.0;
          if (a.Vs) a.Vs[(int64_t)row * l + rk] = v[it][j];
        }
      }
    }
  }
  if (a.sweeps && tid == 0) *a.sweeps = s_sweeps;
  if (!state) return;
  if (tid == 0) {
    state->eig_calls += 1;
    state->eig_sweeps += s_sweeps;
  }
  if (tid == 0 && !(Ssh[l - 1] > tau)) state->deficient = 1;
  if (a.mode != 2) return;

  // Alg. 5 steps 5-7 (power pass)
  __shared__ double s_ratio;
  __shared__ int s_stop;
  const double alpha = state->alpha;
  const int k = a.k;
  const int j = state->pass + 1;
  if (tid == 0) {
    double worst = 0.0;
    const double denom = Ssh[k] + alpha;
    const double ap = state->alpha_prev;
    for (int i = 0; i < k; ++i) {
      const double vv = fabs((a.Sprev[i] + ap) - (Ssh[i] + alpha)) / denom;
      if (vv > worst || vv != vv) worst = vv;
    }
    s_ratio = worst;
    s_stop = (a.tol > 0.0 && worst <= a.tol) ? 1 : 0;
  }
  __syncthreads();
  if (j - 1 < a.trace_cap) {
    for (int i = tid; i < l; i += kEigThreads) a.trace_s[(int64_t)(j - 1) * l + i] = Ssh[i];
  }
  if (!s_stop) {
    for (int i = tid; i < l; i += kEigThreads) a.Sprev[i] = Ssh[i];
  }
  if (tid == 0) {
    const double ratio = s_ratio;
    if (j - 1 < a.trace_cap) {
      a.trace_alpha[j - 1] = alpha;
      a.trace_ratio[j - 1] = ratio;
    }
    state->pass = j;
    state->ratio = ratio;
    if (s_stop) {
      state->done = 1;
      state->converged = 1;
    } else {
      double na = alpha;
      const double Sl = Ssh[l - 1];
      if (a.policy == 0) {  // PAPER
        if (Sl > alpha) na = 0.5 * (Sl + alpha);
      } else if (a.policy == 2) {  // FIXED
        if (j == 1 && Sl > alpha) na = 0.5 * (Sl + alpha);
      } else if (a.policy == 3 || a.policy == 4) {  // SCHEDULE / LEARNED
        const double El = Sl + alpha, Ek1 = Ssh[k] + alpha;
        if (j >= 2 && (ratio > state->prev_ratio || Ek1 < state->prev_ek1)) state->sched_off = 1;
        const bool use = a.sched && !state->sched_off && j < a.sched_len;
        const double cmul = use ? a.sched[j] : 0.5;
        const double cand = cmul * El;
        if (cand > na) na = cand;
        state->prev_ek1 = Ek1;
      }
      state->prev_ratio = ratio;
      state->alpha_prev = a.pve_mode == 1 ? na : alpha;
      state->alpha = na;
    }
  }
}

}  // namespace

hipError_t launch_eig(const EigArgs &a, hipStream_t st) {
  if (a.l < 1 || a.l > kMaxLP) return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void *)k_eig<1>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    hipFuncSetAttribute((const void *)k_eig<2>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    hipFuncSetAttribute((const void *)k_eig<4>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    hipFuncSetAttribute((const void *)k_eig<kMaxNR>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    attr = true;
  }
  const int L = (a.l + 3) & ~3;
  const int LPR = L / 4, RPW = kWave / LPR;
  const int NR = (L + 16 * RPW - 1) / (16 * RPW);
  const size_t shm = sizeof(double) * (size_t)(L * (L + 1) / 2);
  if (NR <= 1)
    hipLaunchKernelGGL(k_eig<1>, dim3(1), dim3(kEigThreads), shm, st, a);
  else if (NR <= 2)
    hipLaunchKernelGGL(k_eig<2>, dim3(1), dim3(kEigThreads), shm, st, a);
  else if (NR <= 4)
    hipLaunchKernelGGL(k_eig<4>, dim3(1), dim3(kEigThreads), shm, st, a);
  else
    hipLaunchKernelGGL(k_eig<kMaxNR>, dim3(1), dim3(kEigThreads), shm, st, a);
  return hipGetLastError();
}

}  // namespace dsv
