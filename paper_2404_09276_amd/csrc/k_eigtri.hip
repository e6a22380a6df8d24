// Eigen-decomposition of the Gram matrix of an eigSVD block (Alg. 3 steps
// 1-4) through a symmetric tridiagonal form, in two kernels:
//   1. k_tri_reduce, one workgroup with G in registers (a TY x 16 thread
//      grid, cyclic: thread (ty, tx) holds rows ty + TY a and columns
//      tx + 16 b): Householder reduction G = H T H^T (Golub & Van Loan
//      Sec. 8.3.1).  Step p: the grid row holding row p forms the reflector
//      v of x = A(p, p+1:) and publishes it (barrier); every thread forms
//      its rows' part of A22 v, summed over its grid row by a DPP
//      reduce-scatter, and of v^T A22 v (barrier); then A22 -= v w^T + w v^T
//      with u = beta A22 v and w = u - (beta/2)(v^T u) v in registers.  The
//      reflectors, T (scaled by a power of two) and the Gershgorin interval
//      go to the workspace;
//   2. k_tri_vectors, one wave per eigenvalue, four a workgroup: the
//      eigenvalue by multisection of the Gershgorin interval on Sturm counts
//      (Sec. 8.4.1; 64 points a step, nine steps narrow the interval below
//      2^-54 of its width); a check that no other eigenvalue lies within
//      2^-30 ||T|| of it; its eigenvector from the twisted factorisation
//      T - lambda I = N_t Delta N_t^T at the twist index t where |gamma_t| is
//      smallest: z_t = 1 and two recurrences outward (one step of inverse
//      iteration from e_t; Dhillon and Parlett, Linear Algebra Appl. 387,
//      2004), normalised; then V = H z (the column in registers, the
//      reflectors staged through LDS for the workgroup, a wave-wide sum a
//      reflector), written to Vs and, divided by S, to W;
//   3. the workgroup of step 2 that finishes last: the columns of W where
//      S <= S_max sqrt(l eps) zeroed, and the pass tail (PVE check, shift
//      rule) for a power-pass block.
// S is sqrt(eig G) in descending order, as from the Jacobi kernels.
// Accuracy is normwise (an eigenvalue to about eps ||G||, an eigenvector to
// about eps ||G|| / gap), as with the paper's LAPACK eigensolver; the solver
// uses these kernels for the FP32 and BF16 forms, whose Jacobi threshold is
// 2^-23.  Where two eigenvalues lie within 2^-30 ||G|| of each other their
// vectors would not be orthogonal to that level, and a non-finite or zero G
// has no usable decomposition: the call then declines (*decline = 1, the
// solver state untouched) and the two-sided Jacobi kernel launched after it
// on the same stream runs.  l <= kTriMaxL.
#include <cstring>
#include <utility>

#include "common.h"
#include "lanes.h"
#include "pass_tail.h"

namespace dsv {

namespace {

constexpr int kVWaves = 4;  // waves (eigenvalues) of a vectors workgroup
constexpr int kVT = kVWaves * kWave;
constexpr int kZRows = (kTriMaxL + kWave - 1) / kWave;  // rows of a column a lane holds
constexpr int kSectPts = kWave;                           // points a multisection step
constexpr int kSectSteps = 9;                             // 65^9 > 2^54
constexpr double kPivMin = 0x1.0p-1000;

// workspace: scaled diagonal, off-diagonal and its squares, reflector
// coefficients (kTriMaxL each), then lo, hi, |T| bound and the exponent,
// two ints (the status and the arrival count of the vectors kernel), and
// the reflector rows
constexpr int kWsTd = 0, kWsTe = kTriMaxL, kWsTe2 = 2 * kTriMaxL, kWsBet = 3 * kTriMaxL, kWsHdr = 4 * kTriMaxL;
constexpr int kWsFlags = kWsHdr + 8;
constexpr int kWsRef = kWsHdr + 16;  // reflector rows, l x l
static_assert(8 * ((size_t)kWsRef + (size_t)kTriMaxL * kTriMaxL) <= kTriWsBytes, "workspace layout");
constexpr int kRefChunk = 8;                                       // reflector rows an LDS chunk
constexpr int kRefLoads = (kRefChunk * kTriMaxL + kVT - 1) / kVT;  // loads a thread a chunk
constexpr int kGo = 0, kDeclined = 1, kSkip = 2;

__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double guard(double q) { return fabs(q) < kPivMin ? -kPivMin : q; }

// sqrt(x) for x > 0: the hardware reciprocal square root refined by two
// Newton steps (near 1 ulp) in [2^-700, 2^700], the library's elsewhere
__device__ __forceinline__ double sqrt_fast(double x) {
  if (x > 0x1.0p-700 && x < 0x1.0p700) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return x * y;
  }
  return sqrt(x);
}

// Number of eigenvalues of the tridiagonal (d, off-diagonal squares e2) below
// x: the negative pivots of the LDL^T factorisation of T - x I, a pivot of
// magnitude below kPivMin taken as -kPivMin (T is scaled so that its entries
// are below 1).
__device__ __forceinline__ int sturm_count(const double *d, const double *e2, int n, double x) {
  double q = guard(d[0] - x);
  int c = q < 0.0 ? 1 : 0;
#pragma unroll 4
  for (int i = 1; i < n; ++i) {
    q = guard((d[i] - x) - e2[i - 1] * rcp_nr(q));
    c += q < 0.0 ? 1 : 0;
  }
  return c;
}

__device__ __forceinline__ double wave_max(double x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, kWave));
  return x;
}
__device__ __forceinline__ double wave_min(double x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x = fmin(x, __shfl_xor(x, o, kWave));
  return x;
}

// One halving level of a reduce-scatter inside a row of 16 lanes: lanes
// with bit B of the lane index clear keep the lower half of the N values,
// the others the upper half, and each adds the half its partner (the DPP
// permutation CTRL, which flips bit B and no bit already split) sent.
template <int N, int B, int CTRL>
__device__ __forceinline__ void rs_level(double *v, int lane) {
  const bool up = (lane >> B) & 1;
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const double send = up ? v[i] : v[i + N / 2];
    const double keep = up ? v[i + N / 2] : v[i];
    v[i] = keep + lanes_dpp<CTRL>(send);
  }
}

// Each of the NV values (NV a power of two <= 16) summed over the 16 lanes
// of a DPP row: lane j of the row ends with the sum of value j >> (4 -
// log2 NV).  Bits 3, 2, 1, 0 of the lane index are split in that order by
// the row mirror (lane ^ 15), half mirror (^ 7), ^ 2 and ^ 1, as long as
// values remain to split, and summed plainly after.
template <int NV>
__device__ __forceinline__ double row_reduce_scatter(double (&v)[NV], int lane) {
  static_assert(NV == 1 || NV == 2 || NV == 4 || NV == 8 || NV == 16, "NV");
  if constexpr (NV >= 2) rs_level<NV, 3, 0x140>(v, lane); else v[0] += lanes_dpp<0x140>(v[0]);
  if constexpr (NV >= 4) rs_level<NV / 2, 2, 0x141>(v, lane); else v[0] += lanes_dpp<0x141>(v[0]);
  if constexpr (NV >= 8) rs_level<NV / 4, 1, 0x4E>(v, lane); else v[0] += lanes_dpp<0x4E>(v[0]);
  if constexpr (NV >= 16) rs_level<NV / 8, 0, 0xB1>(v, lane); else v[0] += lanes_dpp<0xB1>(v[0]);
  return v[0];
}

constexpr int log2c(int n) { return n <= 1 ? 0 : 1 + log2c(n / 2); }

// f(integral_constant<int, K>) for K = 0, 1, ..., in order, each expanded
// at compile time
template <class F, int... Ks>
__device__ __forceinline__ void for_each_const(F &&f, std::integer_sequence<int, Ks...>) {
  (f(std::integral_constant<int, Ks>{}), ...);
}
constexpr int pow2ceil(int n) { return n <= 1 ? 1 : 2 * pow2ceil((n + 1) / 2); }

// Householder reduction by a TY x 16 thread grid: thread (ty, tx) holds
// rows ty + TY a (a < RR) and columns tx + 16 b (b < RC) of G, so that
// the 16 threads of a row of the grid are one DPP row of lanes.
template <int TY, int RR, int RC>
__global__ __launch_bounds__(TY * 16) void k_tri_reduce(EigArgs a) {
  constexpr int TX = 16;
  constexpr int NT = TY * TX, NWv = NT / kWave, TYW = kWave / TX;  // rows of the grid a wave holds
  constexpr int NV = pow2ceil(RR), SPL = log2c(NV);
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // scalar: uniform branches
  const int ty = tid / TX, tx = tid % TX;
  double *ws = a.tri_ws;
  int32_t *flags = reinterpret_cast<int32_t *>(ws + kWsFlags);
  if ((a.run_if && *a.run_if == 0) || (a.skip_if && *a.skip_if)) {
    if (tid == 0) {
      flags[0] = kSkip;
      *a.decline = 0;
    }
    return;
  }
  SolverState *state = a.state;
  if (state && a.call_idx > 0 && tid == 0) signal_started(&state->eig_started, a.call_idx);
  if (state && a.mode == 2) {
    const int stopped = state->done;
    __syncthreads();
    if (tid == 0) state->skip_rescale = stopped;
    if (stopped) {
      if (tid == 0) {
        flags[0] = kSkip;
        *a.decline = 0;
      }
      return;
    }
  }
  const long long t0 = a.prof ? (long long)clock64() : 0;
  long long c1 = 0, c2 = 0;  // profile: cycles to the end of phase 1 and of phase 2, summed
  const int l = a.l;
  constexpr int LR = TY * RR, LC = TX * RC;  // rows and columns the grid covers
  static_assert(LR == LC, "square tiles");
  __shared__ double vb[2][LC];   // reflector of the step (double-buffered by step parity)
  __shared__ double xrow[LC];    // row p, from its holders
  __shared__ double ub[LR];      // u = beta A22 v
  __shared__ double part[NWv];   // partial sums of v^T A22 v
  __shared__ double sbeta[2];
  __shared__ double dd[LR], ee[LR], bl[LR];
  // reflector of step p: entries p+1 .. l-1 from rf[p (2 LC - p - 1) / 2]
  // (the rows of the strict upper triangle, packed), copied out at the end
  __shared__ double rf[LC * (LC - 1) / 2];

  double A[RR][RC];
  int bad = 0;
#pragma unroll
  for (int i0 = 0; i0 < RR; ++i0)
#pragma unroll
    for (int c0 = 0; c0 < RC; ++c0) {
      const int i = ty + TY * i0, c = tx + TX * c0;
      const double g = (i < l && c < l) ? a.G[(size_t)i * l + c] : 0.0;
      if (!(fabs(g) < INFINITY)) bad = 1;
      A[i0][c0] = g;
    }
  if (__syncthreads_or(bad)) {
    if (tid == 0) {
      flags[0] = kDeclined;
      *a.decline = 1;
    }
    return;
  }

  // Step p = k TY + j: row p is row k of the tiles of grid row j.  Each k
  // is a block of code of its own, so that the register row and the tile
  // bounds below are constants.
  auto block = [&](auto kc) __attribute__((always_inline)) {
    constexpr int k = decltype(kc)::value;
    for (int j = 0; j < TY; ++j) {
      const int p = k * TY + j;
      if (p + 2 >= l) break;
      const int buf = p & 1;
      const long long ta = a.prof ? (long long)clock64() : 0;
      if (wave == j / TYW) {
        // grid row j (one DPP row of this wave) forms the reflector of
        // x = A(p, p+1:); the whole wave runs the cross-lane sum
        double sq = 0.0;
        if (ty == j) {
#pragma unroll
          for (int c0 = 0; c0 < RC; ++c0) {
            const int c = tx + TX * c0;
            xrow[c] = A[k][c0];
            if (c > p + 1) sq = fma(A[k][c0], A[k][c0], sq);
          }
        }
        lanes_wave_sync();
        double sv[1] = {sq};
        sq = row_reduce_scatter<1>(sv, lane);
        const double x0 = xrow[p + 1], app = xrow[p];
        double alpha = x0, v0 = 0.0, beta = 0.0;
        if (sq > 0.0) {
          const double nrm = sqrt_fast(fma(x0, x0, sq));
          alpha = x0 >= 0.0 ? -nrm : nrm;
          v0 = x0 - alpha;  // no cancellation: x0 and -alpha share the sign
          const double vv = fma(v0, v0, sq);
          beta = vv > 0x1.0p-1000 && vv < 0x1.0p1000 ? 2.0 * rcp_nr(vv) : 2.0 / vv;
        }
        if (ty == j) {
#pragma unroll
          for (int c0 = 0; c0 < RC; ++c0) {
            const int c = tx + TX * c0;
            const double v = beta == 0.0 ? 0.0 : (c == p + 1 ? v0 : (c > p + 1 ? A[k][c0] : 0.0));
            vb[buf][c] = v;
            if (c > p && c < l) rf[p * (2 * LC - p - 1) / 2 + (c - p - 1)] = v;
          }
          if (tx == 0) {
            dd[p] = app;
            ee[p] = alpha;
            sbeta[buf] = beta;
            bl[p] = beta;
          }
        }
      }
      __syncthreads();
      const long long tb = a.prof ? (long long)clock64() : 0;
      c1 += tb - ta;
      const double beta = sbeta[buf];
      // tiles of rows below k and of columns below C0 lie wholly at or above
      // row p, or at or left of column p (p >= TY k): the loops start past
      // them (bounds known once the loop over k is unrolled)
      const int C0 = (TY * k) / TX;
      double vr[RR], vc[RC], t[NV];
#pragma unroll
      for (int i0 = k; i0 < RR; ++i0) vr[i0] = vb[buf][ty + TY * i0];
#pragma unroll
      for (int c0 = C0; c0 < RC; ++c0) vc[c0] = vb[buf][tx + TX * c0];
      if (beta == 0.0) continue;  // H = I (uniform)
      double kp = 0.0;
#pragma unroll
      for (int i0 = 0; i0 < NV; ++i0) {
        double s = 0.0;
        if (i0 >= k && i0 < RR) {
#pragma unroll
          for (int c0 = C0; c0 < RC; ++c0) s = fma(A[i0 < RR ? i0 : 0][c0], vc[c0], s);
          kp = fma(vr[i0 < RR ? i0 : 0], s, kp);
        }
        t[i0] = s;
      }
      // u for row ty + TY (tx >> (4 - SPL)), held by every lane whose low
      // 4 - SPL bits are zero
      const double us = row_reduce_scatter<NV>(t, lane);
      {
        const int ai = tx >> (4 - SPL);
        const int i = ty + TY * ai;
        if ((tx & ((1 << (4 - SPL)) - 1)) == 0 && ai < RR) ub[i] = i > p ? beta * us : 0.0;
      }
      kp = lanes_wave_sum(kp);
      if (lane == 0) part[wave] = kp;
      __syncthreads();
      if (a.prof) c2 += (long long)clock64() - tb;
      double ksum = 0.0;
#pragma unroll
      for (int w = 0; w < NWv; ++w) ksum += part[w];
      // K = (beta / 2) v^T u with u = beta A22 v
      const double K = 0.5 * beta * beta * ksum;
      double wc[RC], wr[RR];
#pragma unroll
      for (int c0 = C0; c0 < RC; ++c0) wc[c0] = fma(-K, vc[c0], ub[tx + TX * c0]);
#pragma unroll
      for (int i0 = k; i0 < RR; ++i0) wr[i0] = fma(-K, vr[i0], ub[ty + TY * i0]);
#pragma unroll
      for (int i0 = k; i0 < RR; ++i0)
#pragma unroll
        for (int c0 = C0; c0 < RC; ++c0) A[i0][c0] = fma(-vr[i0], wc[c0], fma(-wr[i0], vc[c0], A[i0][c0]));
    }
  };
  for_each_const(block, std::make_integer_sequence<int, RR>{});
  // the last 2 x 2 block (1 x 1 for l = 1)
#pragma unroll
  for (int i0 = 0; i0 < RR; ++i0)
#pragma unroll
    for (int c0 = 0; c0 < RC; ++c0) {
      const int i = ty + TY * i0, c = tx + TX * c0;
      if (i < l && i >= l - 2 && c == i) dd[i] = A[i0][c0];
      if (l >= 2 && i == l - 1 && c == l - 2) ee[l - 2] = A[i0][c0];
    }
  __syncthreads();
  // the reflector rows (zero at and left of the diagonal) and coefficients
  // to the workspace
  {
    // rows of LC columns, NT / LC of them at a time (TX divides both)
    constexpr int RPI = NT / LC > 0 ? NT / LC : 1;
    const int c = tid % LC;
    for (int p = tid / LC; p + 2 < l; p += RPI)
      if (c < l && tid < RPI * LC) ws[kWsRef + (size_t)p * l + c] = c > p ? rf[p * (2 * LC - p - 1) / 2 + (c - p - 1)] : 0.0;
  }
  for (int p = tid; p + 2 < l; p += NT) ws[kWsBet + p] = bl[p];
  if (a.prof && tid == 0) {
    a.prof[0] = (long long)clock64() - t0;
    a.prof[6] = c1;
    a.prof[7] = c2;
  }
  if (wave != 0) return;
  // T scaled by a power of two so that its largest entry lies in [1/2, 1),
  // and the Gershgorin interval of the scaled T
  double mx = 0.0;
  for (int i = lane; i < l; i += kWave) {
    mx = fmax(mx, fabs(dd[i]));
    if (i + 1 < l) mx = fmax(mx, fabs(ee[i]));
  }
  mx = wave_max(mx);
  const bool ok = mx > 0.0 && mx < INFINITY;
  int ex = 0;
  if (ok) (void)frexp(mx, &ex);
  double lo = INFINITY, hi = -INFINITY;
  for (int i = lane; i < l; i += kWave) {
    const double di = ldexp(dd[i], -ex);
    const double em = i > 0 ? ldexp(ee[i - 1], -ex) : 0.0;
    const double ep = i + 1 < l ? ldexp(ee[i], -ex) : 0.0;
    ws[kWsTd + i] = di;
    if (i + 1 < l) {
      ws[kWsTe + i] = ep;
      ws[kWsTe2 + i] = ep * ep;
    }
    const double rad = fabs(em) + fabs(ep);
    lo = fmin(lo, di - rad);
    hi = fmax(hi, di + rad);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  if (lane == 0) {
    const double big = fmax(fabs(lo), fabs(hi));
    // widened by 2^-40 of its magnitude, well above the rounding of the counts
    ws[kWsHdr + 0] = lo - 0x1.0p-40 * big;
    ws[kWsHdr + 1] = hi + 0x1.0p-40 * big;
    ws[kWsHdr + 2] = big;
    ws[kWsHdr + 3] = (double)ex;
    flags[1] = 0;  // arrivals of the vectors kernel
    flags[0] = ok ? kGo : kDeclined;
    *a.decline = ok ? 0 : 1;
  }
}

__global__ __launch_bounds__(kVT) void k_tri_vectors(EigArgs a) {
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  const double *ws = a.tri_ws;
  int32_t *flags = reinterpret_cast<int32_t *>(a.tri_ws + kWsFlags);
  if (flags[0] != kGo) return;  // declined or skipped by the reduction
  const int l = a.l;
  __shared__ double td[kTriMaxL], te[kTriMaxL], te2[kTriMaxL], bet[kTriMaxL];
  __shared__ double dp[kVWaves][kTriMaxL], dm[kVWaves][kTriMaxL], zz[kVWaves][kTriMaxL];
  __shared__ double refl[2][kRefChunk][kTriMaxL];  // reflector rows, double-buffered chunks
  for (int i = tid; i < l; i += kVT) {
    td[i] = ws[kWsTd + i];
    bet[i] = i + 2 < l ? ws[kWsBet + i] : 0.0;
    te[i] = i + 1 < l ? ws[kWsTe + i] : 0.0;
    te2[i] = i + 1 < l ? ws[kWsTe2 + i] : 0.0;
  }
  const double lo = ws[kWsHdr + 0], hi = ws[kWsHdr + 1], big = ws[kWsHdr + 2];
  const int ex = (int)ws[kWsHdr + 3];
  __syncthreads();

  const int r = blockIdx.x * kVWaves + wv;  // eigenvalue (ascending) of this wave
  // optional phase profile: cycles of wave 0 of workgroup 0
  const bool stamp = a.prof && blockIdx.x == 0 && tid == 0;
  long long ts = stamp ? (long long)clock64() : 0;
  auto mark = [&](int slot) {
    if (stamp) {
      const long long now = (long long)clock64();
      a.prof[slot] = now - ts;
      ts = now;
    }
  };
  bool act = false;  // this wave has an isolated eigenvalue and its z (wave-uniform)
  double lam = 0.0;
  double zr[kZRows];
#pragma unroll
  for (int s = 0; s < kZRows; ++s) zr[s] = 0.0;
  if (r < l) {
    // multisection: count(lo_r) <= r < count(hi_r); lane z evaluates point
    // z + 1 of 65, the new interval is between the last point whose count
    // is <= r below the first point whose count passes r
    constexpr double kStep = 1.0 / (double)(kSectPts + 1);
    double lo_r = lo, hi_r = hi;
    for (int it = 0; it < kSectSteps; ++it) {
      const double w = hi_r - lo_r;
      const double x = fma(w, (double)(lane + 1) * kStep, lo_r);
      const int c = sturm_count(td, te2, l, x);
      const unsigned long long above = __ballot(c > r);
      const int first = above ? __builtin_ctzll(above) : kWave;
      const unsigned long long low = first >= kWave ? ~0ull : ((1ull << first) - 1ull);
      const unsigned long long below = __ballot(c <= r) & low;
      const int lastb = below ? 63 - __builtin_clzll(below) : -1;
      const double nhi = first < kWave ? fma(w, (double)(first + 1) * kStep, lo_r) : hi_r;
      const double nlo = lastb >= 0 ? fma(w, (double)(lastb + 1) * kStep, lo_r) : lo_r;
      lo_r = nlo;
      hi_r = nhi;
    }
    lam = 0.5 * (lo_r + hi_r);
    mark(1);
    // isolation: exactly r eigenvalues below lam - d and r + 1 below lam + d
    const double dl = 0x1.0p-30 * big;
    const int cc = sturm_count(td, te2, l, (lane & 1) ? lam + dl : lam - dl);
    bool iso = __shfl(cc, 0, kWave) == r && __shfl(cc, 1, kWave) == r + 1;
    mark(2);
    double *dpw = dp[wv], *dmw = dm[wv], *zw = zz[wv];
    int t = 0;
    if (iso) {
      // D+ forward (lane 0) and D- backward (lane 1)
      if (lane < 2) {
        const bool fw = lane == 0;
        double *dst = fw ? dpw : dmw;
        int i = fw ? 0 : l - 1;
        double q = guard(td[i] - lam);
        dst[i] = q;
        for (int k = 1; k < l; ++k) {
          i = fw ? k : l - 1 - k;
          const double e2 = te2[fw ? i - 1 : i];
          q = guard((td[i] - lam) - e2 * rcp_nr(q));
          dst[i] = q;
        }
      }
      lanes_wave_sync();
      // twist: the smallest |gamma_i|, gamma_i = D+_i + D-_i - (d_i - lambda)
      double best = INFINITY;
      t = 0x7fffffff;
#pragma unroll
      for (int s = 0; s < kZRows; ++s) {
        const int i = lane + kWave * s;
        if (i < l) {
          const double g = fabs(dpw[i] + dmw[i] - (td[i] - lam));
          if (g < best) {
            best = g;
            t = i;
          }
        }
      }
#pragma unroll
      for (int o = kWave / 2; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, kWave);
        const int ot = __shfl_xor(t, o, kWave);
        if (ob < best || (ob == best && ot < t)) {
          best = ob;
          t = ot;
        }
      }
      iso = t < l;
    }
    if (iso) {
      // z_t = 1, then z_i = -(e_i / D+_i) z_(i+1) below t (lane 0) and
      // z_i = -(e_(i-1) / D-_i) z_(i-1) above t (lane 1)
      if (lane < 2) {
        const bool dn = lane == 0;
        const int cnt = dn ? t : l - 1 - t;
        double z = 1.0;
        if (dn) zw[t] = 1.0;
        for (int k = 1; k <= cnt; ++k) {
          const int i = dn ? t - k : t + k;
          const double num = te[dn ? i : i - 1];
          const double den = dn ? dpw[i] : dmw[i];
          z = -(num * rcp_nr(den)) * z;
          zw[i] = z;
        }
      }
      lanes_wave_sync();
      double nz = 0.0;
#pragma unroll
      for (int s = 0; s < kZRows; ++s) {
        const int i = lane + kWave * s;
        zr[s] = i < l ? zw[i] : 0.0;
        nz = fma(zr[s], zr[s], nz);
      }
      nz = lanes_wave_sum(nz);
      const double inv = 1.0 / sqrt(nz);
#pragma unroll
      for (int s = 0; s < kZRows; ++s) zr[s] *= inv;
      act = true;
      mark(3);
    } else if (lane == 0) {
      __hip_atomic_store(a.decline, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }

  // V = H_0 H_1 ... H_(l-3) z.  The reflector rows (zero at and left of the
  // diagonal, all zero where beta_p = 0) pass through LDS in chunks of
  // kRefChunk rows, p descending, loaded by the whole workgroup one chunk
  // ahead; every wave takes part in the loads and barriers.
  {
    const double *Rf = ws + kWsRef;
    const int np = l > 2 ? l - 2 : 0;  // reflectors 0 .. l-3
    const int nch = (np + kRefChunk - 1) / kRefChunk;
    const int per = kRefChunk * l;  // doubles a chunk
    int es[kRefLoads], ei[kRefLoads];  // (row of the chunk, column) of this thread's loads
#pragma unroll
    for (int q = 0; q < kRefLoads; ++q) {
      const int e = tid + kVT * q;
      es[q] = e < per ? e / l : kRefChunk;
      ei[q] = e < per ? e - es[q] * l : 0;
    }
    double reg[kRefLoads];
    auto chunk_load = [&](int c) {
#pragma unroll
      for (int q = 0; q < kRefLoads; ++q) {
        const int p = l - 3 - kRefChunk * c - es[q];
        reg[q] = (es[q] < kRefChunk && p >= 0) ? Rf[(size_t)p * l + ei[q]] : 0.0;
      }
    };
    auto chunk_store = [&](int b) {
#pragma unroll
      for (int q = 0; q < kRefLoads; ++q)
        if (es[q] < kRefChunk) refl[b][es[q]][ei[q]] = reg[q];
    };
    if (nch > 0) {
      chunk_load(0);
      chunk_store(0);
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      if (c + 1 < nch) chunk_load(c + 1);
      if (act) {
        const int rows = min(kRefChunk, np - kRefChunk * c);
#pragma unroll
        for (int s = 0; s < kRefChunk; ++s) {
          if (s < rows) {
            const int p = l - 3 - kRefChunk * c - s;
            const double *vp = refl[c & 1][s];
            double vv[kZRows];
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < kZRows; ++k) {
              const int i = lane + kWave * k;
              vv[k] = i < l ? vp[i] : 0.0;
              sum = fma(vv[k], zr[k], sum);
            }
            sum = lanes_wave_sum(sum) * bet[p];
#pragma unroll
            for (int k = 0; k < kZRows; ++k) zr[k] = fma(-vv[k], sum, zr[k]);
          }
        }
      }
      if (c + 1 < nch) chunk_store((c + 1) & 1);
      __syncthreads();
    }
  }
  if (act) {
    mark(4);
    const int rk = l - 1 - r;
    const double sv = sqrt(fmax(ldexp(lam, ex), 0.0));
    const double iv = 1.0 / sv;  // columns with S <= S_max sqrt(l eps) are zeroed below
#pragma unroll
    for (int s = 0; s < kZRows; ++s) {
      const int i = lane + kWave * s;
      if (i < l) {
        a.Vs[(size_t)i * l + rk] = zr[s];
        a.W[(size_t)i * l + rk] = zr[s] * iv;
      }
    }
    if (lane == 0) a.S[rk] = sv;
  }

  // ------------------------------------------------------------ the last workgroup
  __threadfence();
  __syncthreads();
  __shared__ int s_last;
  if (tid == 0) s_last = atomicAdd(&flags[1], 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const long long tt = a.prof ? (long long)clock64() : 0;
  if (tid == 0) flags[1] = 0;
  if (__hip_atomic_load(a.decline, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  __shared__ double Ssh[kTriMaxL];
  for (int i = tid; i < l; i += kVT) Ssh[i] = a.S[i];
  __syncthreads();
  const double tau = Ssh[0] * sqrt((double)l * 2.220446049250313e-16);
  for (int c = wv; c < l; c += kVWaves)
    if (!(Ssh[c] > tau))
      for (int i = lane; i < l; i += kWave) a.W[(size_t)i * l + c] = 0.0;
  if (a.sweeps && tid == 0) *a.sweeps = 0;
  if (a.prof && tid == 0) a.prof[5] = (long long)clock64() - tt;
  SolverState *state = a.state;
  if (!state) return;
  if (tid == 0) {
    if (a.trace_sweeps && state->eig_calls < a.trace_cap + 2) a.trace_sweeps[state->eig_calls] = 0;
    state->eig_calls += 1;
    if (!(Ssh[l - 1] > tau)) state->deficient = 1;
  }
  if (a.mode != 2) return;
  __syncthreads();
  pass_tail(a, state, Ssh);
}

template <int TY, int RR, int RC>
hipError_t launch_reduce(const EigArgs &a, hipStream_t st) {
  hipLaunchKernelGGL((k_tri_reduce<TY, RR, RC>), dim3(1), dim3(TY * 16), 0, st, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eigtri(const EigArgs &a, hipStream_t st) {
  if (a.l < 1 || a.l > kTriMaxL || !a.Vs || !a.W || !a.S || !a.decline || !a.tri_ws) return hipErrorInvalidValue;
  // one wave a SIMD up to l = 128 (tiles of up to 8 x 8 a thread), two above
  hipError_t e;
  if (a.l <= 32)
    e = launch_reduce<16, 2, 2>(a, st);
  else if (a.l <= 64)
    e = launch_reduce<16, 4, 4>(a, st);
  else if (a.l <= 96)
    e = launch_reduce<16, 6, 6>(a, st);
  else if (a.l <= 128)
    e = launch_reduce<16, 8, 8>(a, st);
  else
    e = launch_reduce<32, 5, 10>(a, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tri_vectors, dim3((a.l + kVWaves - 1) / kVWaves), dim3(kVT), 0, st, a);
  return hipGetLastError();
}

}  // namespace dsv
