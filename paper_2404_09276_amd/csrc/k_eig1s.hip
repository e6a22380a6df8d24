// Eigen-decomposition of the Gram matrix of an eigSVD block (Alg. 3 steps
// 1-4) by one-sided Jacobi on its Cholesky factor, in one workgroup with the
// matrix held in registers.
//
// Method.  G = R^T R (Cholesky, FP64).  One-sided (Hestenes) Jacobi
// rotations J make the columns of X = R^T mutually orthogonal: X J = V Sig.
// Then G (X J) = R^T (R R^T) J = (X J) Sig^2, so the columns of X J are
// eigenvectors of G scaled by the square roots of its eigenvalues:
//   S = column norms of X J (= sqrt(eig G), the singular values of the
//   block), Vs = (X J) S^-1, W = Vs S^-1 = (X J) S^-2,
// and J itself is never formed.  A rotation of columns (p, q) with
// a = |x_p|^2, b = |x_q|^2, c = x_p . x_q is the Jacobi rotation of the
// 2x2 matrix [[a, c], [c, b]] (Golub & Van Loan Sec. 8.5 / 8.6.3); it is
// skipped when |c| <= tol sqrt(a b), and the sweeps stop after one in which
// every pair was skipped.  X^T X = R R^T is closer to diagonal than G is
// (one step of the LR iteration), so fewer sweeps are needed than by the
// two-sided method on G (Drmac and Veselic, SIAM J. Matrix Anal. Appl. 29,
// 2008), and a rotation touches two columns of X only.
//
// Ordering: parallel cyclic with the odd-even (Luk-Park) pairing of
// positions: even steps pair (2g, 2g+1), odd steps (2g+1, 2g+2), and every
// rotation is followed by a swap of the two columns, so L steps (L even)
// meet every pair once (one sweep).  The swap is free: the rotated columns
// are written to each other's position.
//
// Placement (NW waves, L = C NW padded size, P = C / 2):
//   - wave w holds the columns of a window of C + 1 register slots; on even
//     steps slots 0..C-1 are positions wC .. wC+C-1, on odd steps slots
//     1..C are positions wC+1 .. wC+C, so each step pairs P columns inside
//     every wave.  Between steps one column moves to a neighbouring wave
//     through LDS (one barrier a step);
//   - lane i of a wave holds rows i, i + 64, ... (NRW of them) of every
//     column of its window;
//   - the P dot products of a step are summed over the wave by a
//     reduce-scatter (DPP butterflies on the low lane bits, so that lane i
//     ends with the full dot of pair i mod P), the lanes then compute the
//     P rotations at once, and publish them through LDS;
//   - the squared column norms live in LDS by position; they are updated
//     with each rotation (a' = a - t c, b' = b + t c) and recomputed from
//     the columns at the start of every sweep;
//   - every pair swaps at every step (a skipped rotation is a plain swap),
//     so a sweep reverses the positions whatever the data: after s sweeps
//     position p holds the column that started at p (s even) or L-1-p
//     (s odd), which tells the padding columns apart at the end.
// Cholesky: right-looking by panels of C columns: wave w factors its own
// columns (after the updates of the panels before), publishes them through
// LDS, and the waves to its right apply them (one barrier a panel).  A
// non-positive or non-finite pivot (G singular to working precision) makes
// the call decline: *decline is set and nothing else is written; the
// two-sided Jacobi kernel launched after it on the same stream then runs.
//
// Tail: as the two-sided kernel: S descending (ties by label, descending),
// W = Vs diag(1/S) with columns zeroed where S <= S_max sqrt(l eps), the
// pass tail (PVE check, shift rule) for a power-pass block.
#include <cstring>

#include "common.h"
#include "pass_tail.h"

namespace dsv {

namespace {

constexpr int kJ1MaxSweeps = 60;

template <int N>
struct IC1 {
  static constexpr int value = N;
};

// Reciprocal and reciprocal square root: the hardware approximations refined
// by two Newton steps (relative error near 1 ulp).
__device__ __forceinline__ double rcp2(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt2(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// Value of lane `src` of the wave (src wave-uniform).
__device__ __forceinline__ double readlane_d(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// DPP lane permutations (both halves of a double):
//   0xB1 quad_perm [1,0,3,2]: lane ^ 1      0x4E quad_perm [2,3,0,1]: lane ^ 2
//   0x141 row_half_mirror:    lane ^ 7      0x140 row_mirror:         lane ^ 15
//   0x124 row_ror 4, 0x128 row_ror 8 (rotations inside rows of 16 lanes)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// One halving level of the reduce-scatter: lanes with bit B of the lane
// index clear keep the lower half of the N values, the others the upper
// half; each adds the half its partner (the DPP permutation CTRL, which
// flips bit B and no bit already split) sent.
template <int N, int B, int CTRL>
__device__ __forceinline__ void rs_level(double (&v)[16], int lane) {
  const bool up = (lane >> B) & 1;
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const double send = up ? v[i] : v[i + N / 2];
    const double keep = up ? v[i + N / 2] : v[i];
    v[i] = keep + dpp_d<CTRL>(send);
  }
}

// x + (x of lane ^ 16) and x + (x of lane ^ 32): the gfx950 row-pair and
// half swaps (VALU, no LDS) exchange the operands between the two rows /
// halves, so the two results hold the value of each lane of the pair and
// their sum is the same on both.
__device__ __forceinline__ double add_xor16(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const auto l2 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h2 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double u = __longlong_as_double(((long long)(unsigned)l2[0]) | ((long long)h2[0] << 32));
  const double v = __longlong_as_double(((long long)(unsigned)l2[1]) | ((long long)h2[1] << 32));
  return u + v;
}
__device__ __forceinline__ double add_xor32(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const auto l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double u = __longlong_as_double(((long long)(unsigned)l2[0]) | ((long long)h2[0] << 32));
  const double v = __longlong_as_double(((long long)(unsigned)l2[1]) | ((long long)h2[1] << 32));
  return u + v;
}

// Sum over the 64 lanes of each of N values (N = 2, 4, 8 or 16), scattered:
// lane i returns the sum of value i mod N.  The halving levels split on lane
// bits log2(N)-1 .. 0 (the permutations flip bits {0..3}, {0..2}, {1}, {0}:
// independent over GF(2), so every lane's partial sums come from disjoint
// lanes); the remaining bits are summed by rotations inside rows and by
// swaps across rows and halves.
template <int N>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[16], int lane) {
  static_assert(N == 2 || N == 4 || N == 8 || N == 16, "N");
  if constexpr (N == 16) rs_level<16, 3, 0x140>(v, lane);
  if constexpr (N >= 8) rs_level<8, 2, 0x141>(v, lane);
  if constexpr (N >= 4) rs_level<4, 1, 0x4E>(v, lane);
  rs_level<2, 0, 0xB1>(v, lane);
  double x = v[0];
  if constexpr (N == 2) x += dpp_d<0x4E>(x);  // bit 1
  if constexpr (N <= 4) x += dpp_d<0x124>(x);  // bits 2, 3 (with the next)
  if constexpr (N <= 8) x += dpp_d<0x128>(x);  // bit 3
  x = add_xor16(x);
  return add_xor32(x);
}

template <int NRW>
__device__ __forceinline__ double pick(const double (&v)[NRW], int r) {
  double o = v[0];
#pragma unroll
  for (int i = 1; i < NRW; ++i)
    if (r == i) o = v[i];
  return o;
}

// C: columns per wave (even, C/2 pairs a step); NW: waves; NRW: rows per lane
// (64 NRW >= L = C NW).  BATCHED: workgroup b solves arr[b].
constexpr int pow2_ceil(int x) { return x <= 1 ? 1 : 2 * pow2_ceil((x + 1) / 2); }

template <int C, int NW, int NRW, bool BATCHED>
__global__ __launch_bounds__(NW * 64) void k_eig1s(EigArgs a0, const EigArgs *__restrict__ arr) {
  constexpr int P = C / 2;
  constexpr int NP = pow2_ceil(P);  // the reduce-scatter's width (pairs P..NP-1 are empty)
  constexpr int L = C * NW;
  constexpr int NT = NW * 64;
  constexpr int R = NRW * 64;  // rows held per column (>= L)
  static_assert(R >= L && C % 4 == 0 && NP <= 16, "layout");
  const EigArgs &a = BATCHED ? arr[blockIdx.x] : a0;
  if ((a.run_if && *a.run_if == 0) || (a.skip_if && *a.skip_if)) {
    // gated off: nothing for the two-sided kernel after it to do either
    if (threadIdx.x == 0 && a.decline) *a.decline = 0;
    return;
  }
  SolverState *state = a.state;
  if (!BATCHED && state && a.call_idx > 0 && threadIdx.x == 0) signal_started(&state->eig_started, a.call_idx);
  if (state && a.mode == 2) {
    // a pass launched after the check already passed: nothing to do, and
    // its rescale must not run either
    const int stopped = state->done;
    __syncthreads();
    if (threadIdx.x == 0) state->skip_rescale = stopped;
    if (stopped) {
      if (threadIdx.x == 0 && a.decline) *a.decline = 0;
      return;
    }
  }
  // LDS: the panels of the Cholesky phase and the column exchange of the
  // Jacobi phase share the dynamic buffer (2 C R doubles)
  extern __shared__ double dyn[];
  __shared__ double nrm[L + 1];
  __shared__ double2 rot[NW][P];
  __shared__ double Ssh[kTailMaxL];
  __shared__ int rank_of[L];
  __shared__ int s_fail;
  // whether any wave rotated in the sweep, by sweep parity (a flag is
  // cleared one barrier after its last read)
  __shared__ int s_rot[2];

  const int l = a.l;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // below the rounding of a dot product of L terms the rotations would not end
  const double tol = fmax(a.skip, (double)L * 0x1.0p-53);
  const bool fast_angle = tol >= 0x1.0p-30;

  // window slots 0..C-1: columns wC .. wC+C-1 of G; slot C: the column
  // received on odd steps
  double x[C + 1][NRW];
#pragma unroll
  for (int c = 0; c <= C; ++c) {
    const int j = wave * C + c;
#pragma unroll
    for (int r = 0; r < NRW; ++r) {
      const int row = lane + 64 * r;
      // G is symmetric: column j read as row j (consecutive lanes, consecutive words)
      x[c][r] = (c < C && j < l && row < l) ? a.G[(int64_t)j * l + row] : 0.0;
    }
  }
  if (tid == 0) s_fail = s_rot[0] = s_rot[1] = 0;

  // ------------------------------------------------------------ Cholesky
  const long long chol0 = (a.prof && tid == 0) ? clock64() : 0;
  for (int pw = 0; pw < NW; ++pw) {
    double *pan = dyn + (pw & 1) * (C * R);
    if (wave == pw) {
      // column c: pivot d (read from its lane), the multipliers
      // L(j2, j) = A(j2, j) / d of the panel's later columns (read from their
      // lanes before the column is scaled, so the chain to the next pivot
      // has no square root), their rank-1 updates with the unscaled column,
      // then the column scaled by d^-1/2
      bool ok = true;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int j = pw * C + c;
        if (ok && j < l) {
          const double d = readlane_d(pick(x[c], j >> 6), j & 63);
          if (!(d > 0.0) || !(d < INFINITY)) {
            ok = false;
          } else {
            const double rd = rcp2(d);
#pragma unroll
            for (int c2 = c + 1; c2 < C; ++c2) {
              const int j2 = pw * C + c2;
              const double lj = readlane_d(pick(x[c], j2 >> 6), j2 & 63) * rd;
#pragma unroll
              for (int r = 0; r < NRW; ++r) x[c2][r] = fma(-lj, x[c][r], x[c2][r]);
            }
            const double inv = rsqrt2(d);
#pragma unroll
            for (int r = 0; r < NRW; ++r) x[c][r] = (lane + 64 * r >= j) ? x[c][r] * inv : 0.0;
          }
        } else if (j >= l) {
          // a padding column
#pragma unroll
          for (int r = 0; r < NRW; ++r) x[c][r] = 0.0;
        }
      }
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int r = 0; r < NRW; ++r) pan[c * R + lane + 64 * r] = x[c][r];
      if (!ok && lane == 0) s_fail = 1;
    }
    __syncthreads();
    if (s_fail) break;
    if (wave > pw) {
#pragma unroll 1
      for (int c = 0; c < C; ++c) {
        double xr[NRW];
#pragma unroll
        for (int r = 0; r < NRW; ++r) xr[r] = pan[c * R + lane + 64 * r];
#pragma unroll
        for (int c2 = 0; c2 < C; ++c2) {
          const double lj = pan[c * R + wave * C + c2];
#pragma unroll
          for (int r = 0; r < NRW; ++r) x[c2][r] = fma(-lj, xr[r], x[c2][r]);
        }
      }
    }
  }
  if (s_fail) {
    // G is not positive definite to working precision: decline
    if (tid == 0 && a.decline) *a.decline = 1;
    return;
  }
  if (tid == 0 && a.decline) *a.decline = 0;
  if (a.prof && tid == 0) a.prof[5] += clock64() - chol0;
  // entries above the diagonal (left over from the updates) are not part of R^T
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int r = 0; r < NRW; ++r)
      if (lane + 64 * r < wave * C + c) x[c][r] = 0.0;

  // ------------------------------------------------------------ Jacobi
  if (tid == 0) nrm[L] = 0.0;
  double *xb = dyn;  // [2][NW][R]: the column a wave hands to a neighbour
  int sweeps = 0;    // sweeps that rotated
  int executed = 0;  // sweeps run (the last one may only confirm)

  // squared norms of the columns of the even window, by position (four
  // columns per reduce-scatter)
  auto norms = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int c0 = 0; c0 < C; c0 += 4) {
      double v[16];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double s = 0.0;
#pragma unroll
        for (int r = 0; r < NRW; ++r) s = fma(x[c0 + c][r], x[c0 + c][r], s);
        v[c] = s;
      }
      const double s = wave_reduce_scatter<4>(v, lane);
      if (lane < 4) nrm[wave * C + c0 + lane] = s;
    }
  };

  // one step of parity PAR (window offset PAR): returns whether this wave rotated
  // optional profile (thread 0's view): cycles of the dot products and their
  // reduction, of the rotation parameters, of the update, of the column
  // exchange with its barrier; steps; cycles of the Cholesky phase
  const bool prof = a.prof != nullptr && tid == 0;
  long long pc0 = 0, pacc[4] = {0, 0, 0, 0}, psteps = 0;
  auto stamp = [&](int slot) __attribute__((always_inline)) {
    if (prof) {
      const long long c = clock64();
      if (slot >= 0) pacc[slot] += c - pc0;
      pc0 = c;
    }
  };
  auto step = [&](auto par_c) __attribute__((always_inline)) -> bool {
    constexpr int o = decltype(par_c)::value;
    stamp(-1);
    double v[16];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double s = 0.0;
      if (i < P) {
#pragma unroll
        for (int r = 0; r < NRW; ++r) s = fma(x[o + 2 * i][r], x[o + 2 * i + 1][r], s);
      }
      v[i] = s;
    }
    // lanes of an empty pair (P <= pid < NP) work on pair P-1 and write nothing
    const int pid = (lane & (NP - 1)) < P ? (lane & (NP - 1)) : P - 1;
    const int p = wave * C + o + 2 * pid, q = p + 1;
    const double app = nrm[p], aqq = nrm[q];
    const double D = wave_reduce_scatter<NP>(v, lane);
    if (prof) (void)__builtin_amdgcn_readfirstlane(__double2hiint(D));
    stamp(0);
    double cs = 1.0, sn = 0.0, tD = 0.0;
    bool rotd = false;
    if (q >= L) {
      // the last wave's odd-step partner is past the end: keep x_p
      cs = 0.0;
      sn = 1.0;
    } else if (D != 0.0 && !(D * D <= tol * tol * (app * aqq))) {
      // t = tan(theta) = sign(d) 2D / (|d| + sqrt(d^2 + 4 D^2)), d = aqq - app
      // (the root of smaller magnitude of t^2 + (d / D) t - 1 = 0)
      const double d = aqq - app;
      double t;
      if (fast_angle) {
        // the angle to FP32 accuracy (enough for a threshold of 2^-23: the
        // rotation stays exactly orthogonal, it only leaves a 2^-24
        // relative coupling); operands scaled by a power of two first
        int ex;
        (void)frexp(fmax(fabs(d), fabs(D)), &ex);
        const float df = (float)ldexp(d, -ex), Df = (float)ldexp(D, -ex);
        const float rf = __builtin_sqrtf(fmaf(df, df, 4.0f * Df * Df));
        // (an angle below the FP32 range, |D / d| < 2^-126, is taken as zero)
        t = (double)((df >= 0.0f ? 2.0f * Df : -2.0f * Df) * __builtin_amdgcn_rcpf(fabsf(df) + rf));
      } else {
        const double w = fma(d, d, 4.0 * D * D);
        t = (d >= 0.0 ? 2.0 * D : -2.0 * D) * rcp2(fabs(d) + w * rsqrt2(w));
      }
      if (t != 0.0) {
        cs = rsqrt2(fma(t, t, 1.0));
        sn = t * cs;
        tD = t * D;
        rotd = true;
      }
    }
    if (lane < P) {
      // lane == pid here
      rot[wave][pid] = make_double2(cs, sn);
      if (q < L) {
        // position p receives the rotated x_q, position q the rotated x_p
        nrm[p] = aqq + tD;
        nrm[q] = app - tD;
      }
    }
    const bool any = __ballot(rotd && lane < P) != 0;
    stamp(1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const double2 g = rot[wave][i];
#pragma unroll
      for (int r = 0; r < NRW; ++r) {
        const double xp = x[o + 2 * i][r], xq = x[o + 2 * i + 1][r];
        x[o + 2 * i][r] = fma(g.y, xp, g.x * xq);
        x[o + 2 * i + 1][r] = fma(g.x, xp, -(g.y * xq));
      }
    }
    if (prof) (void)__builtin_amdgcn_readfirstlane(__double2hiint(x[o][0] + x[o + 2 * P - 1][NRW - 1]));
    stamp(2);
    return any;
  };

  for (int sweep = 0; sweep < kJ1MaxSweeps; ++sweep) {
    norms();
    __syncthreads();
    if (tid == 0) s_rot[(sweep + 1) & 1] = 0;
    bool rotated = false;
    for (int t = 0; t < L; t += 2) {
      rotated |= step(IC1<0>{});
      // even -> odd window: slot 0 goes to the wave on the left (its slot C),
      // slot C comes from the wave on the right (zero past the end)
      double *b0 = xb;
      if (wave > 0)
#pragma unroll
        for (int r = 0; r < NRW; ++r) b0[wave * R + lane + 64 * r] = x[0][r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < NRW; ++r) x[C][r] = wave + 1 < NW ? b0[(wave + 1) * R + lane + 64 * r] : 0.0;
      stamp(3);
      rotated |= step(IC1<1>{});
      // odd -> even window: slot C goes back to the right, slot 0 comes
      // from the left (wave 0 kept its slot 0)
      double *b1 = xb + NW * R;
      if (wave + 1 < NW)
#pragma unroll
        for (int r = 0; r < NRW; ++r) b1[wave * R + lane + 64 * r] = x[C][r];
      __syncthreads();
      if (wave > 0)
#pragma unroll
        for (int r = 0; r < NRW; ++r) x[0][r] = b1[(wave - 1) * R + lane + 64 * r];
      stamp(3);
      psteps += 2;
    }
    if (rotated && lane == 0) s_rot[sweep & 1] = 1;
    __syncthreads();
    executed = sweep + 1;
    if (!s_rot[sweep & 1]) break;
    sweeps = sweep + 1;
  }
  if (prof) {
    for (int i = 0; i < 4; ++i) a.prof[i] += pacc[i];
    a.prof[4] += psteps;
  }
  // original index of the column at position p
  auto label = [&](int p) __attribute__((always_inline)) { return (executed & 1) ? L - 1 - p : p; };

  // ---------------------------------------------------------------- tail
  // exact norms, then rank the real positions by value, descending; ties by
  // label, descending
  norms();
  __syncthreads();
  for (int p = tid; p < L; p += NT) {
    int rk = -1;
    if (label(p) < l) {
      const double lp = nrm[p];
      rk = 0;
      for (int q = 0; q < L; ++q) {
        if (label(q) >= l || q == p) continue;
        const double lq = nrm[q];
        rk += (lq > lp) || (lq == lp && label(q) > label(p));
      }
      Ssh[rk] = sqrt(lp);
    }
    rank_of[p] = rk;
  }
  __syncthreads();
  const double tau = Ssh[0] * sqrt((double)l * 2.220446049250313e-16);
  for (int i = tid; i < l; i += NT) a.S[i] = Ssh[i];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int rk = rank_of[wave * C + c];
    if (rk >= 0) {
      const double sv = Ssh[rk];
      const double iv = sv > 0.0 ? 1.0 / sv : 0.0;
#pragma unroll
      for (int r = 0; r < NRW; ++r) {
        const int row = lane + 64 * r;
        if (row < l) {
          const double vv = x[c][r] * iv;
          a.W[(int64_t)row * l + rk] = sv > tau ? vv * iv : 0.0;
          if (a.Vs) a.Vs[(int64_t)row * l + rk] = vv;
        }
      }
    }
  }
  if (a.sweeps && tid == 0) *a.sweeps = sweeps;
  if (!state) return;
  if (tid == 0) {
    if (a.trace_sweeps && state->eig_calls < a.trace_cap + 2) a.trace_sweeps[state->eig_calls] = sweeps;
    state->eig_calls += 1;
    state->eig_sweeps += sweeps;
  }
  if (tid == 0 && !(Ssh[l - 1] > tau)) state->deficient = 1;
  if (a.mode != 2) return;
  pass_tail(a, state, Ssh);
}

}  // namespace

// Layout for size l <= 128: (C, NW, NRW) with L = C NW >= l.
template <bool B>
static hipError_t pick_eig1s(int l, void (**fn)(EigArgs, const EigArgs *), int *nt, size_t *shm) {
  int C = 0, NW = 0, NRW = 0;
  if (l < 1) return hipErrorInvalidValue;
  if (l <= 32) {
    C = 4, NW = 8, NRW = 1;
    *fn = k_eig1s<4, 8, 1, B>;
  } else if (l <= 64) {
    C = 8, NW = 8, NRW = 1;
    *fn = k_eig1s<8, 8, 1, B>;
  } else if (l <= 96) {
    C = 16, NW = 6, NRW = 2;
    *fn = k_eig1s<16, 6, 2, B>;
  } else if (l <= 128) {
    C = 16, NW = 8, NRW = 2;
    *fn = k_eig1s<16, 8, 2, B>;
  } else {
    // above 128 the columns of a wave no longer fit its registers; the
    // two-sided kernel serves these sizes
    return hipErrorInvalidValue;
  }
  const int R = 64 * NRW;
  const size_t pan = sizeof(double) * (size_t)2 * C * R, xch = sizeof(double) * (size_t)2 * NW * R;
  *shm = pan > xch ? pan : xch;
  *nt = NW * 64;
  return hipSuccess;
}

hipError_t launch_eig1s(const EigArgs &a, hipStream_t st) {
  void (*fn)(EigArgs, const EigArgs *) = nullptr;
  int nt = 0;
  size_t shm = 0;
  hipError_t e = pick_eig1s<false>(a.l, &fn, &nt, &shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(1), dim3(nt), shm, st, a, (const EigArgs *)nullptr);
  return hipGetLastError();
}

hipError_t launch_eig1s_batched(const EigArgs *arr, int count, int l, hipStream_t st) {
  if (count < 1) return hipSuccess;
  void (*fn)(EigArgs, const EigArgs *) = nullptr;
  int nt = 0;
  size_t shm = 0;
  hipError_t e = pick_eig1s<true>(l, &fn, &nt, &shm);
  if (e != hipSuccess) return e;
  EigArgs none;
  std::memset(&none, 0, sizeof(none));
  hipLaunchKernelGGL(fn, dim3((unsigned)count), dim3(nt), shm, st, none, arr);
  return hipGetLastError();
}

}  // namespace dsv
