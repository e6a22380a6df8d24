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
//   - the rotation parameters of a step are published in LDS, one buffer
//     per parity.
// A step is: rotations (one thread per pair) overlapped with the previous
// step's V update | barrier | 2x2 block updates of G (one thread per block
// pair, addresses decoded once per launch) | barrier.
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
constexpr int kMaxItems = 4;          // block items per thread per parity (L = 160)

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

// Whole-wave shifts by one lane through DPP (a VALU modifier: no LDS
// traffic).  wave_shr1: lane i receives lane i-1; wave_shl1: lane i receives
// lane i+1; the edge lane keeps its own value, which callers never use.
__device__ __forceinline__ double dpp_move(double x, int ctrl_sel) {
  const long long b = __double_as_longlong(x);
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  if (ctrl_sel) {
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
  } else {
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
  }
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}
__device__ __forceinline__ double wave_shr1(double x) { return dpp_move(x, 1); }
__device__ __forceinline__ double wave_shl1(double x) { return dpp_move(x, 0); }

template <int N>
struct IC {
  static constexpr int value = N;
};

// MAXNR: register row slots of V per lane; MAXIT: G block items per thread
// and parity (both upper bounds for the launched size); BATCH: items whose
// loads are issued together; CPL: consecutive V columns per lane (4 up to
// L = 128, 8 above, where L is then a multiple of 8)
template <int MAXNR, int MAXIT, int BATCH, int CPL>
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
  __shared__ double2 rot_cs[2][kMaxPairs];  // (c, s) of each pair's rotation, by parity
  __shared__ double2 rot_tf[2][kMaxPairs];  // (t = s/c, 1 if rotated else 0), by parity
  __shared__ int label[kMaxLP];
  __shared__ int rank_of[kMaxLP];
  __shared__ double Ssh[kMaxLP];
  __shared__ int s_flag;
  __shared__ int s_sweeps;

  const int l = a.l;
  const double kSkip = a.skip;  // rotation / convergence threshold (relative)
  const int L = CPL == 8 ? (l + 7) & ~7 : (l + 3) & ~3;
  const int P = L / 2;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  for (int idx = tid; idx < L * L; idx += kEigThreads) {
    const int i = idx / L, j = idx - i * L;
    if (i <= j) G[pk(i, j, L)] = (i < l && j < l) ? a.G[(int64_t)i * l + j] : 0.0;
  }
  for (int p = tid; p < L; p += kEigThreads) label[p] = p;

  // Block items of this thread for both parities, decoded once: pairs of
  // groups (gb <= ga) enumerated row by row of the packed upper triangle (gb
  // outer, ga inner), so neighbouring lanes touch neighbouring LDS words.
  // Per item: the packed offsets of the block's two b-rows at its first
  // a-index (two 16-bit fields; the second a-index is the next word of the
  // same row) and a meta word: rotation slots of both groups, whether each
  // group holds two indices, whether the block is diagonal, whether the item
  // exists.  For a diagonal block the fields are (p,p) and (q,q); (p,q) is
  // the word after (p,p).
  constexpr uint32_t kA2 = 1u << 16, kB2 = 1u << 17, kDiag = 1u << 18, kValid = 1u << 19;
  uint32_t it_o[2][MAXIT], it_m[2][MAXIT];
#pragma unroll
  for (int par = 0; par < 2; ++par) {
    const int ng = par ? P + 1 : P;
    const int nitems = ng * (ng + 1) / 2;
    const int npairs = par ? P - 1 : P;
#pragma unroll
    for (int s_ = 0; s_ < MAXIT; ++s_) {
      const int t = tid + s_ * kEigThreads;
      uint32_t o = 0, meta = 0;
      if (t < nitems) {
        int gb = 0, rem = t;
        while (rem >= ng - gb) {
          rem -= ng - gb;
          ++gb;
        }
        const int ga = gb + rem;
        int fa, na, fb, nb;
        group_of(par, ga, P, fa, na);
        group_of(par, gb, P, fb, nb);
        int sa = slot_of(par, ga), sb = slot_of(par, gb);
        sa = sa < 0 ? 0 : (sa >= npairs ? npairs - 1 : sa);
        sb = sb < 0 ? 0 : (sb >= npairs ? npairs - 1 : sb);
        if (ga == gb) {
          if (na == 2) {
            o = (uint32_t)pk(fa, fa, L) | ((uint32_t)pk(fa + 1, fa + 1, L) << 16);
            meta = (uint32_t)sa | kDiag | kValid;
          }
        } else {
          // rows fb and fb+1 of the packed triangle at column fa (a single
          // b-index reuses row fb; the word after a single a-index is still
          // inside the array and is loaded but never used or stored)
          const int i00 = pk(fb, fa, L);
          const int i01 = nb == 2 ? pk(fb + 1, fa, L) : i00;
          o = (uint32_t)i00 | ((uint32_t)i01 << 16);
          meta = (uint32_t)sa | ((uint32_t)sb << 8) | (na == 2 ? kA2 : 0u) | (nb == 2 ? kB2 : 0u) | kValid;
        }
      }
      it_o[par][s_] = o;
      it_m[par][s_] = meta;
    }
  }

  // V in registers: lane column block cl owns columns CPL cl .. CPL cl +
  // CPL - 1 of its rows
  const int LPR = L / CPL;           // lanes per row
  const int RPW = kWave / LPR;       // rows per wave
  const int sub = lane / LPR, cl = lane - sub * LPR;
  const bool active = sub < RPW;
  const int row_stride = (kEigThreads / kWave) * RPW;
  const int NR = (L + row_stride - 1) / row_stride;
  const int c0 = CPL * cl;
  double v[MAXNR][CPL];
#pragma unroll
  for (int it = 0; it < MAXNR; ++it) {
    const int row = wave * RPW + sub + it * row_stride;
#pragma unroll
    for (int j = 0; j < CPL; ++j) v[it][j] = (active && row < L && row == c0 + j) ? 1.0 : 0.0;
  }
  if (tid == 0) s_sweeps = 0;
  __syncthreads();

  // V <- V M for the column pairs of one parity, with that parity's
  // published rotations; waves that hold no row skip.  M = [[s, c], [c, -s]]
  // (rotation then swap; c = 1, s = 0 is the plain swap), M = I outside the
  // pairs of the step.  Even steps pair (c0 + 2i, c0 + 2i + 1) inside the
  // lane (slot c0/2 + i); odd steps pair (c0 + 2i + 1, c0 + 2i + 2) inside
  // it (slot c0/2 + i) and the two edge columns with the neighbouring lanes
  // (slots c0/2 - 1 and c0/2 + CPL/2 - 1).
  auto v_update = [&](int vpar) __attribute__((always_inline)) {
    if (wave * RPW >= L) return;
    const int npairs = vpar ? P - 1 : P;
    const double2 *rcs = rot_cs[vpar];
    const bool first = cl == 0, last = cl == LPR - 1;
    if (!vpar) {
      double2 cs[CPL / 2];
#pragma unroll
      for (int i = 0; i < CPL / 2; ++i) {
        const int sl = c0 / 2 + i;
        cs[i] = rcs[sl < npairs ? sl : npairs - 1];
        if (sl >= npairs) cs[i] = make_double2(0.0, 1.0);  // only on idle lanes
      }
#pragma unroll
      for (int it = 0; it < MAXNR; ++it) {
        if (it < NR) {
#pragma unroll
          for (int i = 0; i < CPL / 2; ++i) {
            const double x = v[it][2 * i], y = v[it][2 * i + 1];
            v[it][2 * i] = x * cs[i].y + y * cs[i].x;
            v[it][2 * i + 1] = x * cs[i].x - y * cs[i].y;
          }
        }
      }
    } else {
      double2 cs[CPL / 2 + 1];  // [0]: left edge pair, [1..]: inner pairs, [CPL/2]: right edge
#pragma unroll
      for (int i = 0; i <= CPL / 2; ++i) {
        const int sl = c0 / 2 - 1 + i;
        const int slc = sl < 0 ? 0 : (sl >= npairs ? npairs - 1 : sl);
        cs[i] = rcs[slc];
      }
#pragma unroll
      for (int it = 0; it < MAXNR; ++it) {
        if (it < NR) {
          const double nxt = wave_shl1(v[it][0]);
          const double prv = wave_shr1(v[it][CPL - 1]);
#pragma unroll
          for (int i = 0; i < CPL / 2 - 1; ++i) {
            const double2 r = cs[i + 1];
            const double x = v[it][2 * i + 1], y = v[it][2 * i + 2];
            v[it][2 * i + 1] = x * r.y + y * r.x;
            v[it][2 * i + 2] = x * r.x - y * r.y;
          }
          const double x0 = v[it][0], xl = v[it][CPL - 1];
          v[it][0] = first ? x0 : prv * cs[0].x - x0 * cs[0].y;
          v[it][CPL - 1] = last ? xl : xl * cs[CPL / 2].y + nxt * cs[CPL / 2].x;
        }
      }
    }
  };

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
    // A step has two phases separated by barriers:
    //   1. one thread per pair computes this step's rotation (and swaps the
    //      two labels), while every thread applies the previous step's
    //      rotations to its rows of V (rotations are double-buffered by
    //      parity; L is even, so parity = step & 1 in every sweep);
    //   2. the 2x2 blocks of G are updated, B <- Ma^T B Mb, all loads of a
    //      thread issued before its first store.
    for (int step = 0; step < L; ++step) {
      const int par = step & 1;
      const int npairs = par ? P - 1 : P;
      long long c0 = 0, w0 = 0, ca_ = 0, cv = 0;
      if (a.prof && tid == 0) {
        c0 = clock64();
        w0 = wall_clock64();
      }
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
        rot_cs[par][tid] = make_double2(c, s);
        rot_tf[par][tid] = make_double2(t, rot);
        label[p] = lq;
        label[q] = lp;
      }
      if (a.prof && tid == 0) ca_ = clock64();
      if (step > 0) v_update(par ^ 1);
      if (a.prof && tid == 0) cv = clock64();
      __syncthreads();
      long long c1 = 0;
      if (a.prof && tid == 0) c1 = clock64();

      // the parity is a compile-time index into the item tables, so they stay
      // in registers
      auto g_update = [&](auto par_c) __attribute__((always_inline)) {
        constexpr int PAR = decltype(par_c)::value;
        const double2 *rcs = rot_cs[PAR];
        const double2 *rtf = rot_tf[PAR];
        // items in batches of BATCH (register pressure of the large sizes)
#pragma unroll
        for (int b0 = 0; b0 < MAXIT; b0 += BATCH) {
          double g[BATCH][4];
          double2 pa[BATCH], pb[BATCH];
          // loads: the two words of each b-row are adjacent, so each row is
          // one paired 8-byte load and a wave's lanes cover contiguous LDS
#pragma unroll
          for (int s_ = b0; s_ < b0 + BATCH; ++s_) {
            const uint32_t meta = it_m[PAR][s_], o = it_o[PAR][s_];
            g[s_ - b0][0] = g[s_ - b0][1] = g[s_ - b0][2] = g[s_ - b0][3] = 0.0;
            pa[s_ - b0] = pb[s_ - b0] = make_double2(0.0, 0.0);
            if (meta & kValid) {
              const int r0 = o & 0xffff, r1 = o >> 16;
              const int sa = meta & 0xff, sb = (meta >> 8) & 0xff;
              g[s_ - b0][0] = G[r0];
              g[s_ - b0][1] = G[r0 + 1];
              g[s_ - b0][2] = G[r1];
              if (meta & kDiag) {
                pa[s_ - b0] = rtf[sa];
              } else {
                g[s_ - b0][3] = G[r1 + 1];
                pa[s_ - b0] = rcs[sa];
                pb[s_ - b0] = rcs[sb];
              }
            }
          }
#pragma unroll
          for (int s_ = b0; s_ < b0 + BATCH; ++s_) {
            const uint32_t meta = it_m[PAR][s_], o = it_o[PAR][s_];
            if (!(meta & kValid)) continue;
            const int r0 = o & 0xffff, r1 = o >> 16;
            if (meta & kDiag) {
              // (p,p), (p,q), (q,q) of a rotated-and-swapped pair: the diagonal
              // becomes (a_qq + t a_pq, a_pp - t a_pq) and the coupling vanishes
              const double app = g[s_ - b0][0], apq = g[s_ - b0][1], aqq = g[s_ - b0][2];
              const double2 tf = pa[s_ - b0];
              if (tf.y != 0.0) {
                G[r0] = fma(tf.x, apq, aqq);
                G[r0 + 1] = 0.0;
                G[r1] = fma(-tf.x, apq, app);
              } else {
                G[r0] = aqq;
                G[r1] = app;
              }
              continue;
            }
            // off-diagonal block B[a][b] at row fb + b, column fa + a; a
            // single-index group has M = [1]
            const bool a2 = meta & kA2, b2 = meta & kB2;
            const double2 csa = pa[s_ - b0], csb = pb[s_ - b0];
            const double ma00 = a2 ? csa.y : 1.0, ma01 = a2 ? csa.x : 0.0;
            const double ma10 = a2 ? csa.x : 0.0, ma11 = a2 ? -csa.y : 1.0;
            const double mb00 = b2 ? csb.y : 1.0, mb01 = b2 ? csb.x : 0.0;
            const double mb10 = b2 ? csb.x : 0.0, mb11 = b2 ? -csb.y : 1.0;
            const double g00 = g[s_ - b0][0];
            const double b10 = a2 ? g[s_ - b0][1] : 0.0;
            const double b01 = b2 ? g[s_ - b0][2] : 0.0;
            const double b11 = (a2 && b2) ? g[s_ - b0][3] : 0.0;
            // T = B Mb ; B' = Ma^T T
            const double t00 = g00 * mb00 + b01 * mb10, t01 = g00 * mb01 + b01 * mb11;
            const double t10 = b10 * mb00 + b11 * mb10, t11 = b10 * mb01 + b11 * mb11;
            const double n00 = ma00 * t00 + ma10 * t10, n10 = ma01 * t00 + ma11 * t10;
            const double n01 = ma00 * t01 + ma10 * t11, n11 = ma01 * t01 + ma11 * t11;
            if (a2) {
              G[r0] = n00;
              G[r0 + 1] = n10;
            } else {
              G[r0] = n00;
            }
            if (b2) {
              if (a2) {
                G[r1] = n01;
                G[r1 + 1] = n11;
              } else {
                G[r1] = n01;
              }
            }
          }
        }
      };
      if (par)
        g_update(IC<1>{});
      else
        g_update(IC<0>{});
      __syncthreads();
      if (a.prof && tid == 0) {
        // step profile (thread 0): cycles of phase 1 and of phase 2 (each up
        // to its barrier), wall-clock ticks (100 MHz), steps, cycles of this
        // thread's rotation work and of its V update in phase 1
        const long long c2 = clock64();
        a.prof[0] += c1 - c0;
        a.prof[1] += c2 - c1;
        a.prof[2] += wall_clock64() - w0;
        a.prof[3] += 1;
        a.prof[4] += ca_ - c0;
        a.prof[5] += cv - ca_;
      }
    }
    // the sweep's last step is odd: its V update is still pending
    v_update(1);
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
      for (int j = 0; j < CPL; ++j) {
        const int p = c0 + j;
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
  // the layout rules of the kernel, mirrored: CPL columns of V per lane,
  // L = l padded to a multiple of CPL
  const int L4 = (a.l + 3) & ~3;
  const int CPL = L4 > 128 ? 8 : 4;
  const int L = CPL == 8 ? (a.l + 7) & ~7 : L4;
  const int P = L / 2;
  const int LPR = L / CPL, RPW = kWave / LPR;
  const int NR = (L + 16 * RPW - 1) / (16 * RPW);
  const int IT = ((P + 1) * (P + 2) / 2 + kEigThreads - 1) / kEigThreads;  // odd parity has more
  const size_t shm = sizeof(double) * (size_t)(L * (L + 1) / 2);
  void (*fn)(EigArgs) = nullptr;
  if (CPL == 4 && NR <= 1 && IT <= 1)
    fn = k_eig<1, 1, 1, 4>;
  else if (CPL == 4 && NR <= 2 && IT <= 2)
    fn = k_eig<2, 2, 2, 4>;
  else if (CPL == 4 && NR <= 4 && IT <= 2)
    fn = k_eig<4, 2, 2, 4>;
  else if (CPL == 4 && NR <= 4 && IT <= 3)
    fn = k_eig<4, 3, 1, 4>;
  else if (CPL == 8 && NR <= 4 && IT <= kMaxItems)
    fn = k_eig<4, kMaxItems, 1, 8>;
  else
    return hipErrorInvalidValue;
  static bool attr = false;
  if (!attr) {
    hipFuncSetAttribute((const void *)k_eig<1, 1, 1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    hipFuncSetAttribute((const void *)k_eig<2, 2, 2, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    hipFuncSetAttribute((const void *)k_eig<4, 2, 2, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    hipFuncSetAttribute((const void *)k_eig<4, 3, 1, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, 128 * 1024);
    hipFuncSetAttribute((const void *)k_eig<4, kMaxItems, 1, 8>, hipFuncAttributeMaxDynamicSharedMemorySize,
                        128 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL(fn, dim3(1), dim3(kEigThreads), shm, st, a);
  return hipGetLastError();
}

}  // namespace dsv
