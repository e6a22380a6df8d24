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
#include <cstring>

#include "common.h"
#include "pass_tail.h"

namespace dsv {

namespace {

constexpr int kEigThreadsS = 256;      // threads up to L = 32
constexpr int kEigThreads = 1024;      // threads up to L = 128
constexpr int kEigThreadsL = 512;      // threads above
constexpr int kMaxLP = 160;           // padded size L (multiple of 4)
constexpr int kMaxPairs = kMaxLP / 2;
constexpr int kMaxItems = 7;          // block items per thread per parity (L = 160, 512 threads)

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
// lane i+1; the edge lane receives zero, which callers never use.
__device__ __forceinline__ double dpp_move(double x, int ctrl_sel) {
  const long long b = __double_as_longlong(x);
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  if (ctrl_sel) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x138, 0xf, 0xf, true);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x138, 0xf, 0xf, true);
  } else {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x130, 0xf, 0xf, true);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x130, 0xf, 0xf, true);
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
// L = 128, 8 above, where L is then a multiple of 8); NT: threads (1024, or
// 512 for the largest sizes, so that 2 waves per SIMD leave room for V)
// BATCHED: workgroup b solves arr[b] (a0 unused); else a0.
template <int MAXNR, int MAXIT, int BATCH, int CPL, int NT, bool BATCHED, bool RSV>
__global__ __launch_bounds__(NT) void k_eig(EigArgs a0, const EigArgs *__restrict__ arr) {
  const EigArgs &a = BATCHED ? arr[blockIdx.x] : a0;
  if (a.run_if && *a.run_if == 0) return;
  if (a.skip_if && *a.skip_if) return;
  SolverState *state = a.state;
  if (!BATCHED && state && a.call_idx > 0 && threadIdx.x == 0) signal_started(&state->eig_started, a.call_idx);
  if (state && a.mode == 2) {
    // a pass launched after the check already passed: nothing to do, and
    // its rescale must not run either
    const int stopped = state->done;
    __syncthreads();
    if (threadIdx.x == 0) state->skip_rescale = stopped;
    if (stopped) return;
  }
  extern __shared__ double G[];  // packed upper, L(L+1)/2, then 2 zero words
  // rotation of each index group, by parity: (c, s) with M = [[s, c], [c, -s]]
  // (rotation then swap); a single-index group holds (0, 1), whose M keeps
  // its one index and multiplies the absent partner by -1
  __shared__ double2 rot_cs[2][kMaxPairs + 1];
  __shared__ double2 rot_tf[2][kMaxPairs + 1];  // (t = s/c, 1 if rotated else 0)
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

  for (int idx = tid; idx < L * L; idx += NT) {
    const int i = idx / L, j = idx - i * L;
    if (i <= j) G[pk(i, j, L)] = (i < l && j < l) ? a.G[(int64_t)i * l + j] : 0.0;
  }
  for (int p = tid; p < L; p += NT) label[p] = p;
  if (tid == 0) {
    // the word after (q,q) of the last diagonal block is read (and unused)
    G[L * (L + 1) / 2] = G[L * (L + 1) / 2 + 1] = 0.0;
    rot_cs[1][0] = rot_cs[1][P] = make_double2(0.0, 1.0);
    rot_tf[1][0] = rot_tf[1][P] = make_double2(0.0, 0.0);
  }

  // Block items of this thread for both parities, decoded once.  Index
  // groups: even parity g = {2g, 2g+1} (g < P); odd parity g = {2g-1, 2g}
  // (0 < g < P) and the single groups {0}, {L-1} (g = 0, P).  An item is a
  // pair of groups (gb <= ga), i.e. a block of G with b-rows and a-columns.
  // Items are listed as: blocks of two size-2 groups (row by row of the
  // packed upper triangle, so neighbouring lanes touch neighbouring LDS
  // words), then blocks with a single group, then diagonal blocks, so that
  // waves mostly take one code path.  Per item: the packed offsets of the
  // block's two b-rows at its first a-index (16-bit fields; the second
  // a-index is the next word of the row) and a meta word (groups ga, gb,
  // flags).  A diagonal block stores (p,p) and (q,q); (p,q) follows (p,p).
  // The tables live in registers, or (CPL = 8, the largest sizes) in LDS
  // after G with a 16-bit meta (ga | gb << 8, 0xffff = none) whose flags are
  // derived again when read.
  constexpr uint32_t kA2 = 1u << 16, kB2 = 1u << 17, kDiag = 1u << 18, kValid = 1u << 19;
  constexpr bool kTabLds = CPL == 8;
  uint32_t it_o[2][kTabLds ? 1 : MAXIT], it_m[2][kTabLds ? 1 : MAXIT];
  uint32_t *tab_o = reinterpret_cast<uint32_t *>(G + L * (L + 1) / 2 + 2);
  uint16_t *tab_m = reinterpret_cast<uint16_t *>(tab_o + 2 * MAXIT * NT);
#pragma unroll
  for (int par = 0; par < 2; ++par) {
    // full groups gf0..gf1 (size 2)
    const int gf0 = par ? 1 : 0, gf1 = par ? P - 1 : P - 1;
    const int nf = gf1 - gf0 + 1;
    const int n_full = nf * (nf - 1) / 2;
    const int n_part = par ? 2 * P - 1 : 0;
    const int n_diag = nf;
#pragma unroll
    for (int s_ = 0; s_ < MAXIT; ++s_) {
      int t = tid + s_ * NT;
      uint32_t o = 0, meta = 0;
      int ga = -1, gb = -1;
      bool diag = false;
      if (t < n_full) {
        int row = 0;
        while (t >= nf - 1 - row) {
          t -= nf - 1 - row;
          ++row;
        }
        gb = gf0 + row;
        ga = gb + 1 + t;
      } else if ((t -= n_full) < n_part) {
        // odd parity only: (0, 1..P), then (1..P-1, P)
        if (t < P) {
          gb = 0;
          ga = t + 1;
        } else {
          gb = t - P + 1;
          ga = P;
        }
      } else if ((t -= n_part) < n_diag) {
        ga = gb = gf0 + t;
        diag = true;
      }
      if (ga >= 0) {
        int fa, na, fb, nb;
        group_of(par, ga, P, fa, na);
        group_of(par, gb, P, fb, nb);
        if (diag) {
          o = (uint32_t)pk(fa, fa, L) | ((uint32_t)pk(fa + 1, fa + 1, L) << 16);
          meta = (uint32_t)ga | ((uint32_t)gb << 8) | kDiag | kValid;
        } else {
          // rows fb and fb+1 of the packed triangle at column fa (a single
          // b-index reads row fb twice; the word after a single a-index is
          // still inside the array, is finite, and only meets a zero
          // coefficient; neither is ever stored)
          const int i00 = pk(fb, fa, L);
          const int i01 = nb == 2 ? pk(fb + 1, fa, L) : i00;
          o = (uint32_t)i00 | ((uint32_t)i01 << 16);
          meta = (uint32_t)ga | ((uint32_t)gb << 8) | (na == 2 ? kA2 : 0u) | (nb == 2 ? kB2 : 0u) | kValid;
        }
      }
      if constexpr (kTabLds) {
        tab_o[(par * MAXIT + s_) * NT + tid] = o;
        tab_m[(par * MAXIT + s_) * NT + tid] =
            (meta & kValid) ? (uint16_t)(meta & 0xffff) : (uint16_t)0xffff;
      } else {
        it_o[par][s_] = o;
        it_m[par][s_] = meta;
      }
    }
  }

  // V in registers: lane column block cl owns columns CPL cl .. CPL cl +
  // CPL - 1 of its rows
  const int LPR = L / CPL;           // lanes per row
  const int RPW = kWave / LPR;       // rows per wave
  const int sub = lane / LPR, cl = lane - sub * LPR;
  const bool active = sub < RPW;
  // RSV: wave 0 holds no rows of V (it computes the rotations while the
  // other waves update V)
  const int vwave = RSV ? wave - 1 : wave;
  const int row_stride = (NT / kWave - (RSV ? 1 : 0)) * RPW;
  const int NR = (L + row_stride - 1) / row_stride;
  const int c0 = CPL * cl;
  double v[MAXNR][CPL];
#pragma unroll
  for (int it = 0; it < MAXNR; ++it) {
    const int row = vwave * RPW + sub + it * row_stride;
#pragma unroll
    for (int j = 0; j < CPL; ++j) v[it][j] = (vwave >= 0 && active && row < L && row == c0 + j) ? 1.0 : 0.0;
  }
  if (tid == 0) s_sweeps = 0;
  __syncthreads();

  // V <- V M for the index groups of one parity; waves that hold no row skip.
  // Even steps: groups c0/2 + i = (c0 + 2i, c0 + 2i + 1) inside the lane.
  // Odd steps: groups c0/2 + i + 1 = (c0 + 2i + 1, c0 + 2i + 2) inside the
  // lane, and the edge groups c0/2 (this lane holds the second member) and
  // c0/2 + CPL/2 (this lane holds the first member) shared with the
  // neighbouring lanes.  The first lane of a row holds the single group {0}
  // alone, which keeps its value.
  auto v_update = [&](auto vpar_c) __attribute__((always_inline)) {
    constexpr int VPAR = decltype(vpar_c)::value;
    if (vwave < 0 || vwave * RPW >= L) return;
    const double2 *rcs = rot_cs[VPAR];
    if constexpr (VPAR == 0) {
      double2 cs[CPL / 2];
#pragma unroll
      for (int i = 0; i < CPL / 2; ++i) cs[i] = rcs[c0 / 2 + i];
#pragma unroll
      for (int it = 0; it < MAXNR; ++it) {
        if (it < NR) {
#pragma unroll
          for (int i = 0; i < CPL / 2; ++i) {
            const double x = v[it][2 * i], y = v[it][2 * i + 1];
            v[it][2 * i] = fma(x, cs[i].y, y * cs[i].x);
            v[it][2 * i + 1] = fma(x, cs[i].x, -(y * cs[i].y));
          }
        }
      }
    } else {
      double2 cs[CPL / 2 + 1];  // [0]: left edge group, [1..]: inner groups, [CPL/2]: right edge
#pragma unroll
      for (int i = 0; i <= CPL / 2; ++i) cs[i] = rcs[c0 / 2 + i];
      const bool first = cl == 0;
#pragma unroll
      for (int it = 0; it < MAXNR; ++it) {
        if (it < NR) {
          const double nxt = wave_shl1(v[it][0]);
          const double prv = wave_shr1(v[it][CPL - 1]);
#pragma unroll
          for (int i = 0; i < CPL / 2 - 1; ++i) {
            const double2 r = cs[i + 1];
            const double x = v[it][2 * i + 1], y = v[it][2 * i + 2];
            v[it][2 * i + 1] = fma(x, r.y, y * r.x);
            v[it][2 * i + 2] = fma(x, r.x, -(y * r.y));
          }
          const double x0 = v[it][0], xl = v[it][CPL - 1];
          const double y0 = fma(prv, cs[0].x, -(x0 * cs[0].y));
          v[it][0] = first ? x0 : y0;
          // the last lane's right group is the single {L-1}: (c, s) = (0, 1)
          v[it][CPL - 1] = fma(xl, cs[CPL / 2].y, nxt * cs[CPL / 2].x);
        }
      }
    }
  };

  for (int sweep = 0; sweep < 60; ++sweep) {
    // convergence test before the sweep: any entry above the skip threshold?
    if (tid == 0) s_flag = 0;
    __syncthreads();
    for (int idx = tid; idx < L * L; idx += NT) {
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
    //   2. the blocks of G are updated, B <- Ma^T B Mb, all loads of a batch
    //      issued before its first store.
    auto do_step = [&](auto par_c, int step) __attribute__((always_inline)) {
      constexpr int par = decltype(par_c)::value;
      const int npairs = par ? P - 1 : P;
      long long c0_ = 0, w0 = 0, ca_ = 0, cv = 0;
      if (a.prof && tid == 0) {
        c0_ = clock64();
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
        const int grp = par ? tid + 1 : tid;
        rot_cs[par][grp] = make_double2(c, s);
        rot_tf[par][grp] = make_double2(t, rot);
        label[p] = lq;
        label[q] = lp;
      }
      if (a.prof && tid == 0) ca_ = clock64();
      if (step > 0) v_update(IC<par ^ 1>{});
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
        auto item = [&](int s_, uint32_t &o, uint32_t &meta) __attribute__((always_inline)) {
          if constexpr (kTabLds) {
            o = tab_o[(PAR * MAXIT + s_) * NT + tid];
            const uint32_t m16 = tab_m[(PAR * MAXIT + s_) * NT + tid];
            const uint32_t ga = m16 & 0xff, gb = m16 >> 8;
            const bool a1 = PAR == 1 && (ga == 0 || ga == (uint32_t)P);
            const bool b1 = PAR == 1 && (gb == 0 || gb == (uint32_t)P);
            meta = m16 == 0xffff ? 0u
                                 : (m16 | kValid | (ga == gb ? kDiag : 0u) | (a1 ? 0u : kA2) | (b1 ? 0u : kB2));
          } else {
            o = it_o[PAR][s_];
            meta = it_m[PAR][s_];
          }
        };
#pragma unroll
        for (int b0 = 0; b0 < MAXIT; b0 += BATCH) {
          uint32_t ob[BATCH], mb[BATCH];
#pragma unroll
          for (int s_ = b0; s_ < b0 + BATCH; ++s_) item(s_, ob[s_ - b0], mb[s_ - b0]);
          double g[BATCH][4];
          double2 pa[BATCH], pb[BATCH];
          // loads: the two words of each b-row are adjacent (paired loads).
          // An absent item (meta 0) reads the first words of G and of the
          // rotation table and is then skipped, so no load needs a branch.
#pragma unroll
          for (int s_ = b0; s_ < b0 + BATCH; ++s_) {
            const int j = s_ - b0;
            const uint32_t meta = mb[j], o = ob[j];
            const int r0 = o & 0xffff, r1 = o >> 16;
            const int ga = meta & 0xff, gb = (meta >> 8) & 0xff;
            g[j][0] = G[r0];
            g[j][1] = G[r0 + 1];
            g[j][2] = G[r1];
            g[j][3] = G[r1 + 1];
            pa[j] = ((meta & kDiag) ? rtf : rcs)[ga];
            pb[j] = rcs[gb];
          }
#pragma unroll
          for (int s_ = b0; s_ < b0 + BATCH; ++s_) {
            const int j = s_ - b0;
            const uint32_t meta = mb[j], o = ob[j];
            if (!(meta & kValid)) continue;
            const int r0 = o & 0xffff, r1 = o >> 16;
            if (meta & kDiag) {
              // (p,p), (p,q), (q,q) of a rotated-and-swapped pair: the diagonal
              // becomes (a_qq + t a_pq, a_pp - t a_pq) and the coupling vanishes
              const double app = g[j][0], apq = g[j][1], aqq = g[j][2];
              const double2 tf = pa[j];
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
            // off-diagonal block B[a][b] at row fb + b, column fa + a:
            // T = B Mb, B' = Ma^T T with M = [[s, c], [c, -s]]
            const double ca = pa[j].x, sa = pa[j].y, cb = pb[j].x, sb = pb[j].y;
            const double g00 = g[j][0], g10 = g[j][1], g01 = g[j][2], g11 = g[j][3];
            const double t00 = fma(g00, sb, g01 * cb), t01 = fma(g00, cb, -(g01 * sb));
            const double t10 = fma(g10, sb, g11 * cb), t11 = fma(g10, cb, -(g11 * sb));
            const double n00 = fma(sa, t00, ca * t10), n10 = fma(ca, t00, -(sa * t10));
            const double n01 = fma(sa, t01, ca * t11), n11 = fma(ca, t01, -(sa * t11));
            if ((meta & (kA2 | kB2)) == (kA2 | kB2)) {
              G[r0] = n00;
              G[r0 + 1] = n10;
              G[r1] = n01;
              G[r1 + 1] = n11;
            } else {
              G[r0] = n00;
              if (meta & kA2) G[r0 + 1] = n10;
              if (meta & kB2) G[r1] = n01;
            }
          }
        }
      };
      g_update(IC<par>{});
      __syncthreads();
      if (a.prof && tid == 0) {
        // step profile (thread 0): cycles of phase 1 and of phase 2 (each up
        // to its barrier), wall-clock ticks (100 MHz), steps, cycles of this
        // thread's rotation work and of its V update in phase 1
        const long long c2 = clock64();
        a.prof[0] += c1 - c0_;
        a.prof[1] += c2 - c1;
        a.prof[2] += wall_clock64() - w0;
        a.prof[3] += 1;
        a.prof[4] += ca_ - c0_;
        a.prof[5] += cv - ca_;
      }
    };
    for (int step = 0; step < L; step += 2) {
      do_step(IC<0>{}, step);
      do_step(IC<1>{}, step + 1);
    }
    // the sweep's last step is odd: its V update is still pending
    v_update(IC<1>{});
  }

  // ---------------------------------------------------------------- tail
  // rank the real positions by eigenvalue, descending; ties by label, descending
  for (int p = tid; p < L; p += NT) {
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
  for (int i = tid; i < l; i += NT) a.S[i] = Ssh[i];
#pragma unroll
  for (int it = 0; it < MAXNR; ++it) {
    const int row = vwave * RPW + sub + it * row_stride;
    if (vwave >= 0 && it < NR && active && row < l) {
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
    if (a.trace_sweeps && state->eig_calls < a.trace_cap + 2) a.trace_sweeps[state->eig_calls] = s_sweeps;
    state->eig_calls += 1;
    state->eig_sweeps += s_sweeps;
  }
  if (tid == 0 && !(Ssh[l - 1] > tau)) state->deficient = 1;
  if (a.mode != 2) return;

  pass_tail(a, state, Ssh);
}

// Accuracy control without the surrogate: the check of eq. (18) on
// E_i = Sb_i^2, the squared singular values of B = M Q, against the
// previous pass's E' (the same ratio as the surrogate check of Alg. 5
// step 5 with every shift set to zero).
__global__ __launch_bounds__(kWave) void k_pve_nosurr(int k, int l, const double *__restrict__ Sb,
                                                      double *__restrict__ Ebp, double tol, double cq_switch,
                                                      SolverState *__restrict__ state,
                                                      double *__restrict__ trace_ratio, int trace_cap,
                                                      const int32_t *__restrict__ gate) {
  if (gate && *gate) return;
  const int tid = threadIdx.x;
  double worst = 0.0;
  const double ek1 = Sb[k] * Sb[k];
  for (int i = tid; i < k; i += kWave) {
    const double e = Sb[i] * Sb[i];
    const double v = fabs(Ebp[i] - e) / ek1;
    if (v > worst || v != v) worst = v;
  }
  // wavefront maximum (NaN wins, as in the surrogate check)
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const double o = __shfl_xor(worst, off, kWave);
    if (o > worst || o != o) worst = o;
  }
  const bool stop = tol > 0.0 && worst <= tol;
  if (!stop)
    for (int i = tid; i < l; i += kWave) Ebp[i] = Sb[i] * Sb[i];
  if (tid == 0) {
    const int j = state->pass;
    if (j >= 1 && j - 1 < trace_cap) trace_ratio[j - 1] = worst;
    state->ratio = worst;
    if (cq_switch > 0.0 && tol > 0.0 && worst <= cq_switch * tol) state->cq_off = 1;
    if (stop) {
      state->converged = 1;
      __hip_atomic_store(&state->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace

hipError_t launch_pve_nosurr(int k, int l, const double *Sb, double *Ebp, double tol, double cq_switch,
                             SolverState *state, double *trace_ratio, int trace_cap, const int32_t *gate,
                             hipStream_t st) {
  if (k < 1 || l <= k || !state) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_pve_nosurr, dim3(1), dim3(kWave), 0, st, k, l, Sb, Ebp, tol, cq_switch, state, trace_ratio,
                     trace_cap, gate);
  return hipGetLastError();
}

// Kernel variant, block size and dynamic LDS for size l (the layout rules of
// the kernel, mirrored): CPL columns of V per lane, L = l padded to a
// multiple of CPL, NT threads.
template <bool B>
static hipError_t pick_eig(int l, void (**fn)(EigArgs, const EigArgs *), int *nt, size_t *shm) {
  if (l < 1 || l > kMaxLP) return hipErrorInvalidValue;
  const int L4 = (l + 3) & ~3;
  const int CPL = L4 > 128 ? 8 : 4;
  const int NT = CPL == 8 ? kEigThreadsL : (L4 <= 32 ? kEigThreadsS : kEigThreads);
  const int L = CPL == 8 ? (l + 7) & ~7 : L4;
  const int P = L / 2;
  const int LPR = L / CPL, RPW = kWave / LPR;
  const int NR = (L + (NT / kWave) * RPW - 1) / ((NT / kWave) * RPW);
  // with wave 0 kept free of V rows (its lanes compute the P <= 64 rotations)
  const int NRr = (L + (NT / kWave - 1) * RPW - 1) / ((NT / kWave - 1) * RPW);
  const int IT = ((P + 1) * (P + 2) / 2 + NT - 1) / NT;  // odd parity has more
  size_t s = sizeof(double) * (size_t)(L * (L + 1) / 2 + 2);
  if (CPL == 8) s += (size_t)2 * kMaxItems * NT * (sizeof(uint32_t) + sizeof(uint16_t));
  void (*f)(EigArgs, const EigArgs *) = nullptr;
  if (NT == kEigThreadsS && NR <= 1 && IT <= 1)
    f = k_eig<1, 1, 1, 4, kEigThreadsS, B, false>;
  else if (CPL == 4 && NT == kEigThreads && NRr <= 1 && IT <= 1)
    f = k_eig<1, 1, 1, 4, kEigThreads, B, true>;
  else if (CPL == 4 && NT == kEigThreads && NRr <= 2 && IT <= 2)
    f = k_eig<2, 2, 2, 4, kEigThreads, B, true>;
  else if (CPL == 4 && NT == kEigThreads && NRr <= 4 && IT <= 2)
    f = k_eig<4, 2, 2, 4, kEigThreads, B, true>;
  else if (CPL == 4 && NT == kEigThreads && NR <= 4 && IT <= 2)
    f = k_eig<4, 2, 2, 4, kEigThreads, B, false>;
  else if (CPL == 4 && NT == kEigThreads && NR <= 4 && IT <= 3)
    f = k_eig<4, 3, 1, 4, kEigThreads, B, false>;
  else if (CPL == 8 && NR <= 7 && IT <= kMaxItems)
    f = k_eig<7, kMaxItems, 1, 8, kEigThreadsL, B, false>;
  else
    return hipErrorInvalidValue;
  // dynamic LDS above the default limit: allow exactly what this size needs
  if (s > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute((const void *)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)s);
    if (e != hipSuccess) return e;
  }
  *fn = f;
  *nt = NT;
  *shm = s;
  return hipSuccess;
}

hipError_t launch_eig(const EigArgs &a, hipStream_t st) {
  void (*fn)(EigArgs, const EigArgs *) = nullptr;
  int nt = 0;
  size_t shm = 0;
  hipError_t e = pick_eig<false>(a.l, &fn, &nt, &shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(1), dim3(nt), shm, st, a, (const EigArgs *)nullptr);
  return hipGetLastError();
}

hipError_t launch_eig_batched(const EigArgs *arr, int count, int l, hipStream_t st) {
  if (count < 1) return hipSuccess;
  void (*fn)(EigArgs, const EigArgs *) = nullptr;
  int nt = 0;
  size_t shm = 0;
  hipError_t e = pick_eig<true>(l, &fn, &nt, &shm);
  if (e != hipSuccess) return e;
  EigArgs none;
  std::memset(&none, 0, sizeof(none));
  hipLaunchKernelGGL(fn, dim3((unsigned)count), dim3(nt), shm, st, none, arr);
  return hipGetLastError();
}

}  // namespace dsv
