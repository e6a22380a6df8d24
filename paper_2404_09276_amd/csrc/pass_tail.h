// Alg. 5 steps 5-7 after the eigSVD of a power pass, shared by the
// eigensolvers of a pass block (Jacobi, k_eig.hip; Cholesky-QR with
// eigenvalues only, k_cholqr.hip): the PVE ratio of eq. (19) with the
// surrogate E = S + alpha (Prop. 3), the learned shift's inference after
// pass 2, the traces, the stop flag and the shift rule.  Run by every
// thread of one workgroup; S (LDS or global, l values, descending) are the
// singular values of the pass block.
#pragma once

#include "common.h"

namespace dsv {

constexpr int kTailMaxL = 160;

__device__ __forceinline__ void pass_tail(const EigArgs &a, SolverState *state, const double *Ssh) {
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  const int l = a.l;
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
  if (a.policy == 4 && a.mlp && j == 2 && a.sched && !s_stop) {
    // Learned shift: features of passes 1 and 2 (E_i = S_i + the shift that
    // produced them), the MLP forward pass, then the multiplier c for the
    // shifts of passes 3, 4, ... into the schedule read below.
    __shared__ float mf[3 * kTailMaxL + 3];
    __shared__ float mh1[kMlpH], mh2[kMlpH];
    __shared__ float mo[2];
    const int D = a.mlp_D, H = a.mlp_H;
    const double a1 = a.trace_alpha[0];
    const double e11 = a.trace_s[0] + a1, e21 = Ssh[0] + alpha;
    for (int i = tid; i < l; i += NT) {
      const double e1 = a.trace_s[i] + a1, e2 = Ssh[i] + alpha;
      mf[i] = e11 > 0.0 ? (float)(e1 / e11) : 0.0f;
      mf[l + i] = e21 > 0.0 ? (float)(e2 / e21) : 0.0f;
      mf[2 * l + i] = e1 > 0.0 ? (float)(e2 / e1) : 0.0f;
    }
    if (tid < 3) mf[3 * l + tid] = (float)a.shape_feat[tid];
    __syncthreads();
    const float *W1 = a.mlp, *b1 = W1 + (int64_t)H * D, *W2 = b1 + H, *b2 = W2 + (int64_t)H * H;
    const float *W3 = b2 + H, *b3 = W3 + 2 * H;
    for (int o = tid; o < H; o += NT) {
      float s = b1[o];
      for (int i = 0; i < D; ++i) s = fmaf(mf[i], W1[(int64_t)o * D + i], s);
      mh1[o] = s > 0.0f ? s : 0.0f;
    }
    __syncthreads();
    for (int o = tid; o < H; o += NT) {
      float s = b2[o];
      for (int i = 0; i < H; ++i) s = fmaf(mh1[i], W2[(int64_t)o * H + i], s);
      mh2[o] = s > 0.0f ? s : 0.0f;
    }
    __syncthreads();
    if (tid < 2) {
      float s = b3[tid];
      for (int i = 0; i < H; ++i) s = fmaf(mh2[i], W3[(int64_t)tid * H + i], s);
      mo[tid] = s;
    }
    __syncthreads();
    const float sg = 1.0f / (1.0f + expf(-mo[0]));
    const double c = 0.5 + (a.mlp_cmax - 0.5) * (double)sg;
    for (int t = 2 + tid; t < a.sched_len; t += NT) const_cast<double *>(a.sched)[t] = c;
    if (tid == 0) {
      state->learned_ready = 1;
      const float ln = mo[1];
      state->learned_n = ln > 0.0f && ln < 10.0f ? (int32_t)lrintf(expf(ln)) : 0;
    }
    __syncthreads();
  }
  if (j - 1 < a.trace_cap) {
    for (int i = tid; i < l; i += NT) a.trace_s[(int64_t)(j - 1) * l + i] = Ssh[i];
  }
  if (!s_stop) {
    for (int i = tid; i < l; i += NT) a.Sprev[i] = Ssh[i];
  }
  if (tid == 0) {
    const double ratio = s_ratio;
    if (j - 1 < a.trace_cap) {
      a.trace_alpha[j - 1] = alpha;
      a.trace_ratio[j - 1] = ratio;
    }
    state->pass = j;
    state->ratio = ratio;
    if (a.cq_switch > 0.0 && a.tol > 0.0 && ratio <= a.cq_switch * a.tol) state->cq_off = 1;
    if (s_stop) {
      // published at device scope: the transposed product of this pass,
      // running beside the eigensolver, stops early once it sees the flag
      __hip_atomic_store(&state->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      state->converged = 1;
      if (a.ndone) atomicAdd(a.ndone, 1);
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
      if (a.stagnation_guard && a.tol > 0.0) {
        // the check keeps failing and the ratio has reached a plateau (less
        // than 20 % gained in a pass): the BF16 panels limit the attainable
        // accuracy.  Ordinary convergence gains ~45 % per pass or more.
        const bool stag = j >= 2 && ratio > 0.8 * state->prev_ratio;
        state->stagnant = stag ? state->stagnant + 1 : 0;
        if (state->stagnant >= 2 && !state->promote) {
          state->promote = 1;
          if (a.ndone) atomicAdd(a.ndone + 1, 1);  // batched form: promotions so far
        }
      }
      state->prev_ratio = ratio;
      state->alpha_prev = a.pve_mode == 1 ? na : alpha;
      state->alpha = na;
    }
  }
}

}  // namespace dsv
