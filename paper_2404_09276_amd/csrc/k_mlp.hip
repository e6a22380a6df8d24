// Learned shift proposal: a small MLP (features of passes 1-2 -> shift
// multiplier c for the later passes and a predicted pass count), trained and
// evaluated with the kernels below.  The paper sets the shift by a fixed rule
// (Alg. 5 step 6); this model proposes c_j in alpha_j = c_j E_l(j-1), and the
// PVE check still decides termination.
//
// Network: x (D) -> relu(W1 x + b1) (H) -> relu(W2 . + b2) (H) -> W3 . + b3
// (2 outputs o).  c = 0.5 + (c_max - 0.5) sigmoid(o_0); log N = o_1.
// Parameters are one FP32 vector: W1 (H x D), b1, W2 (H x H), b2, W3 (2 x H),
// b3, row-major.  All products accumulate in FP32 in a fixed order, so
// results repeat bit for bit.
//
// Loss of a batch of B samples with targets (c*, log N*):
//   L = (1/B) sum_b [ (c_b - c*_b)^2 + lambda (o1_b - log N*_b)^2 ].
#include "common.h"

namespace dsv {

namespace {

constexpr int kMT = 256;

// Y[b, o] = act(sum_i X[b, i] W[o, i] + bias[o]), act = relu or identity
__global__ __launch_bounds__(kMT) void k_dense_fwd(const float *__restrict__ X, int B, int Din,
                                                   const float *__restrict__ W, const float *__restrict__ bias,
                                                   int Dout, int relu, float *__restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * kMT + threadIdx.x;
  if (t >= (int64_t)B * Dout) return;
  const int b = (int)(t / Dout), o = (int)(t - (int64_t)b * Dout);
  const float *x = X + (int64_t)b * Din, *w = W + (int64_t)o * Din;
  float s = bias[o];
  for (int i = 0; i < Din; ++i) s = fmaf(x[i], w[i], s);
  Y[t] = relu ? (s > 0.0f ? s : 0.0f) : s;
}

// Head and loss: per-sample loss terms and dL/do.  One block sums the loss
// in a fixed order.
__global__ __launch_bounds__(kMT) void k_head_loss(const float *__restrict__ O, const float *__restrict__ T, int B,
                                                   float cmax, float lambda, float *__restrict__ dO,
                                                   float *__restrict__ loss) {
  __shared__ float part[kMT];
  float acc = 0.0f;
  for (int b = threadIdx.x; b < B; b += kMT) {
    const float o0 = O[2 * b], o1 = O[2 * b + 1];
    const float sg = 1.0f / (1.0f + expf(-o0));
    const float c = 0.5f + (cmax - 0.5f) * sg;
    const float e0 = c - T[2 * b], e1 = o1 - T[2 * b + 1];
    acc += e0 * e0 + lambda * e1 * e1;
    dO[2 * b] = 2.0f * e0 * (cmax - 0.5f) * sg * (1.0f - sg) / (float)B;
    dO[2 * b + 1] = 2.0f * lambda * e1 / (float)B;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kMT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] / (float)B;
}

// dW[o, i] = sum_b dY[b, o] X[b, i], db[o] = sum_b dY[b, o] (thread i = Din
// computes db)
__global__ __launch_bounds__(kMT) void k_dense_bwd_w(const float *__restrict__ dY, const float *__restrict__ X,
                                                     int B, int Din, int Dout, float *__restrict__ dW,
                                                     float *__restrict__ db) {
  const int64_t t = (int64_t)blockIdx.x * kMT + threadIdx.x;
  if (t >= (int64_t)Dout * (Din + 1)) return;
  const int o = (int)(t / (Din + 1)), i = (int)(t - (int64_t)o * (Din + 1));
  float s = 0.0f;
  if (i < Din) {
    for (int b = 0; b < B; ++b) s = fmaf(dY[(int64_t)b * Dout + o], X[(int64_t)b * Din + i], s);
    dW[(int64_t)o * Din + i] = s;
  } else {
    for (int b = 0; b < B; ++b) s += dY[(int64_t)b * Dout + o];
    db[o] = s;
  }
}

// dX[b, i] = (sum_o dY[b, o] W[o, i]) * [A[b, i] > 0], A the relu output
// that fed the layer
__global__ __launch_bounds__(kMT) void k_dense_bwd_x(const float *__restrict__ dY, const float *__restrict__ W,
                                                     const float *__restrict__ A, int B, int Din, int Dout,
                                                     float *__restrict__ dX) {
  const int64_t t = (int64_t)blockIdx.x * kMT + threadIdx.x;
  if (t >= (int64_t)B * Din) return;
  const int b = (int)(t / Din), i = (int)(t - (int64_t)b * Din);
  float s = 0.0f;
  for (int o = 0; o < Dout; ++o) s = fmaf(dY[(int64_t)b * Dout + o], W[(int64_t)o * Din + i], s);
  dX[t] = A[t] > 0.0f ? s : 0.0f;
}

// Adam (Kingma & Ba) with bias correction; step t >= 1
__global__ __launch_bounds__(kMT) void k_adam(float *__restrict__ P, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, int64_t n, float lr,
                                              float b1, float b2, float eps, int t) {
  const int64_t i = (int64_t)blockIdx.x * kMT + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - powf(b1, (float)t));
  const float vh = vi / (1.0f - powf(b2, (float)t));
  P[i] -= lr * mh / (sqrtf(vh) + eps);
}

unsigned nb(int64_t work) { return (unsigned)((work + kMT - 1) / kMT); }

}  // namespace

hipError_t mlp_forward(const MlpDims &d, const float *P, const float *X, int B, float *A1, float *A2, float *O,
                       hipStream_t st) {
  if (B < 1) return hipSuccess;
  const float *W1 = P, *b1 = W1 + (int64_t)d.H * d.D, *W2 = b1 + d.H, *b2 = W2 + (int64_t)d.H * d.H;
  const float *W3 = b2 + d.H, *b3 = W3 + 2 * d.H;
  hipLaunchKernelGGL(k_dense_fwd, dim3(nb((int64_t)B * d.H)), dim3(kMT), 0, st, X, B, d.D, W1, b1, d.H, 1, A1);
  hipLaunchKernelGGL(k_dense_fwd, dim3(nb((int64_t)B * d.H)), dim3(kMT), 0, st, A1, B, d.H, W2, b2, d.H, 1, A2);
  hipLaunchKernelGGL(k_dense_fwd, dim3(nb((int64_t)B * 2)), dim3(kMT), 0, st, A2, B, d.H, W3, b3, 2, 0, O);
  return hipGetLastError();
}

hipError_t mlp_backward(const MlpDims &d, const float *P, const float *X, const float *T, int B, float cmax,
                        float lambda, float *A1, float *A2, float *O, float *dO, float *dA2, float *dA1, float *G,
                        float *loss, hipStream_t st) {
  hipError_t e = mlp_forward(d, P, X, B, A1, A2, O, st);
  if (e != hipSuccess) return e;
  const float *W2 = P + (int64_t)d.H * d.D + d.H, *W3 = W2 + (int64_t)d.H * d.H + d.H;
  float *gW1 = G, *gb1 = gW1 + (int64_t)d.H * d.D, *gW2 = gb1 + d.H, *gb2 = gW2 + (int64_t)d.H * d.H;
  float *gW3 = gb2 + d.H, *gb3 = gW3 + 2 * d.H;
  hipLaunchKernelGGL(k_head_loss, dim3(1), dim3(kMT), 0, st, O, T, B, cmax, lambda, dO, loss);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb(2 * (int64_t)(d.H + 1))), dim3(kMT), 0, st, dO, A2, B, d.H, 2, gW3, gb3);
  hipLaunchKernelGGL(k_dense_bwd_x, dim3(nb((int64_t)B * d.H)), dim3(kMT), 0, st, dO, W3, A2, B, d.H, 2, dA2);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb((int64_t)d.H * (d.H + 1))), dim3(kMT), 0, st, dA2, A1, B, d.H, d.H, gW2,
                     gb2);
  hipLaunchKernelGGL(k_dense_bwd_x, dim3(nb((int64_t)B * d.H)), dim3(kMT), 0, st, dA2, W2, A1, B, d.H, d.H, dA1);
  hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb((int64_t)d.H * (d.D + 1))), dim3(kMT), 0, st, dA1, X, B, d.D, d.H, gW1,
                     gb1);
  return hipGetLastError();
}

hipError_t mlp_adam(float *P, const float *G, float *m, float *v, int64_t n, float lr, int t, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(nb(n)), dim3(kMT), 0, st, P, G, m, v, n, lr, 0.9f, 0.999f, 1e-8f, t);
  return hipGetLastError();
}

}  // namespace dsv
