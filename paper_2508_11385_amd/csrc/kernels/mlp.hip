// Kernels of the learned launch-configuration cost model: a 3-Linear-layer ReLU
// network (in -> H1 -> H2 -> 1) trained with masked mean-squared error and Adam,
// all in binary32.  Row-major activations (sample-major), weights W[out][in].
// Every sum runs in a fixed order (one thread per output, sequential loop), so
// results do not depend on timing.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

// Z[b][o] = bias[o] + sum_k X[b][k] * W[o][k];  A = relu(Z) if relu else Z.
__global__ __launch_bounds__(256) void dense_fwd(const float* __restrict__ X, int B, int K, const float* __restrict__ W,
                                                 const float* __restrict__ bias, int O, float* __restrict__ Z,
                                                 float* __restrict__ A, int relu) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * O) return;
  const int b = idx / O, o = idx % O;
  const float* x = X + (size_t)b * K;
  const float* w = W + (size_t)o * K;
  float z = bias[o];
  for (int k = 0; k < K; ++k) z = __builtin_fmaf(x[k], w[k], z);
  Z[idx] = z;
  A[idx] = relu ? (z > 0.0f ? z : 0.0f) : z;
}

// dZ[b] = 2 m_b (out_b - y_b) * inv_count   (output layer, O = 1); loss terms to L[b].
__global__ __launch_bounds__(256) void mse_grad(const float* __restrict__ out, const float* __restrict__ y,
                                                const float* __restrict__ mask, int B, float inv_count,
                                                float* __restrict__ dZ, float* __restrict__ L) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const float d = out[b] - y[b];
  dZ[b] = 2.0f * mask[b] * d * inv_count;
  L[b] = mask[b] * d * d * inv_count;
}

// Sum of L[0..B) into *loss (one workgroup, fixed order).
__global__ __launch_bounds__(256) void sum_into(const float* __restrict__ L, int B, float* __restrict__ loss) {
  __shared__ float s[256];
  float a = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) a += L[b];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = s[0];
}

// dW[o][k] = sum_b dZ[b][o] * A[b][k];  db[o] = sum_b dZ[b][o]  (one thread per (o, k); k == K does db)
__global__ __launch_bounds__(256) void dense_wgrad(const float* __restrict__ dZ, const float* __restrict__ A, int B,
                                                   int K, int O, float* __restrict__ dW, float* __restrict__ db) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= O * (K + 1)) return;
  const int o = idx / (K + 1), k = idx % (K + 1);
  float g = 0.0f;
  if (k < K) {
    for (int b = 0; b < B; ++b) g = __builtin_fmaf(dZ[(size_t)b * O + o], A[(size_t)b * K + k], g);
    dW[(size_t)o * K + k] = g;
  } else {
    for (int b = 0; b < B; ++b) g += dZ[(size_t)b * O + o];
    db[o] = g;
  }
}

// dZp[b][k] = (sum_o dZ[b][o] * W[o][k]) * (Zp[b][k] > 0)   (gradient through the previous ReLU)
__global__ __launch_bounds__(256) void dense_xgrad(const float* __restrict__ dZ, const float* __restrict__ W, int B,
                                                   int K, int O, const float* __restrict__ Zp,
                                                   float* __restrict__ dZp) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= B * K) return;
  const int b = idx / K, k = idx % K;
  float g = 0.0f;
  for (int o = 0; o < O; ++o) g = __builtin_fmaf(dZ[(size_t)b * O + o], W[(size_t)o * K + k], g);
  dZp[idx] = Zp[idx] > 0.0f ? g : 0.0f;
}

// Adam with bias correction: c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ __launch_bounds__(256) void adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                                            float* __restrict__ V, int n, float lr, float b1, float b2, float eps,
                                            float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = b1 * M[i] + (1.0f - b1) * g;
  const float v = b2 * V[i] + (1.0f - b2) * g * g;
  M[i] = m;
  V[i] = v;
  const float mh = m / c1, vh = v / c2;
  P[i] = P[i] - lr * mh / (__builtin_sqrtf(vh) + eps);
}

// Xb[r][k] = X[idx[r]][k], yb[r] = y[idx[r]], mb[r] = mask[idx[r]]
__global__ __launch_bounds__(256) void gather_rows(const float* __restrict__ X, const float* __restrict__ y,
                                                   const float* __restrict__ mask, const int* __restrict__ idx, int B,
                                                   int K, float* __restrict__ Xb, float* __restrict__ yb,
                                                   float* __restrict__ mb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * (K + 1)) return;
  const int r = t / (K + 1), k = t % (K + 1);
  const int src = idx[r];
  if (k < K) {
    Xb[(size_t)r * K + k] = X[(size_t)src * K + k];
  } else {
    yb[r] = y[src];
    mb[r] = mask[src];
  }
}

inline unsigned blocks(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" {

hipError_t coot_mlp_k_dense_fwd(const float* X, int B, int K, const float* W, const float* bias, int O, float* Z,
                                float* A, int relu, hipStream_t s) {
  if (B * O == 0) return hipSuccess;
  hipLaunchKernelGGL(dense_fwd, dim3(blocks((long)B * O)), dim3(256), 0, s, X, B, K, W, bias, O, Z, A, relu);
  return hipGetLastError();
}

hipError_t coot_mlp_k_mse_grad(const float* out, const float* y, const float* mask, int B, float inv_count,
                               float* dZ, float* L, float* loss, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(mse_grad, dim3(blocks(B)), dim3(256), 0, s, out, y, mask, B, inv_count, dZ, L);
  if (loss) hipLaunchKernelGGL(sum_into, dim3(1), dim3(256), 0, s, (const float*)L, B, loss);
  return hipGetLastError();
}

hipError_t coot_mlp_k_dense_bwd(const float* dZ, const float* A, const float* W, int B, int K, int O, float* dW,
                                float* db, const float* Zp, float* dZp, hipStream_t s) {
  hipLaunchKernelGGL(dense_wgrad, dim3(blocks((long)O * (K + 1))), dim3(256), 0, s, dZ, A, B, K, O, dW, db);
  if (dZp && B * K) hipLaunchKernelGGL(dense_xgrad, dim3(blocks((long)B * K)), dim3(256), 0, s, dZ, W, B, K, O, Zp, dZp);
  return hipGetLastError();
}

hipError_t coot_mlp_k_adam(float* P, const float* G, float* M, float* V, int n, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(adam, dim3(blocks(n)), dim3(256), 0, s, P, G, M, V, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t coot_mlp_k_gather(const float* X, const float* y, const float* mask, const int* idx, int B, int K,
                             float* Xb, float* yb, float* mb, hipStream_t s) {
  hipLaunchKernelGGL(gather_rows, dim3(blocks((long)B * (K + 1))), dim3(256), 0, s, X, y, mask, idx, B, K, Xb, yb, mb);
  return hipGetLastError();
}

}  // extern "C"
