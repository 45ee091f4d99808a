// Small MLP (8 -> 64 -> 64 -> 1, tanh, FP32) that predicts per-vector
// convergence of the Chebyshev filter from the solver's own logs: forward,
// backward (mean squared error), gradient reduction and Adam, each a
// hand-written kernel.  Gradients are summed in a fixed order, so training
// is deterministic.
//
// Parameter blob (floats), shared with the host code and the CPU oracle:
//   [0, 8)      feature mean            [8, 16)     feature scale (std)
//   [16, 528)   W1 (64 x 8, row-major)  [528, 592)  b1
//   [592, 4688) W2 (64 x 64, row-major) [4688, 4752) b2
//   [4752, 4816) w3                     [4816]      b3
//   [4817]      degree margin (set from held-out data, not trained)
#include "internal.h"

namespace chfsi {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ void layer1(const float* prm, const float* x, float* z, float* h1) {
  for (int i = 0; i < MLP_IN; ++i) {
    const float sd = prm[MLP_STD + i];
    z[i] = (x[i] - prm[MLP_MEAN + i]) / (sd > 0.f ? sd : 1.f);
  }
  for (int a = 0; a < MLP_H; ++a) {
    float s = prm[MLP_B1 + a];
    for (int i = 0; i < MLP_IN; ++i) s += prm[MLP_W1 + a * MLP_IN + i] * z[i];
    h1[a] = tanhf(s);
  }
}

// y[s] = MLP(X[s, :]); parameters staged in LDS.
__global__ void __launch_bounds__(NT) k_mlp_forward(int n, const float* X, const float* prm_g,
                                                    float* Y) {
  __shared__ float prm[MLP_PARAMS];
  for (int i = threadIdx.x; i < MLP_PARAMS; i += NT) prm[i] = prm_g[i];
  __syncthreads();
  const int s = blockIdx.x * NT + threadIdx.x;
  if (s >= n) return;
  float x[MLP_IN], z[MLP_IN], h1[MLP_H];
  for (int i = 0; i < MLP_IN; ++i) x[i] = X[(long)s * MLP_IN + i];
  layer1(prm, x, z, h1);
  float y = prm[MLP_B3];
  for (int a = 0; a < MLP_H; ++a) {
    float t = prm[MLP_B2 + a];
    for (int b = 0; b < MLP_H; ++b) t += prm[MLP_W2 + a * MLP_H + b] * h1[b];
    y += prm[MLP_W3 + a] * tanhf(t);
  }
  Y[s] = y;
}

// Per-sample forward and backward of the loss (1/n) sum (y - t)^2.
// Writes Z (n x 8), H1, H2, D1, D2 (n x 64: activations and the loss
// gradients with respect to the pre-activations) and dy (n), and the
// per-block partial sums of the squared error.
__global__ void __launch_bounds__(NT) k_mlp_fwd_bwd(int n, const float* X, const float* T,
                                                    const float* prm_g, float* Z, float* H1,
                                                    float* H2, float* D1, float* D2, float* DY,
                                                    float* loss_part) {
  __shared__ float prm[MLP_PARAMS];
  __shared__ float red[NT];
  for (int i = threadIdx.x; i < MLP_PARAMS; i += NT) prm[i] = prm_g[i];
  __syncthreads();
  const int s = blockIdx.x * NT + threadIdx.x;
  float sq = 0.f;
  if (s < n) {
    float x[MLP_IN], z[MLP_IN], h1[MLP_H];
    for (int i = 0; i < MLP_IN; ++i) x[i] = X[(long)s * MLP_IN + i];
    layer1(prm, x, z, h1);
    float y = prm[MLP_B3];
    for (int a = 0; a < MLP_H; ++a) {
      float t = prm[MLP_B2 + a];
      for (int b = 0; b < MLP_H; ++b) t += prm[MLP_W2 + a * MLP_H + b] * h1[b];
      const float h2 = tanhf(t);
      H2[(long)s * MLP_H + a] = h2;
      y += prm[MLP_W3 + a] * h2;
    }
    const float err = y - T[s];
    sq = err * err;
    const float dy = 2.f * err / (float)n;
    DY[s] = dy;
    float g1[MLP_H];
    for (int b = 0; b < MLP_H; ++b) g1[b] = 0.f;
    for (int a = 0; a < MLP_H; ++a) {
      const float h2 = H2[(long)s * MLP_H + a];
      const float d2 = dy * prm[MLP_W3 + a] * (1.f - h2 * h2);
      D2[(long)s * MLP_H + a] = d2;
      for (int b = 0; b < MLP_H; ++b) g1[b] += prm[MLP_W2 + a * MLP_H + b] * d2;
    }
    for (int b = 0; b < MLP_H; ++b) {
      D1[(long)s * MLP_H + b] = g1[b] * (1.f - h1[b] * h1[b]);
      H1[(long)s * MLP_H + b] = h1[b];
    }
    for (int i = 0; i < MLP_IN; ++i) Z[(long)s * MLP_IN + i] = z[i];
  }
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Gradient partial sums: thread p of grid row c adds the contributions of
// samples [c * MLP_CHUNK, (c + 1) * MLP_CHUNK) to parameter p, in sample
// order (W2 in k_mlp_grad_w2).  The chunk sums are then added in chunk
// order, so the result does not depend on scheduling.
__global__ void __launch_bounds__(NT) k_mlp_grad_partial(int n, const float* Z, const float* H1,
                                                         const float* H2, const float* D1,
                                                         const float* D2, const float* DY,
                                                         float* part) {
  const int p = blockIdx.x * NT + threadIdx.x;
  if (p >= MLP_PARAMS) return;
  const int s0 = blockIdx.y * MLP_CHUNK;
  const int s1 = min(n, s0 + MLP_CHUNK);
  float g = 0.f;
  if (p >= MLP_W1 && p < MLP_B1) {
    const int a = (p - MLP_W1) / MLP_IN, i = (p - MLP_W1) % MLP_IN;
    for (int s = s0; s < s1; ++s) g += D1[(long)s * MLP_H + a] * Z[(long)s * MLP_IN + i];
  } else if (p >= MLP_B1 && p < MLP_W2) {
    const int a = p - MLP_B1;
    for (int s = s0; s < s1; ++s) g += D1[(long)s * MLP_H + a];
  } else if (p >= MLP_W2 && p < MLP_B2) {
    return;   // k_mlp_grad_w2
  } else if (p >= MLP_B2 && p < MLP_W3) {
    const int a = p - MLP_B2;
    for (int s = s0; s < s1; ++s) g += D2[(long)s * MLP_H + a];
  } else if (p >= MLP_W3 && p < MLP_B3) {
    const int a = p - MLP_W3;
    for (int s = s0; s < s1; ++s) g += DY[s] * H2[(long)s * MLP_H + a];
  } else if (p == MLP_B3) {
    for (int s = s0; s < s1; ++s) g += DY[s];
  }
  part[(long)blockIdx.y * MLP_PARAMS + p] = g;   // 0 for the statistics and the margin
}

// W2 part of the same partial sums: G[a][b] = sum_s D2[s][a] H1[s][b] over
// the chunk's samples.  The chunk's D2 and H1 rows are staged through LDS
// 64 samples at a time; thread t accumulates the 4 x 4 block of (a, b)
// with a = 4 (t / 16) + i, b = 4 (t % 16) + j, samples in order.
__global__ void __launch_bounds__(NT) k_mlp_grad_w2(int n, const float* H1, const float* D2,
                                                    float* part) {
  constexpr int TS = 64;
  __shared__ float d2s[TS][MLP_H + 1];
  __shared__ float h1s[TS][MLP_H + 1];
  const int t = threadIdx.x;
  const int a0 = 4 * (t >> 4), b0 = 4 * (t & 15);
  const int s0 = blockIdx.x * MLP_CHUNK;
  const int s1 = min(n, s0 + MLP_CHUNK);
  float acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
  for (int base = s0; base < s1; base += TS) {
    const int cnt = min(TS, s1 - base);
    for (int e = t; e < TS * MLP_H; e += NT) {
      const int r = e / MLP_H, c = e % MLP_H;
      const bool in = r < cnt;
      d2s[r][c] = in ? D2[(long)(base + r) * MLP_H + c] : 0.f;
      h1s[r][c] = in ? H1[(long)(base + r) * MLP_H + c] : 0.f;
    }
    __syncthreads();
    for (int r = 0; r < cnt; ++r) {
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = d2s[r][a0 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = h1s[r][b0 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
  float* out = part + (long)blockIdx.x * MLP_PARAMS + MLP_W2;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) out[(a0 + i) * MLP_H + b0 + j] = acc[i][j];
}

__global__ void __launch_bounds__(NT) k_mlp_grad_final(int chunks, const float* part, float* G) {
  const int p = blockIdx.x * NT + threadIdx.x;
  if (p >= MLP_PARAMS) return;
  float g = 0.f;
  for (int c = 0; c < chunks; ++c) g += part[(long)c * MLP_PARAMS + p];
  G[p] = g;
}

__global__ void k_mlp_loss_sum(int nparts, const float* part, float* out) {
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < nparts; ++i) s += part[i];
    out[0] = s;
  }
}

// Adam on the trained entries [MLP_W1, MLP_B3].
__global__ void k_mlp_adam(float* prm, const float* G, float* M, float* V, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * NT + threadIdx.x;
  if (p < MLP_W1 || p > MLP_B3) return;
  const float g = G[p];
  const float m = b1 * M[p] + (1.f - b1) * g;
  const float v = b2 * V[p] + (1.f - b2) * g * g;
  M[p] = m;
  V[p] = v;
  prm[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

}  // namespace

size_t mlp_grad_work_floats(int n) {
  const size_t blocks = (size_t)(n + NT - 1) / NT;
  const size_t chunks = (size_t)(n + MLP_CHUNK - 1) / MLP_CHUNK;
  return (size_t)n * (MLP_IN + 4 * MLP_H + 1) + blocks + chunks * MLP_PARAMS + 64;
}

int mlp_forward(hipStream_t s, int n, const float* X, const float* prm, float* Y) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_mlp_forward, dim3((n + NT - 1) / NT), dim3(NT), 0, s, n, X, prm, Y);
  return (int)hipGetLastError();
}

int mlp_gradient(hipStream_t s, int n, const float* X, const float* T, const float* prm,
                 float* G, float* loss_dev, float* work) {
  if (n <= 0) return (int)hipErrorInvalidValue;
  const int blocks = (n + NT - 1) / NT;
  const int chunks = (n + MLP_CHUNK - 1) / MLP_CHUNK;
  const int pblocks = (MLP_PARAMS + NT - 1) / NT;
  float* Z = work;
  float* H1 = Z + (size_t)n * MLP_IN;
  float* H2 = H1 + (size_t)n * MLP_H;
  float* D1 = H2 + (size_t)n * MLP_H;
  float* D2 = D1 + (size_t)n * MLP_H;
  float* DY = D2 + (size_t)n * MLP_H;
  float* lpart = DY + n;
  float* gpart = lpart + blocks;
  hipLaunchKernelGGL(k_mlp_fwd_bwd, dim3(blocks), dim3(NT), 0, s, n, X, T, prm, Z, H1, H2, D1, D2,
                     DY, lpart);
  int e = (int)hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_mlp_grad_partial, dim3(pblocks, chunks), dim3(NT), 0, s, n,
                     (const float*)Z, (const float*)H1, (const float*)H2, (const float*)D1,
                     (const float*)D2, (const float*)DY, gpart);
  e = (int)hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_mlp_grad_w2, dim3(chunks), dim3(NT), 0, s, n, (const float*)H1,
                     (const float*)D2, gpart);
  e = (int)hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_mlp_grad_final, dim3(pblocks), dim3(NT), 0, s, chunks, (const float*)gpart,
                     G);
  e = (int)hipGetLastError();
  if (e) return e;
  hipLaunchKernelGGL(k_mlp_loss_sum, dim3(1), dim3(64), 0, s, blocks, (const float*)lpart,
                     loss_dev);
  return (int)hipGetLastError();
}

int mlp_adam(hipStream_t s, float* prm, const float* G, float* M, float* V, float lr, int t) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_PARAMS + NT - 1) / NT), dim3(NT), 0, s, prm, G, M, V, lr,
                     b1, b2, 1e-8f, c1, c2);
  return (int)hipGetLastError();
}

}  // namespace chfsi
