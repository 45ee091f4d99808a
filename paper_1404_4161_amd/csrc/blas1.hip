// Memory-bound helper kernels of the ChFSI path: column norms and residual
// norms (wave64 reductions in a fixed order, so results are bitwise
// repeatable), column gathers and permutations, Hermitian fills, the
// Cholesky leaf, Lanczos vector operations and the SplitMix64 start block.
#include "internal.h"

namespace chfsi {

namespace {

constexpr int NT = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum over the 256 threads of a block, fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

__device__ __forceinline__ zc block_sum_c(zc v, double* red) {
  double re = wave_sum(v.x), im = wave_sum(v.y);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[w] = re;
    red[4 + w] = im;
  }
  __syncthreads();
  zc s = zc{0.0, 0.0};
  if (threadIdx.x == 0) {
    s.x = (red[0] + red[1]) + (red[2] + red[3]);
    s.y = (red[4] + red[5]) + (red[6] + red[7]);
  }
  __syncthreads();
  return s;
}

__global__ void k_col_norms(int n, const zc* X, long ldx, double* out) {
  __shared__ double red[8];
  const zc* x = X + (long)blockIdx.x * ldx;
  double s = 0.0;
  for (int r = threadIdx.x; r < n; r += NT) {
    const zc v = x[r];
    s += v.x * v.x + v.y * v.y;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(s);
}

__global__ void k_resid_norms(int n, const zc* Q, long ldq, const zc* Z, long ldz,
                              const double* mu, double* out) {
  __shared__ double red[8];
  const int j = blockIdx.x;
  const zc* q = Q + (long)j * ldq;
  const zc* z = Z + (long)j * ldz;
  const double m = mu[j];
  double s = 0.0;
  for (int r = threadIdx.x; r < n; r += NT) {
    const zc a = z[r], b = q[r];
    const double dr = a.x - m * b.x, di = a.y - m * b.y;
    s += dr * dr + di * di;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[j] = sqrt(s);
}

__global__ void k_scale_cols_inv(int n, zc* X, long ldx, const double* nrm) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  const double f = 1.0 / nrm[blockIdx.y];
  zc* p = X + r + (long)blockIdx.y * ldx;
  zc v = *p;
  v.x *= f;
  v.y *= f;
  *p = v;
}

__global__ void k_gather_cols(int n, const zc* src, long lds, zc* dst, long ldd, const int* perm) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  dst[r + (long)blockIdx.y * ldd] = src[r + (long)perm[blockIdx.y] * lds];
}

__global__ void k_gather_parity(int n, const zc* P0, const zc* P1, long ldp, zc* dst, long ldd,
                                const int* deg) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  const int j = blockIdx.y;
  const zc* src = (deg[j] & 1) ? P1 : P0;
  dst[r + (long)j * ldd] = src[r + (long)j * ldp];
}

__global__ void k_copy2d(int rows, const zc* src, long lds, zc* dst, long ldd) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= rows) return;
  dst[r + (long)blockIdx.y * ldd] = src[r + (long)blockIdx.y * lds];
}

__global__ void k_herm_from_lower(int k, zc* G, long ldg) {
  const int r = blockIdx.x * NT + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= k) return;
  if (r < c) {
    const zc v = G[c + (long)r * ldg];
    G[r + (long)c * ldg] = zc{v.x, -v.y};
  } else if (r == c) {
    G[r + (long)c * ldg].y = 0.0;
  }
}

// scale (H + H^H) on 32x32 tile pairs (bi >= bj) through LDS.
__global__ void k_symmetrize(int n, zc* H, long ldh, double scale) {
  __shared__ zc a[32][33], b[32][33];
  const int bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  // a = tile (bi, bj), b = tile (bj, bi); stored [col][row]
  for (int c = ty; c < 32; c += 8) {
    const int row_a = bi * 32 + tx, col_a = bj * 32 + c;
    if (row_a < n && col_a < n) a[c][tx] = H[row_a + (long)col_a * ldh];
    const int row_b = bj * 32 + tx, col_b = bi * 32 + c;
    if (row_b < n && col_b < n) b[c][tx] = H[row_b + (long)col_b * ldh];
  }
  __syncthreads();
  for (int c = ty; c < 32; c += 8) {
    // a(r, c) pairs with b(c, r)
    const int row_a = bi * 32 + tx, col_a = bj * 32 + c;
    const int row_b = bj * 32 + tx, col_b = bi * 32 + c;
    if (row_a < n && col_a < n) {
      const zc x = a[c][tx], y = b[tx][c];
      H[row_a + (long)col_a * ldh] = zc{scale * (x.x + y.x), scale * (x.y - y.y)};
    }
    if (row_b < n && col_b < n) {
      const zc x = b[c][tx], y = a[tx][c];
      H[row_b + (long)col_b * ldh] = zc{scale * (x.x + y.x), scale * (x.y - y.y)};
    }
  }
}

// ||G - I||_F of a k x k matrix: one workgroup of 1024 threads, partial
// sums in a fixed order (repeatable).
__global__ void __launch_bounds__(1024) k_gram_offnorm(int k, const zc* G, long ldg, double* out) {
  __shared__ double red[1024];
  const int t = threadIdx.x;
  double acc = 0.0;
  const long total = (long)k * k;
  for (long e = t; e < total; e += 1024) {
    const int r = (int)(e % k), c = (int)(e / k);
    zc v = G[r + (long)c * ldg];
    if (r == c) v.x -= 1.0;
    acc += v.x * v.x + v.y * v.y;
  }
  red[t] = acc;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) out[0] = sqrt(red[0]);
}

// D = tril(A) with the diagonal halved (zero above the diagonal).
__global__ void k_lower_half_diag(int n, const zc* A, long lda, zc* D, long ldd) {
  const int r = blockIdx.x * NT + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= n) return;
  zc v = zc{0.0, 0.0};
  if (r > c) v = A[r + (long)c * lda];
  else if (r == c) {
    const zc d = A[r + (long)c * lda];
    v = zc{0.5 * d.x, 0.5 * d.y};
  }
  D[r + (long)c * ldd] = v;
}

__global__ void k_conj_transpose(int n, const zc* src, long lds, zc* dst, long ldd) {
  __shared__ zc t[32][33];
  const int bi = blockIdx.x, bj = blockIdx.y;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int c = ty; c < 32; c += 8) {
    const int row = bi * 32 + tx, col = bj * 32 + c;
    if (row < n && col < n) t[c][tx] = src[row + (long)col * lds];
  }
  __syncthreads();
  for (int c = ty; c < 32; c += 8) {
    // dst(bj*32 + tx, bi*32 + c) = conj(src(bi*32 + c, bj*32 + tx))
    const int row = bj * 32 + tx, col = bi * 32 + c;
    if (row < n && col < n) {
      const zc v = t[tx][c];
      dst[row + (long)col * ldd] = zc{v.x, -v.y};
    }
  }
}

__global__ void k_zero_upper(int n, zc* L, long ldl) {
  const int r = blockIdx.x * NT + threadIdx.x;
  const int c = blockIdx.y;
  if (r < c && r < n) L[r + (long)c * ldl] = zc{0.0, 0.0};
}

__global__ void k_set_identity(int n, zc* X, long ldx) {
  const int r = blockIdx.x * NT + threadIdx.x;
  const int c = blockIdx.y;
  if (r < n) X[r + (long)c * ldx] = zc{r == c ? 1.0 : 0.0, 0.0};
}

__global__ void k_add_diag(int n, zc* G, long ldg, double v) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r < n) G[r + (long)r * ldg].x += v;
}

__global__ void k_check_finite(int rows, const zc* X, long ldx, int* flag) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= rows) return;
  const zc v = X[r + (long)blockIdx.y * ldx];
  if (!isfinite(v.x) || !isfinite(v.y)) *flag = 1;
}

__device__ __forceinline__ unsigned long long splitmix_mix(unsigned long long z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

__device__ __forceinline__ double splitmix_uniform(unsigned long long base, unsigned long long i) {
  const unsigned long long x = splitmix_mix(base + (i + 1ull) * 0x9E3779B97F4A7C15ull);
  return (double)(x >> 11) * 0x1.0p-53;
}

__global__ void k_fill_random(int n, zc* X, long ldx, unsigned long long base) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  const unsigned long long p = (unsigned long long)r + (unsigned long long)blockIdx.y * n;
  X[r + (long)blockIdx.y * ldx] =
      zc{splitmix_uniform(base, 2 * p) - 0.5, splitmix_uniform(base, 2 * p + 1) - 0.5};
}

__global__ void k_add_random(int n, zc* X, long ldx, unsigned long long base, double eps) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  const unsigned long long p = (unsigned long long)r + (unsigned long long)blockIdx.y * n;
  zc* x = X + r + (long)blockIdx.y * ldx;
  zc v = *x;
  v.x += eps * (splitmix_uniform(base, 2 * p) - 0.5);
  v.y += eps * (splitmix_uniform(base, 2 * p + 1) - 0.5);
  *x = v;
}

// Order-independent 64-bit fingerprint of a matrix: the wrapping sum over
// entries of SplitMix64-mixed (bits, position) words.  Integer addition is
// associative, so the value does not depend on the reduction order.
__device__ __forceinline__ unsigned long long entry_hash(zc v, unsigned long long p) {
  const unsigned long long re = (unsigned long long)__double_as_longlong(v.x);
  const unsigned long long im = (unsigned long long)__double_as_longlong(v.y);
  return splitmix_mix(re ^ splitmix_mix(2 * p + 1)) + splitmix_mix(im ^ splitmix_mix(2 * p + 2));
}

__global__ void k_hash_part(int rows, int cols, const zc* X, long ldx, unsigned long long* part) {
  __shared__ unsigned long long red[NT];
  unsigned long long h = 0;
  const long total = (long)rows * cols;
  for (long i = (long)blockIdx.x * NT + threadIdx.x; i < total; i += (long)gridDim.x * NT) {
    const int r = (int)(i % rows), c = (int)(i / rows);
    h += entry_hash(X[r + (long)c * ldx], (unsigned long long)i);
  }
  red[threadIdx.x] = h;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_hash_sum(int nparts, const unsigned long long* part, unsigned long long* out) {
  if (threadIdx.x == 0) {
    unsigned long long h = 0;
    for (int i = 0; i < nparts; ++i) h += part[i];
    out[0] = h;
  }
}

__global__ void k_fill_zero(size_t count, zc* X) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i < count) X[i] = zc{0.0, 0.0};
}

// Cholesky of one nb x nb (nb <= 64) diagonal block in LDS, right-looking
// (1024 threads: thread t owns row t % 64 and the columns (t / 64) + 16 q,
// q = 0..3; two barriers per column), plus the inverse of the factor by
// forward substitution, 16 threads per column of the inverse.  A pivot d_j
// <= rel_tol * (original diagonal entry j) counts as a breakdown.
//
// The pivot of column j (its square root and reciprocal) is computed once,
// by the thread that applies the last update to entry (j, j) -- during the
// update of column j - 1 -- and published in LDS with that column's
// barrier; the other threads only read it (FP64 square roots and divisions
// repeated by all 16 waves would cost more than the factorisation itself).
__global__ void __launch_bounds__(1024) k_potrf_leaf(int nb, zc* G, long ldg, zc* inv, int* info,
                                                     int col_offset, double rel_tol) {
  __shared__ zc S[64][65];    // S[col][row]
  __shared__ double D0[64];
  __shared__ double Pi[64];   // 1 / L(j, j)
  __shared__ int bad;
  const int t = threadIdx.x;
  const int r = t & 63, cg = t >> 6;   // row, column group (16 groups of 4 columns)
  // pivot of column j from its final diagonal value d (one thread per column;
  // columns are separated by barriers, so `bad` keeps the first breakdown)
  auto pivot = [&](int j, double d) {
    if (!(d > rel_tol * D0[j]) || !(d > 0.0) || !isfinite(d)) {
      if (bad == 0) bad = j + 1;
      d = 1.0;
    }
    const double l = sqrt(d);
    Pi[j] = 1.0 / l;
    S[j][j] = zc{l, 0.0};
  };
  if (t == 0) bad = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = cg + 16 * q;
    if (r < nb && c < nb) {
      const zc v = (r >= c) ? G[r + (long)c * ldg] : zc{0.0, 0.0};
      S[c][r] = v;
      if (r == c) {
        D0[r] = fabs(v.x);
        if (r == 0) pivot(0, v.x);   // thread 0 holds entry (0, 0)
      }
    }
  }
  __syncthreads();
  // right-looking factorisation; per column j every thread first reads what
  // it needs of column j (scaled in registers), then, after a barrier, the
  // scaled column is written and the trailing lower triangle updated:
  // S(r, p) -= L(r, j) conj(L(p, j)), j < p <= r
  for (int j = 0; j < nb; ++j) {
    const double inv_l = Pi[j];
    const bool row_active = r > j && r < nb;
    zc a = zc{0.0, 0.0};
    zc bp[4];
    if (row_active) {
      const zc v = S[j][r];
      a = zc{v.x * inv_l, v.y * inv_l};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = cg + 16 * q;
        const zc w = (p > j && p <= r) ? S[j][p] : zc{0.0, 0.0};
        bp[q] = zc{w.x * inv_l, w.y * inv_l};
      }
    }
    __syncthreads();
    if (row_active) {
      if (cg == 0) S[j][r] = a;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = cg + 16 * q;
        if (p > j && p <= r) {
          const zc b = bp[q];
          zc v = S[p][r];
          v.x -= a.x * b.x + a.y * b.y;
          v.y -= a.y * b.x - a.x * b.y;
          S[p][r] = v;
          // entry (j + 1, j + 1) is final after this update
          if (p == r && r == j + 1) pivot(r, v.x);
        }
      }
    }
    __syncthreads();
  }
  // inverse X = inv(L) by columns, 16 threads per column: x_i = (delta_ic -
  // sum_{c <= k < i} L(i, k) x_k) / L(i, i), the sum split over the 16
  // threads (k = sub mod 16, their x_k kept in registers) and reduced by
  // shuffles; no barriers
  const int c = t >> 4, sub = t & 15;
  zc xr[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) xr[m] = zc{0.0, 0.0};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    for (int s = 0; s < 16; ++s) {
      const int i = 16 * m + s;
      zc part = zc{0.0, 0.0};
#pragma unroll
      for (int m2 = 0; m2 < 4; ++m2) {
        const int k = sub + 16 * m2;
        if (k >= c && k < i && i < nb) {
          const zc l = S[k][i];   // L(i, k)
          part.x += l.x * xr[m2].x - l.y * xr[m2].y;
          part.y += l.x * xr[m2].y + l.y * xr[m2].x;
        }
      }
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) {
        part.x += __shfl_xor(part.x, off, 16);
        part.y += __shfl_xor(part.y, off, 16);
      }
      if (i < nb && i >= c && s == sub) {
        const double f = Pi[i];
        xr[m] = zc{((i == c ? 1.0 : 0.0) - part.x) * f, -part.y * f};
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int cc = cg + 16 * q;
    if (r < nb && cc < nb) G[r + (long)cc * ldg] = S[cc][r];
  }
  if (c < nb) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int row = sub + 16 * m;
      if (row < nb) inv[row + (long)c * nb] = row >= c ? xr[m] : zc{0.0, 0.0};
    }
  }
  if (t == 0 && bad != 0 && *info == 0) *info = col_offset + bad;
}

// y_part[s][r] = sum over the s-th column chunk of H[r, k] x[k]
// T = zc (FP64 H) or cf (FP32 H, products and sums in FP64)
template <typename T>
__global__ void k_gemv_part(int n, const T* H, long ldh, const zc* x, zc* part, int chunk) {
  __shared__ zc xs[NT];
  const int r = blockIdx.x * NT + threadIdx.x;
  const int c0 = blockIdx.y * chunk;
  const int c1 = min(n, c0 + chunk);
  zc acc = zc{0.0, 0.0};
  for (int cb = c0; cb < c1; cb += NT) {
    const int cc = cb + threadIdx.x;
    xs[threadIdx.x] = cc < c1 ? x[cc] : zc{0.0, 0.0};
    __syncthreads();
    const int cnt = min(NT, c1 - cb);
    if (r < n) {
      for (int q = 0; q < cnt; ++q) {
        const T hv = H[r + (long)(cb + q) * ldh];
        const zc h = zc{(double)hv.x, (double)hv.y}, v = xs[q];
        acc.x += h.x * v.x - h.y * v.y;
        acc.y += h.x * v.y + h.y * v.x;
      }
    }
    __syncthreads();
  }
  if (r < n) part[(long)blockIdx.y * n + r] = acc;
}

__global__ void k_sum_parts(int n, int splits, const zc* part, zc* y) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  zc s = zc{0.0, 0.0};
  for (int p = 0; p < splits; ++p) {
    const zc v = part[(long)p * n + r];
    s.x += v.x;
    s.y += v.y;
  }
  y[r] = s;
}

// h[i] = V[:, i]^H w
__global__ void k_dots_c(int n, const zc* V, long ldv, const zc* w, zc* h) {
  __shared__ double red[8];
  const zc* v = V + (long)blockIdx.x * ldv;
  zc s = zc{0.0, 0.0};
  for (int r = threadIdx.x; r < n; r += NT) {
    const zc a = v[r], b = w[r];
    s.x += a.x * b.x + a.y * b.y;
    s.y += a.x * b.y - a.y * b.x;
  }
  s = block_sum_c(s, red);
  if (threadIdx.x == 0) h[blockIdx.x] = s;
}

// w -= V h (cnt columns)
__global__ void k_sub_vh(int n, int cnt, const zc* V, long ldv, const zc* h, zc* w) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  zc acc = w[r];
  for (int i = 0; i < cnt; ++i) {
    const zc a = V[r + (long)i * ldv], b = h[i];
    acc.x -= a.x * b.x - a.y * b.y;
    acc.y -= a.x * b.y + a.y * b.x;
  }
  w[r] = acc;
}

// alpha_j = Re h[j];  w -= alpha_j v_j + beta_{j-1} v_{j-1}
__global__ void k_lanczos_axpy(int n, int j, const zc* V, long ldv, const zc* h,
                               const double* betas, zc* w, double* alphas) {
  const int r = blockIdx.x * NT + threadIdx.x;
  const double a = h[j].x;
  if (r == 0) alphas[j] = a;
  if (r >= n) return;
  zc acc = w[r];
  const zc vj = V[r + (long)j * ldv];
  acc.x -= a * vj.x;
  acc.y -= a * vj.y;
  if (j > 0) {
    const double b = betas[j - 1];
    const zc vp = V[r + (long)(j - 1) * ldv];
    acc.x -= b * vp.x;
    acc.y -= b * vp.y;
  }
  w[r] = acc;
}

__global__ void k_normalize_into(int n, const zc* w, zc* v, double* beta_out) {
  __shared__ double red[8];
  __shared__ double nrm;
  double s = 0.0;
  for (int r = threadIdx.x; r < n; r += NT) {
    const zc a = w[r];
    s += a.x * a.x + a.y * a.y;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    nrm = sqrt(s);
    *beta_out = nrm;
  }
  __syncthreads();
  const double f = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int r = threadIdx.x; r < n; r += NT) {
    const zc a = w[r];
    v[r] = zc{a.x * f, a.y * f};
  }
}

inline dim3 grid_rows(int rows, int cols) {
  return dim3((unsigned)((rows + NT - 1) / NT), (unsigned)cols);
}

inline int last() { return (int)hipGetLastError(); }

}  // namespace

int col_norms(hipStream_t s, int n, int k, const zc* X, long ldx, double* out) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(k_col_norms, dim3(k), dim3(NT), 0, s, n, X, ldx, out);
  return last();
}

int resid_norms(hipStream_t s, int n, int k, const zc* Q, long ldq, const zc* Z, long ldz,
                const double* mu, double* out) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(k_resid_norms, dim3(k), dim3(NT), 0, s, n, Q, ldq, Z, ldz, mu, out);
  return last();
}

int scale_cols_inv(hipStream_t s, int n, int k, zc* X, long ldx, const double* nrm) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(k_scale_cols_inv, grid_rows(n, k), dim3(NT), 0, s, n, X, ldx, nrm);
  return last();
}

int gather_cols(hipStream_t s, int n, int cnt, const zc* src, long lds, zc* dst, long ldd,
                const int* perm) {
  if (cnt <= 0) return 0;
  hipLaunchKernelGGL(k_gather_cols, grid_rows(n, cnt), dim3(NT), 0, s, n, src, lds, dst, ldd,
                     perm);
  return last();
}

int gather_parity(hipStream_t s, int n, int k, const zc* P0, const zc* P1, long ldp, zc* dst,
                  long ldd, const int* deg) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(k_gather_parity, grid_rows(n, k), dim3(NT), 0, s, n, P0, P1, ldp, dst, ldd,
                     deg);
  return last();
}

int copy2d(hipStream_t s, int rows, int cols, const zc* src, long lds, zc* dst, long ldd) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL(k_copy2d, grid_rows(rows, cols), dim3(NT), 0, s, rows, src, lds, dst, ldd);
  return last();
}

int herm_from_lower(hipStream_t s, int k, zc* G, long ldg) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(k_herm_from_lower, grid_rows(k, k), dim3(NT), 0, s, k, G, ldg);
  return last();
}

int symmetrize(hipStream_t s, int n, zc* H, long ldh) {
  if (n <= 0) return 0;
  const unsigned nb = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_symmetrize, dim3(nb, nb), dim3(NT), 0, s, n, H, ldh, 0.5);
  return last();
}

int add_conj_transpose(hipStream_t s, int n, zc* H, long ldh) {
  if (n <= 0) return 0;
  const unsigned nb = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_symmetrize, dim3(nb, nb), dim3(NT), 0, s, n, H, ldh, 1.0);
  return last();
}

int gram_offnorm(hipStream_t s, int k, const zc* G, long ldg, double* out) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(k_gram_offnorm, dim3(1), dim3(1024), 0, s, k, G, ldg, out);
  return last();
}

int lower_half_diag(hipStream_t s, int n, const zc* A, long lda, zc* D, long ldd) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_lower_half_diag, grid_rows(n, n), dim3(NT), 0, s, n, A, lda, D, ldd);
  return last();
}

int conj_transpose(hipStream_t s, int n, const zc* src, long lds, zc* dst, long ldd) {
  if (n <= 0) return 0;
  const unsigned nb = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_conj_transpose, dim3(nb, nb), dim3(NT), 0, s, n, src, lds, dst, ldd);
  return last();
}

int zero_upper(hipStream_t s, int n, zc* L, long ldl) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_zero_upper, grid_rows(n, n), dim3(NT), 0, s, n, L, ldl);
  return last();
}

int set_identity(hipStream_t s, int n, zc* X, long ldx) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_set_identity, grid_rows(n, n), dim3(NT), 0, s, n, X, ldx);
  return last();
}

int add_diag(hipStream_t s, int n, zc* G, long ldg, double v) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(k_add_diag, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, n, G, ldg,
                     v);
  return last();
}

int check_finite(hipStream_t s, int rows, int cols, const zc* X, long ldx, int* flag) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL(k_check_finite, grid_rows(rows, cols), dim3(NT), 0, s, rows, X, ldx, flag);
  return last();
}

int fill_counter_random(hipStream_t s, int n, int k, zc* X, long ldx, unsigned long long seed,
                        int stream_id) {
  if (n <= 0 || k <= 0) return 0;
  const unsigned long long base = seed + ((unsigned long long)stream_id << 48);
  hipLaunchKernelGGL(k_fill_random, grid_rows(n, k), dim3(NT), 0, s, n, X, ldx, base);
  return last();
}

int matrix_hash(hipStream_t s, int rows, int cols, const zc* X, long ldx,
                unsigned long long* part, unsigned long long* out) {
  hipLaunchKernelGGL(k_hash_part, dim3(HASH_PARTS), dim3(NT), 0, s, rows, cols, X, ldx, part);
  int e = last();
  if (e) return e;
  hipLaunchKernelGGL(k_hash_sum, dim3(1), dim3(64), 0, s, HASH_PARTS, (const unsigned long long*)part,
                     out);
  return last();
}

int fill_zero(hipStream_t s, size_t count, zc* X) {
  if (count == 0) return 0;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((count + NT - 1) / NT)), dim3(NT), 0, s, count,
                     X);
  return last();
}

int potrf_leaf(hipStream_t s, int nb, zc* G, long ldg, zc* inv, int* info, int col_offset,
               double rel_tol) {
  if (nb <= 0 || nb > 64) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(k_potrf_leaf, dim3(1), dim3(1024), 0, s, nb, G, ldg, inv, info, col_offset,
                     rel_tol);
  return last();
}

int add_random(hipStream_t s, int n, int k, zc* X, long ldx, unsigned long long seed,
               int stream_id, double eps) {
  if (n <= 0 || k <= 0) return 0;
  const unsigned long long base = seed + ((unsigned long long)stream_id << 48);
  hipLaunchKernelGGL(k_add_random, grid_rows(n, k), dim3(NT), 0, s, n, X, ldx, base, eps);
  return last();
}

int gemv_n(hipStream_t s, int n, const zc* H, long ldh, const zc* x, zc* y, zc* part,
           int splits, const void* H32) {
  if (n <= 0) return 0;
  if (splits < 1) splits = 1;
  const int chunk = (n + splits - 1) / splits;
  splits = (n + chunk - 1) / chunk;
  if (H32)
    hipLaunchKernelGGL(k_gemv_part<float2>, grid_rows(n, splits), dim3(NT), 0, s, n,
                       (const float2*)H32, (long)n, x, part, chunk);
  else
    hipLaunchKernelGGL(k_gemv_part<zc>, grid_rows(n, splits), dim3(NT), 0, s, n, H, ldh, x,
                       part, chunk);
  int e = last();
  if (e) return e;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, n, splits,
                     (const zc*)part, y);
  return last();
}

int dots_c(hipStream_t s, int n, int cnt, const zc* V, long ldv, const zc* w, zc* h) {
  if (cnt <= 0) return 0;
  hipLaunchKernelGGL(k_dots_c, dim3(cnt), dim3(NT), 0, s, n, V, ldv, w, h);
  return last();
}

int sub_vh(hipStream_t s, int n, int cnt, const zc* V, long ldv, const zc* h, zc* w) {
  if (cnt <= 0) return 0;
  hipLaunchKernelGGL(k_sub_vh, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, n, cnt, V,
                     ldv, h, w);
  return last();
}

int lanczos_axpy(hipStream_t s, int n, int j, const zc* V, long ldv, const zc* h,
                 const double* betas, zc* w, double* alphas) {
  hipLaunchKernelGGL(k_lanczos_axpy, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, n, j,
                     V, ldv, h, betas, w, alphas);
  return last();
}

int normalize_into(hipStream_t s, int n, const zc* w, zc* v, double* beta_out) {
  hipLaunchKernelGGL(k_normalize_into, dim3(1), dim3(NT), 0, s, n, w, v, beta_out);
  return last();
}

}  // namespace chfsi
