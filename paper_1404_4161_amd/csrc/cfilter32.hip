// Mixed-precision Chebyshev filter: the three-term recurrence of Alg. 2 run
// on the defect of the current Ritz vectors, in complex FP32 on
// v_mfma_f32_16x16x4_f32.
//
// Let Q be Ritz vectors with Ritz values mu and residual matrix R = H Q -
// Q diag(mu) (from the last Rayleigh-Ritz, in FP64), Ht = (H - cI)/e,
// mu_t = (mu - c)/e and p_i the scaled Chebyshev polynomials of Alg. 2
// (p_0 = 1, p_1 = sigma_1 t, p_{i+1} = 2 sigma_{i+1} t p_i - sigma_{i+1}
// sigma_i p_{i-1}).  The filtered block p_i(Ht) Q splits into
// Q diag(p_i(mu_t)), computed exactly from scalars, and the defect
// E_i = p_i(Ht) Q - Q diag(p_i(mu_t)), which obeys
//   E_0 = 0,  E_1 = sigma_1 R / e,
//   E_{i+1} = 2 sigma_{i+1} (Ht E_i + R diag(p_i(mu_t)) / e)
//             - sigma_{i+1} sigma_i E_{i-1}.
// Only E_i goes through the GEMM.  Its rounding error is relative to
// ||E_i|| ~ ||R||, not to ||Q||, so FP32 arithmetic keeps the filtered
// vectors accurate to about eps_fp32 * ||R|| / ||H|| times the filter
// growth -- far below the residual the filter is aiming at once the
// residuals are small.  The GEMM is the same 64x64-tile, 4-wave design as
// the FP64 kernel, with K staged 16 deep (the LDS tile has the same size),
// and a 128x128-tile, 16-wave form for wide unsplit windows.
#include "internal.h"

#include <atomic>

#include <algorithm>
#include <cstring>

namespace chfsi {

namespace {

typedef float2 cf;                 // complex64
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;
constexpr int PA = BM + 1, PB = BN + 1;
constexpr int NXCD = 8;

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

struct DefArgs {
  int M, N, K;
  const cf* A; long lda;        // H in FP32 (n x n)
  const cf* Ecur; long lde;     // E_i (B operand), columns of the window
  const cf* Eold;               // E_{i-1} (same leading dimension)
  cf* Eout;                     // E_{i+1} (may alias Eold)
  const cf* R; long ldr;        // residual block (FP32)
  const float* cr;              // per-column coefficient of R
  float shift, sa, sb;
  int splits, kchunk;
  cf* part;                     // split-K partials: part[s*M*N + i + j*M]
  int tiles_m, tiles_n;
};

template <int PARTIAL>
__device__ __forceinline__ void defect_gemm_body(const DefArgs& g, int bid) {
  __shared__ cf As[2][BK][PA];
  __shared__ cf Bs[2][BK][PB];
  const int xcd = bid % NXCD, slot = bid / NXCD;
  const int vrows = g.splits * g.tiles_m;
  const int rows_x = (vrows - xcd + NXCD - 1) / NXCD;
  const int ri = slot / g.tiles_n;
  const int tn = slot - ri * g.tiles_n;
  if (ri >= rows_x) return;
  const int v = xcd + NXCD * ri;
  const int split = v / g.tiles_m;
  const int tm = v - split * g.tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = split * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int lr = lane & 15, lk = lane >> 4;

  f4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  cf ra[4], rb[4];
  auto load = [&](int k0) {
    const int m = m0 + (t & 63);
#pragma unroll
    for (int i = 0; i < 4; ++i) {     // A: m contiguous
      const int k = k0 + (t >> 6) + 4 * i;
      ra[i] = (m < g.M && k < kend) ? g.A[m + (long)k * g.lda] : cf{0.f, 0.f};
    }
    const int kb = k0 + (t & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {     // B: k contiguous
      const int n = n0 + (t >> 4) + 16 * i;
      rb[i] = (n < g.N && kb < kend) ? g.Ecur[kb + (long)n * g.lde] : cf{0.f, 0.f};
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) As[buf][(t >> 6) + 4 * i][t & 63] = ra[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) Bs[buf][t & 15][(t >> 4) + 16 * i] = rb[i];
  };
  const int nk = (kend - kbeg + BK - 1) / BK;
  if (nk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) load(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      cf a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[cur][kk * 4 + lk][wm * 32 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[cur][kk * 4 + lk][wn * 32 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accR[i][j] = mfma32(a[i].x, b[j].x, accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accI[i][j] = mfma32(a[i].x, b[j].y, accI[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accR[i][j] = mfma32(-a[i].y, b[j].y, accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accI[i][j] = mfma32(a[i].y, b[j].x, accI[i][j]);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
  }
  // FP32 MFMA output layout: lane l, register r holds row 4 (l / 16) + r
  // and column l % 16 of the 16x16 tile.
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + i * 16 + 4 * lk + r;
        const int col = n0 + wn * 32 + j * 16 + lr;
        if (row >= g.M || col >= g.N) continue;
        const cf acc = cf{accR[i][j][r], accI[i][j][r]};
        if (PARTIAL) {
          g.part[(long)split * g.M * g.N + row + (long)col * g.M] = acc;
        } else {
          const cf ec = g.Ecur[row + (long)col * g.lde];
          const cf rr = g.R[row + (long)col * g.ldr];
          const float crj = g.cr[col];
          cf out = cf{g.sa * (acc.x - g.shift * ec.x) + crj * rr.x,
                      g.sa * (acc.y - g.shift * ec.y) + crj * rr.y};
          if (g.sb != 0.f) {
            const cf eo = g.Eold[row + (long)col * g.lde];
            out.x -= g.sb * eo.x;
            out.y -= g.sb * eo.y;
          }
          g.Eout[row + (long)col * g.lde] = out;
        }
      }
}

template <int PARTIAL>
__global__ void __launch_bounds__(NT, 4) defect_gemm(DefArgs g) {
  defect_gemm_body<PARTIAL>(g, blockIdx.x);
}

// Grouped form (batches of independent problems): problem p of the list
// owns the workgroups [slot_begin[p], slot_begin[p+1]), a multiple of 8,
// so that the XCD interleaving inside each range is that of a launch of its
// own; no split-K.
__global__ void __launch_bounds__(NT, 4) defect_gemm_group(const DefArgs* list,
                                                          const int* slot_begin, int count) {
  int lo = 0, hi = count;
  const int b = blockIdx.x;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (slot_begin[mid] <= b) lo = mid; else hi = mid;
  }
  defect_gemm_body<0>(list[lo], b - slot_begin[lo]);
}

// Wide defect step for unsplit launches of wide windows: 128 x 128 output
// tiles, 16 waves in a 4 x 4 grid of 32 x 32 sub-tiles, K 16 deep, one
// workgroup per CU (each H element staged in LDS serves 128 columns).
constexpr int WBM = 128, WBN = 128, WNT = 1024, WPA = WBM + 1, WPB = WBN + 1;
constexpr int WIDE_MIN_N = 384;

__global__ void __launch_bounds__(WNT, 1) defect_gemm_wide(DefArgs g) {
  __shared__ cf As[2][BK][WPA];
  __shared__ cf Bs[2][BK][WPB];
  const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD;
  const int rows_x = (g.tiles_m - xcd + NXCD - 1) / NXCD;
  const int ri = slot / g.tiles_n;
  const int tn = slot - ri * g.tiles_n;
  if (ri >= rows_x) return;
  const int tm = xcd + NXCD * ri;
  const int m0 = tm * WBM, n0 = tn * WBN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave & 3, wn = wave >> 2;
  const int lr = lane & 15, lk = lane >> 4;
  f4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  // two elements of each operand per thread and stage
  constexpr int LE = BK * WBM / WNT;
  cf ra[LE], rb[LE];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LE; ++i) {
      const int idx = t + i * WNT;
      const int m = m0 + idx % WBM, k = k0 + idx / WBM;          // A: m contiguous
      ra[i] = (m < g.M && k < g.K) ? g.A[m + (long)k * g.lda] : cf{0.f, 0.f};
      const int kb = k0 + idx % BK, n = n0 + idx / BK;           // B: k contiguous
      rb[i] = (n < g.N && kb < g.K) ? g.Ecur[kb + (long)n * g.lde] : cf{0.f, 0.f};
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LE; ++i) {
      const int idx = t + i * WNT;
      As[buf][idx / WBM][idx % WBM] = ra[i];
      Bs[buf][idx % BK][idx / BK] = rb[i];
    }
  };
  const int nk = (g.K + BK - 1) / BK;
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      cf a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[cur][kk * 4 + lk][wm * 32 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[cur][kk * 4 + lk][wn * 32 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accR[i][j] = mfma32(a[i].x, b[j].x, accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accI[i][j] = mfma32(a[i].x, b[j].y, accI[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accR[i][j] = mfma32(-a[i].y, b[j].y, accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accI[i][j] = mfma32(a[i].y, b[j].x, accI[i][j]);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
  }
  // FP32 MFMA output: row 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + i * 16 + 4 * lk + r;
        const int col = n0 + wn * 32 + j * 16 + lr;
        if (row >= g.M || col >= g.N) continue;
        const cf ec = g.Ecur[row + (long)col * g.lde];
        const cf rr = g.R[row + (long)col * g.ldr];
        const float crj = g.cr[col];
        cf out = cf{g.sa * (accR[i][j][r] - g.shift * ec.x) + crj * rr.x,
                    g.sa * (accI[i][j][r] - g.shift * ec.y) + crj * rr.y};
        if (g.sb != 0.f) {
          const cf eo = g.Eold[row + (long)col * g.lde];
          out.x -= g.sb * eo.x;
          out.y -= g.sb * eo.y;
        }
        g.Eout[row + (long)col * g.lde] = out;
      }
}

__global__ void defect_reduce(int M, int N, int splits, const cf* part, const cf* Ecur,
                              const cf* Eold, cf* Eout, long lde, const cf* R, long ldr,
                              const float* cr, float shift, float sa, float sb) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M * N) return;
  const int row = (int)(idx % M), col = (int)(idx / M);
  cf s = cf{0.f, 0.f};
  for (int p = 0; p < splits; ++p) {
    const cf v = part[(long)p * M * N + idx];
    s.x += v.x;
    s.y += v.y;
  }
  const cf ec = Ecur[row + (long)col * lde];
  const cf rr = R[row + (long)col * ldr];
  cf out = cf{sa * (s.x - shift * ec.x) + cr[col] * rr.x, sa * (s.y - shift * ec.y) + cr[col] * rr.y};
  if (sb != 0.f) {
    const cf eo = Eold[row + (long)col * lde];
    out.x -= sb * eo.x;
    out.y -= sb * eo.y;
  }
  Eout[row + (long)col * lde] = out;
}

// R32[:, j] = fp32(Z[:, perm[j]] - mu[perm[j]] Q[:, perm[j]]); Qs[:, j] =
// Q[:, perm[j]] (FP64 copy in degree order); E1[:, j] = s1 * R32[:, j];
// E0[:, j] = 0.
__global__ void defect_setup(int n, const zc* Q, const zc* Z, long ld, const double* mu,
                             const int* perm, zc* Qs, cf* R32, cf* E0, cf* E1, long lde,
                             float s1) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  const int j = blockIdx.y;
  const int p = perm[j];
  const zc q = Q[r + (long)p * ld];
  const zc z = Z[r + (long)p * ld];
  const double m = mu[p];
  const cf res = cf{(float)(z.x - m * q.x), (float)(z.y - m * q.y)};
  Qs[r + (long)j * ld] = q;
  R32[r + (long)j * lde] = res;
  E0[r + (long)j * lde] = cf{0.f, 0.f};
  E1[r + (long)j * lde] = cf{s1 * res.x, s1 * res.y};
}

// Y[:, j] = pm[j] Qs[:, j] + E_{m_j}[:, j], E_{m_j} in E1 for odd m_j.
__global__ void defect_assemble(int n, const zc* Qs, long ld, const cf* E0, const cf* E1,
                                long lde, const int* deg, const double* pm, zc* Y, long ldy) {
  const int r = blockIdx.x * NT + threadIdx.x;
  if (r >= n) return;
  const int j = blockIdx.y;
  const cf* E = (deg[j] & 1) ? E1 : E0;
  const cf e = E[r + (long)j * lde];
  const zc q = Qs[r + (long)j * ld];
  const double s = pm[j];
  Y[r + (long)j * ldy] = zc{s * q.x + (double)e.x, s * q.y + (double)e.y};
}

__global__ void to_fp32(long count, const zc* src, cf* dst) {
  const long i = (long)blockIdx.x * NT + threadIdx.x;
  if (i < count) {
    const zc v = src[i];
    dst[i] = cf{(float)v.x, (float)v.y};
  }
}

int device_slots32() {
  static std::atomic<int> cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev] = 4 * cus;
  }
  return cache[dev];
}

}  // namespace

int matrix_to_fp32(hipStream_t s, int n, const zc* H, long ldh, void* H32) {
  // H is copied column by column when ldh != n
  cf* dst = (cf*)H32;
  if (ldh == n) {
    const long count = (long)n * n;
    hipLaunchKernelGGL(to_fp32, dim3((unsigned)((count + NT - 1) / NT)), dim3(NT), 0, s, count, H,
                       dst);
    return (int)hipGetLastError();
  }
  for (int c = 0; c < n; ++c) {
    hipLaunchKernelGGL(to_fp32, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, (long)n,
                       H + (long)c * ldh, dst + (long)c * n);
  }
  return (int)hipGetLastError();
}

int defect_setup_launch(hipStream_t s, int n, int k, const zc* Q, const zc* Z, long ld,
                        const double* mu, const int* perm, zc* Qs, void* R32, void* E0, void* E1,
                        float s1) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(defect_setup, dim3((unsigned)((n + NT - 1) / NT), (unsigned)k), dim3(NT), 0, s,
                     n, Q, Z, ld, mu, perm, Qs, (cf*)R32, (cf*)E0, (cf*)E1, (long)n, s1);
  return (int)hipGetLastError();
}

int defect_assemble_launch(hipStream_t s, int n, int k, const zc* Qs, long ld, const void* E0,
                           const void* E1, const int* deg, const double* pm, zc* Y, long ldy) {
  if (k <= 0) return 0;
  hipLaunchKernelGGL(defect_assemble, dim3((unsigned)((n + NT - 1) / NT), (unsigned)k), dim3(NT), 0,
                     s, n, Qs, ld, (const cf*)E0, (const cf*)E1, (long)n, deg, pm, Y, ldy);
  return (int)hipGetLastError();
}

int defect_reduce_launch(hipStream_t s, int M, int N, int splits, const void* part,
                         const void* Ecur, const void* Eold, void* Eout, long lde, const void* R,
                         long ldr, const float* cr, float shift, float sa, float sb) {
  const long total = (long)M * N;
  if (total <= 0) return 0;
  hipLaunchKernelGGL(defect_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, M, N,
                     splits, (const cf*)part, (const cf*)Ecur, (const cf*)Eold, (cf*)Eout, lde,
                     (const cf*)R, ldr, cr, shift, sa, sb);
  return (int)hipGetLastError();
}

size_t defect_group_arg_bytes() { return sizeof(DefArgs); }

int defect_group_fill(int n, int N, const void* H32, const void* Ecur, const void* Eold,
                      void* Eout, const void* R32, const float* cr, float shift, float sa,
                      float sb, void* out) {
  DefArgs g = {};
  g.M = n; g.N = N; g.K = n;
  g.A = (const cf*)H32; g.lda = n;
  g.Ecur = (const cf*)Ecur; g.Eold = (const cf*)Eold; g.Eout = (cf*)Eout; g.lde = n;
  g.R = (const cf*)R32; g.ldr = n; g.cr = cr;
  g.shift = shift; g.sa = sa; g.sb = sb;
  g.tiles_m = (n + BM - 1) / BM;
  g.tiles_n = (N + BN - 1) / BN;
  g.splits = 1;
  g.kchunk = ((n + BK - 1) / BK) * BK;
  std::memcpy(out, &g, sizeof(g));
  return ((g.tiles_m + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
}

int defect_group_launch(hipStream_t s, const void* dargs, const int* dslots, int count,
                        int total) {
  if (count <= 0 || total <= 0) return 0;
  hipLaunchKernelGGL(defect_gemm_group, dim3(total), dim3(NT), 0, s, (const DefArgs*)dargs,
                     dslots, count);
  return (int)hipGetLastError();
}

int defect_step(hipStream_t s, int n, int N, const void* H32, const void* Ecur, const void* Eold,
                void* Eout, const void* R32, const float* cr, float shift, float sa, float sb,
                void* part, size_t part_elems) {
  if (N <= 0) return 0;
  DefArgs g = {};
  g.M = n; g.N = N; g.K = n;
  g.A = (const cf*)H32; g.lda = n;
  g.Ecur = (const cf*)Ecur; g.Eold = (const cf*)Eold; g.Eout = (cf*)Eout; g.lde = n;
  g.R = (const cf*)R32; g.ldr = n; g.cr = cr;
  g.shift = shift; g.sa = sa; g.sb = sb;
  g.tiles_m = (n + BM - 1) / BM;
  g.tiles_n = (N + BN - 1) / BN;
  const int tiles = g.tiles_m * g.tiles_n;
  // split-K that fills the resident slots evenly (partials in FP32)
  int splits = 1;
  const int slots = device_slots32();
  const int max_s = (int)std::min<size_t>(8, part ? part_elems / ((size_t)n * N) : 1);
  double best_u = 0.0;
  for (int sp = 1; sp <= max_s; ++sp) {
    if (sp > 1 && n / sp < 512) break;
    const long wg = (long)tiles * sp;
    const double u = (double)wg / (double)(((wg + slots - 1) / slots) * slots);
    if (u > best_u + 1e-9) { best_u = u; splits = sp; }
    if (u >= 0.9) break;
  }
  int chunk = (n + splits - 1) / splits;
  chunk = ((chunk + BK - 1) / BK) * BK;
  g.kchunk = chunk;
  g.splits = (n + chunk - 1) / chunk;
  const int grid = ((g.splits * g.tiles_m + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
  if (g.splits == 1 && N >= WIDE_MIN_N) {
    DefArgs w = g;
    w.tiles_m = (n + WBM - 1) / WBM;
    w.tiles_n = (N + WBN - 1) / WBN;
    const int wgrid = ((w.tiles_m + NXCD - 1) / NXCD) * w.tiles_n * NXCD;
    hipLaunchKernelGGL(defect_gemm_wide, dim3(wgrid), dim3(WNT), 0, s, w);
    return (int)hipGetLastError();
  }
  if (g.splits == 1) {
    hipLaunchKernelGGL(defect_gemm<0>, dim3(grid), dim3(NT), 0, s, g);
    return (int)hipGetLastError();
  }
  g.part = (cf*)part;
  hipLaunchKernelGGL(defect_gemm<1>, dim3(grid), dim3(NT), 0, s, g);
  int e = (int)hipGetLastError();
  if (e) return e;
  const long total = (long)n * N;
  hipLaunchKernelGGL(defect_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, N,
                     g.splits, (const cf*)part, (const cf*)Ecur, (const cf*)Eold, (cf*)Eout,
                     (long)n, (const cf*)R32, (long)n, cr, shift, sa, sb);
  return (int)hipGetLastError();
}

}  // namespace chfsi
