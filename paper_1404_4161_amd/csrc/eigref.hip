// Eigen-decomposition of the projected matrix of Rayleigh-Ritz by iterative
// refinement, for the case that dominates a warm-started sequence: after a
// filter and an orthonormalisation the block's columns are already close to
// eigenvectors, so G = Q^H H Q is nearly diagonal.
//
// Starting from X = I, each iteration forms S = X^H G X and R = I - X^H X
// (GEMMs), the Rayleigh quotients lam_i = Re s_ii / (1 - Re r_ii), and the
// first-order correction F with X <- X (I + F):
//   f_ii = r_ii / 2,
//   f_ij = (s_ij + lam_j r_ij) / (lam_j - lam_i)   for i < j,
//   f_ji = r_ji - conj(f_ij),
// which makes the update orthogonalise exactly to first order (F + F^H = R)
// and diagonalise to first order; the error is squared per iteration while
// the couplings are small against the gaps (Ogita and Aishima, Japan J.
// Indust. Appl. Math. 2018, restated for complex Hermitian matrices).
// Pairs whose coupling is not small against their gap (close or degenerate
// Ritz values) are grouped into clusters (connected components); each
// cluster's block of S is diagonalised on the host by cyclic complex Jacobi
// and X is rotated by the block-diagonal result before the next iteration
// (the clustered-eigenvalue extension of the same authors, 2019).
// Converged when every coupling is below 8 k eps max|lam| and every entry
// of R below 8 k eps; one last update with f = R / 2 then restores
// orthonormality to rounding.  The caller falls back to a dense
// eigensolver when this returns "not refined" (far from diagonal, clusters
// larger than 32 columns or covering half the block, or 10 iterations).
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <vector>

namespace chfsi {

namespace {

constexpr int NT = 256;
constexpr double TAU = 0.1;          // coupling / gap limit of a Newton pair
constexpr int MAX_ITERS = 10;
constexpr int MAX_CLUSTER = 32;

const zc ONE = {1.0, 0.0}, ZERO = {0.0, 0.0}, MONE = {-1.0, 0.0};

__device__ __forceinline__ double zabs(zc a) { return sqrt(a.x * a.x + a.y * a.y); }

// non-negative doubles order like their bit patterns
__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v) {
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// lam_i and f_ii; stats[2] = max |lam|
__global__ void k_ref_diag(int k, const zc* S, const zc* R, double* lam, zc* F,
                           unsigned long long* stats) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= k) return;
  const long d = i + (long)i * k;
  const double l = S[d].x / (1.0 - R[d].x);
  lam[i] = l;
  F[d] = zc{0.5 * R[d].x, 0.0};
  atomic_max_nonneg(stats + 2, fabs(l));
}

// Couplings, the update F off the diagonal, convergence measures and the
// strongly coupled pairs (i < j).  stats[0] = max |coupling|, stats[1] = max
// |r_ij| (incl. the diagonal), stats[3] = number of strong pairs (pairs
// beyond `cap` are counted, not stored).
__global__ void k_ref_pairs(int k, const zc* S, const zc* R, const double* lam, zc* F,
                            unsigned long long* stats, int2* pairs, int cap, double tol_off) {
  const int i = blockIdx.x * NT + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= k) return;
  const long ij = i + (long)j * k, ji = j + (long)i * k;
  if (i == j) {
    atomic_max_nonneg(stats + 1, fabs(R[ij].x));
    return;
  }
  if (i > j) return;
  // Hermitian parts of S and R at (i, j)
  const zc s = zc{0.5 * (S[ij].x + S[ji].x), 0.5 * (S[ij].y - S[ji].y)};
  const zc r = zc{0.5 * (R[ij].x + R[ji].x), 0.5 * (R[ij].y - R[ji].y)};
  const double lj = lam[j], li = lam[i];
  const zc c = zc{s.x + lj * r.x, s.y + lj * r.y};
  const double gap = lj - li;
  const double ac = zabs(c);
  atomic_max_nonneg(stats + 0, ac);
  atomic_max_nonneg(stats + 1, zabs(r));
  zc f;
  const bool newton = fabs(gap) > tol_off && ac <= TAU * fabs(gap);
  if (newton) {
    f = zc{c.x / gap, c.y / gap};
  } else {
    f = zc{0.5 * r.x, 0.5 * r.y};
    if (ac > tol_off) {
      const unsigned long long slot = atomicAdd(stats + 3, 1ull);
      if (slot < (unsigned long long)cap) pairs[slot] = make_int2(i, j);
    }
  }
  F[ij] = f;
  // f_ji = r_ji - conj(f_ij), r_ji = conj(r)
  F[ji] = zc{r.x - f.x, -r.y + f.y};
}

// F = R / 2 (Hermitian part): the final orthonormalising update
__global__ void k_ref_half(int k, const zc* R, zc* F) {
  const int i = blockIdx.x * NT + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= k) return;
  const zc a = R[i + (long)j * k], b = R[j + (long)i * k];
  F[i + (long)j * k] = zc{0.25 * (a.x + b.x), 0.25 * (a.y - b.y)};
}

// X = I + F
__global__ void k_ref_identity_plus(int k, const zc* F, zc* X) {
  const int i = blockIdx.x * NT + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= k) return;
  zc v = F[i + (long)j * k];
  if (i == j) v.x += 1.0;
  X[i + (long)j * k] = v;
}

// S = Hermitian part of G, R = 0 (the first iteration, X = I)
__global__ void k_ref_start(int k, const zc* G, long ldg, zc* S, zc* R) {
  const int i = blockIdx.x * NT + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= k) return;
  const zc a = G[i + (long)j * ldg], b = G[j + (long)i * ldg];
  S[i + (long)j * k] = zc{0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
  R[i + (long)j * k] = zc{0.0, 0.0};
}

__global__ void k_ref_gather_entries(int cnt, const int2* idx, const zc* S, int k, zc* out) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t < cnt) out[t] = S[idx[t].x + (long)idx[t].y * k];
}

__global__ void k_ref_scatter_entries(int cnt, const int2* idx, const zc* val, zc* V, int k) {
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t < cnt) V[idx[t].x + (long)idx[t].y * k] = val[t];
}

// W[:, j] = X[:, perm[j]], mu[j] = lam[perm[j]]
__global__ void k_ref_sort_out(int k, const zc* X, const int* perm, const double* lam, zc* W,
                               long ldw, double* mu) {
  const int i = blockIdx.x * NT + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= k) return;
  const int p = perm[j];
  W[i + (long)j * ldw] = X[i + (long)p * k];
  if (i == 0) mu[j] = lam[p];
}

dim3 grid2(int k) { return dim3((unsigned)((k + NT - 1) / NT), (unsigned)k); }
dim3 grid1(int k) { return dim3((unsigned)((k + NT - 1) / NT)); }

#define RCK(expr)                         \
  do {                                    \
    int _e = (int)(expr);                 \
    if (_e != 0) return _e;               \
  } while (0)

typedef std::complex<double> cd;

// Cyclic Jacobi for a small Hermitian matrix a (c x c, column-major); v
// receives the eigenvectors (columns).  Each rotation removes a_pq: with
// a_pq = |a_pq| e^{i phi}, the phase diag(1, e^{-i phi}) makes the pair
// real and the real symmetric Jacobi rotation (Golub and Van Loan, Sec.
// 8.5) follows.
void jacobi_herm(int c, std::vector<cd>& a, std::vector<cd>& v) {
  v.assign((size_t)c * c, cd(0.0, 0.0));
  for (int i = 0; i < c; ++i) v[i + (size_t)i * c] = 1.0;
  auto A = [&](int i, int j) -> cd& { return a[i + (size_t)j * c]; };
  double scale = 0.0;
  for (int i = 0; i < c; ++i) scale = std::max(scale, std::abs(A(i, i)));
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0.0;
    for (int j = 0; j < c; ++j)
      for (int i = 0; i < j; ++i) off = std::max(off, std::abs(A(i, j)));
    if (off <= 4.0 * std::ldexp(1.0, -52) * std::max(scale, 1e-300)) break;
    for (int p = 0; p < c - 1; ++p)
      for (int q = p + 1; q < c; ++q) {
        const cd apq = A(p, q);
        const double m = std::abs(apq);
        if (m == 0.0) continue;
        const cd ph = apq / m;   // e^{i phi}
        const double zeta = (A(q, q).real() - A(p, p).real()) / (2.0 * m);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        // J: columns p, q of the identity replaced by
        //   J_pp = cs, J_qp = -sn conj(ph), J_pq = sn, J_qq = cs conj(ph)
        const cd jpp = cs, jqp = -sn * std::conj(ph), jpq = sn, jqq = cs * std::conj(ph);
        // A <- A J (columns p, q)
        for (int i = 0; i < c; ++i) {
          const cd aip = A(i, p), aiq = A(i, q);
          A(i, p) = aip * jpp + aiq * jqp;
          A(i, q) = aip * jpq + aiq * jqq;
        }
        // A <- J^H A (rows p, q)
        for (int j = 0; j < c; ++j) {
          const cd apj = A(p, j), aqj = A(q, j);
          A(p, j) = std::conj(jpp) * apj + std::conj(jqp) * aqj;
          A(q, j) = std::conj(jpq) * apj + std::conj(jqq) * aqj;
        }
        A(p, q) = 0.0;
        A(q, p) = 0.0;
        A(p, p) = A(p, p).real();
        A(q, q) = A(q, q).real();
        for (int i = 0; i < c; ++i) {
          const cd vip = v[i + (size_t)p * c], viq = v[i + (size_t)q * c];
          v[i + (size_t)p * c] = vip * jpp + viq * jqp;
          v[i + (size_t)q * c] = vip * jpq + viq * jqq;
        }
      }
  }
}

int find_root(std::vector<int>& parent, int x) {
  while (parent[x] != x) {
    parent[x] = parent[parent[x]];
    x = parent[x];
  }
  return x;
}

}  // namespace

size_t eig_refine_elems(int k) { return (size_t)7 * k * k; }

int eig_refine(hipStream_t s, int k, const zc* G, long ldg, zc* W, long ldw, double* mu,
               EigRefineBufs& rb, int* refined, int* iterations) {
  *refined = 0;
  if (iterations) *iterations = 0;
  if (k <= 0) return 0;
  const size_t kk = (size_t)k * k;
  zc* X = rb.mat;
  zc* Xn = X + kk;
  zc* P = Xn + kk;
  zc* S = P + kk;
  zc* R = S + kk;
  zc* F = R + kk;
  zc* V = F + kk;
  const double eps = std::ldexp(1.0, -52);
  RCK(hipMemsetAsync(rb.stats, 0, 4 * sizeof(unsigned long long), s));
  RCK(hipGetLastError());
  hipLaunchKernelGGL(k_ref_start, grid2(k), dim3(NT), 0, s, k, G, ldg, S, R);
  RCK(hipGetLastError());
  bool x_is_identity = true;
  double tol_off = 0.0;
  for (int it = 0; it < MAX_ITERS; ++it) {
    if (iterations) *iterations = it + 1;
    if (!x_is_identity) {
      RCK(zgemm(s, OP_N, OP_N, k, k, k, ONE, G, ldg, X, k, ZERO, P, k, false, nullptr, 0));
      RCK(zgemm(s, OP_C, OP_N, k, k, k, ONE, X, k, P, k, ZERO, S, k, false, nullptr, 0));
      RCK(set_identity(s, k, R, k));
      RCK(zgemm(s, OP_C, OP_N, k, k, k, MONE, X, k, X, k, ONE, R, k, false, nullptr, 0));
    }
    RCK(hipMemsetAsync(rb.stats, 0, 4 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_ref_diag, grid1(k), dim3(NT), 0, s, k, S, R, rb.lam, F, rb.stats);
    RCK(hipGetLastError());
    // tol_off needs max |lam|: the first pass reads it back
    unsigned long long st[4];
    if (it == 0) {
      RCK(hipMemcpyAsync(st, rb.stats, sizeof(st), hipMemcpyDeviceToHost, s));
      RCK(hipStreamSynchronize(s));
      double lmax;
      std::memcpy(&lmax, &st[2], sizeof(double));
      tol_off = 8.0 * k * eps * std::max(lmax, 1e-300);
    }
    hipLaunchKernelGGL(k_ref_pairs, grid2(k), dim3(NT), 0, s, k, S, R, rb.lam, F, rb.stats,
                       rb.pairs, rb.pair_cap, tol_off);
    RCK(hipGetLastError());
    RCK(hipMemcpyAsync(st, rb.stats, sizeof(st), hipMemcpyDeviceToHost, s));
    RCK(hipStreamSynchronize(s));
    double cmax, rmax;
    std::memcpy(&cmax, &st[0], sizeof(double));
    std::memcpy(&rmax, &st[1], sizeof(double));
    const unsigned long long nstrong = st[3];
    if (!std::isfinite(cmax) || !std::isfinite(rmax)) return 0;
    if (nstrong == 0 && cmax <= tol_off && rmax <= 8.0 * k * eps) {
      // converged: orthonormalise once more, sort ascending
      if (!x_is_identity) {
        hipLaunchKernelGGL(k_ref_half, grid2(k), dim3(NT), 0, s, k, R, F);
        RCK(hipGetLastError());
        RCK(copy2d(s, k, k, X, k, Xn, k));
        RCK(zgemm(s, OP_N, OP_N, k, k, k, ONE, X, k, F, k, ONE, Xn, k, false, nullptr, 0));
        std::swap(X, Xn);
      } else {
        RCK(set_identity(s, k, X, k));
      }
      std::vector<double> lam(k);
      RCK(hipMemcpyAsync(lam.data(), rb.lam, sizeof(double) * k, hipMemcpyDeviceToHost, s));
      RCK(hipStreamSynchronize(s));
      std::vector<int> perm(k);
      std::iota(perm.begin(), perm.end(), 0);
      std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return lam[a] < lam[b]; });
      RCK(hipMemcpyAsync(rb.perm, perm.data(), sizeof(int) * k, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_ref_sort_out, grid2(k), dim3(NT), 0, s, k, X, rb.perm, rb.lam, W, ldw,
                         mu);
      RCK(hipGetLastError());
      RCK(hipStreamSynchronize(s));
      *refined = 1;
      return 0;
    }
    if (nstrong > 0) {
      if (nstrong > (unsigned long long)rb.pair_cap) return 0;
      std::vector<int2> pr((size_t)nstrong);
      RCK(hipMemcpyAsync(pr.data(), rb.pairs, sizeof(int2) * pr.size(), hipMemcpyDeviceToHost, s));
      RCK(hipStreamSynchronize(s));
      std::vector<int> parent(k);
      std::iota(parent.begin(), parent.end(), 0);
      for (const int2& p : pr) {
        const int a = find_root(parent, p.x), b = find_root(parent, p.y);
        if (a != b) parent[a] = b;
      }
      std::vector<std::vector<int>> groups(k);
      for (int i = 0; i < k; ++i) groups[find_root(parent, i)].push_back(i);
      std::vector<std::vector<int>> clusters;
      size_t covered = 0, entries = 0;
      for (auto& g : groups) {
        if (g.size() < 2) continue;
        if ((int)g.size() > MAX_CLUSTER) return 0;
        covered += g.size();
        entries += g.size() * g.size();
        clusters.push_back(g);
      }
      if (covered * 2 > (size_t)k || entries > (size_t)rb.entry_cap) return 0;
      // gather the cluster blocks of S, diagonalise them on the host
      std::vector<int2> idx;
      idx.reserve(entries);
      for (const auto& g : clusters)
        for (int b : g)
          for (int a : g) idx.push_back(make_int2(a, b));
      RCK(hipMemcpyAsync(rb.idx, idx.data(), sizeof(int2) * idx.size(), hipMemcpyHostToDevice,
                         s));
      hipLaunchKernelGGL(k_ref_gather_entries, grid1((int)idx.size()), dim3(NT), 0, s,
                         (int)idx.size(), rb.idx, S, k, rb.val);
      RCK(hipGetLastError());
      std::vector<zc> blk(idx.size());
      RCK(hipMemcpyAsync(blk.data(), rb.val, sizeof(zc) * blk.size(), hipMemcpyDeviceToHost, s));
      RCK(hipStreamSynchronize(s));
      std::vector<zc> vals(idx.size());
      size_t off = 0;
      for (const auto& g : clusters) {
        const int c = (int)g.size();
        std::vector<cd> a((size_t)c * c), v;
        for (int b = 0; b < c; ++b)
          for (int q = 0; q < c; ++q) {
            const zc e1 = blk[off + q + (size_t)b * c], e2 = blk[off + b + (size_t)q * c];
            a[q + (size_t)b * c] = cd(0.5 * (e1.x + e2.x), 0.5 * (e1.y - e2.y));
          }
        jacobi_herm(c, a, v);
        for (size_t e = 0; e < (size_t)c * c; ++e) vals[off + e] = zc{v[e].real(), v[e].imag()};
        off += (size_t)c * c;
      }
      RCK(set_identity(s, k, V, k));
      RCK(hipMemcpyAsync(rb.val, vals.data(), sizeof(zc) * vals.size(), hipMemcpyHostToDevice,
                         s));
      hipLaunchKernelGGL(k_ref_scatter_entries, grid1((int)idx.size()), dim3(NT), 0, s,
                         (int)idx.size(), rb.idx, rb.val, V, k);
      RCK(hipGetLastError());
      if (x_is_identity) {
        RCK(copy2d(s, k, k, V, k, X, k));
      } else {
        RCK(zgemm(s, OP_N, OP_N, k, k, k, ONE, X, k, V, k, ZERO, Xn, k, false, nullptr, 0));
        std::swap(X, Xn);
      }
      // the host buffers are reused by the next iteration: wait here
      RCK(hipStreamSynchronize(s));
      x_is_identity = false;
      continue;
    }
    // Newton step X <- X (I + F)
    if (x_is_identity) {
      hipLaunchKernelGGL(k_ref_identity_plus, grid2(k), dim3(NT), 0, s, k, F, X);
      RCK(hipGetLastError());
    } else {
      RCK(copy2d(s, k, k, X, k, Xn, k));
      RCK(zgemm(s, OP_N, OP_N, k, k, k, ONE, X, k, F, k, ONE, Xn, k, false, nullptr, 0));
      std::swap(X, Xn);
    }
    x_is_identity = false;
  }
  return 0;
}

}  // namespace chfsi
