// Host driver of the ChFSI library: the outer loop of Alg. 1 (Lanczos
// bound, filter, orthonormalisation, Rayleigh-Ritz, residuals, locking,
// degree optimisation) over the device kernels of zgemm.hip and blas1.hip,
// and the C ABI declared in include/chfsi.h.
#include "chfsi.h"
#include "internal.h"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <thread>
#include <new>
#include <numeric>
#include <vector>

namespace chfsi {
namespace {

constexpr int NB = 64;          // Cholesky / triangular-solve block size
constexpr size_t ALIGN = 256;
// A Gram-matrix pivot below this fraction of its (unit) diagonal entry is a
// CholeskyQR breakdown: kappa(Y) near 1e6 or worse.
constexpr double GRAM_PIVOT_TOL = 1e-12;
// ||G - I||_F of the normalised Gram matrix below which one CholeskyQR
// pass suffices.
constexpr double CHOLQR_ONE_PASS = 0.1;
// Largest filter degree the mixed-precision coefficient table holds.
constexpr int CR_ROWS = 256;

const zc ONE = {1.0, 0.0}, ZERO = {0.0, 0.0}, MONE = {-1.0, 0.0};


// With the environment variable CHFSI_DEBUG set, every failed device call
// is reported on stderr (call text, source line, HIP or library code).
bool debug_enabled() {
  static const bool on = std::getenv("CHFSI_DEBUG") != nullptr;
  return on;
}

void report_failure(const char* what, int line, int code) {
  if (debug_enabled()) {
    std::fprintf(stderr, "chfsi: %s failed (line %d, code %d)\n", what, line, code);
    std::fflush(stderr);
  }
}

#define CK(expr)                                  \
  do {                                            \
    int _e = (int)(expr);                         \
    if (_e != 0) {                                \
      report_failure(#expr, __LINE__, _e);        \
      return CHFSI_DEVICE_ERROR;                  \
    }                                             \
  } while (0)

#define CKS(expr)                                 \
  do {                                            \
    int _s = (expr);                              \
    if (_s != CHFSI_OK) return _s;                \
  } while (0)

// ---------------------------------------------------------------------------
// workspace carving

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + ALIGN - 1) / ALIGN * ALIGN;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

size_t splitk_elems(int n, int nev, int k) {
  size_t s = 0;
  s = std::max(s, zgemm_work_elems(k, k, n));
  // the lower-only Gram has fewer tiles and may use more splits: bound it
  const int tm = (k + NB - 1) / NB;
  const int lower = tm * (tm + 1) / 2;
  if (lower < 512 && n >= 1024) {
    int want = (1024 + lower - 1) / lower;
    int maxs = n / 256;
    int sp = std::min(want, maxs);
    s = std::max(s, (size_t)std::max(sp, 1) * (size_t)k * (size_t)k);
  }
  s = std::max(s, zgemm_work_elems(nev, k, n));
  return s;
}

int gemv_splits(int n) {
  const int rowblocks = (n + 255) / 256;
  int sp = 1024 / std::max(rowblocks, 1);
  sp = std::max(1, std::min(sp, std::max(1, n / 128)));
  return sp;
}

// Device buffers of the step-level routines on an n x k block.
struct StepBufs {
  zc *T1, *T2, *G, *K2, *invk, *scratch, *gv_part, *V, *w, *h, *fpart;
  size_t fpart_elems;
  void *R32, *E0, *E1;          // mixed-precision filter: complex64 n x k each
  void *S0, *S1;                // BF16 / FP16 splits of E_i (k rows of split_kp(n) values)
  float* colscale;              // FP16 splits: 1 / scale of each column of E_i (k)
  float* h16part;               // FP16 splits: partial maxima of |H| (1024)
  float* crtab;                 // CR_ROWS x k coefficients of the residual term
  double* pm;                   // k final scalars p_{m_j}(mu_t)
  float *mlp_p, *mlp_x, *mlp_y;  // degree network: parameters, k x 8 inputs, k outputs
  EigRefineBufs ref;            // projected eigenproblem by refinement
  double *mu, *res, *nrm, *E, *alph, *bet, *dummy;
  int *perm, *deg, *info;
  size_t scratch_elems;
  int lanczos_cap;
};

void carve_step(Carver& c, StepBufs& b, int n, int k, int nev, int lanczos_steps) {
  const size_t nk = (size_t)n * k;
  b.T1 = c.take<zc>(nk);
  b.T2 = c.take<zc>(nk);
  b.fpart_elems = (size_t)CHEB_MAX_SPLITS * nk;
  b.fpart = c.take<zc>(b.fpart_elems);
  b.G = c.take<zc>((size_t)k * k);
  b.K2 = c.take<zc>((size_t)k * k);
  b.invk = c.take<zc>((size_t)((k + NB - 1) / NB) * NB * NB);
  b.scratch_elems = splitk_elems(n, nev, k);
  b.scratch = c.take<zc>(std::max<size_t>(b.scratch_elems, 1));
  b.gv_part = c.take<zc>((size_t)n * gemv_splits(n));
  b.lanczos_cap = std::max(1, std::min(lanczos_steps, n));
  b.V = c.take<zc>((size_t)n * (b.lanczos_cap + 1));
  b.w = c.take<zc>(n);
  b.h = c.take<zc>(b.lanczos_cap + 1);
  b.mu = c.take<double>(k);
  b.res = c.take<double>(k);
  b.nrm = c.take<double>(k);
  b.E = c.take<double>(k);
  b.alph = c.take<double>(b.lanczos_cap + 1);
  b.bet = c.take<double>(b.lanczos_cap + 1);
  b.dummy = c.take<double>(8);
  b.perm = c.take<int>(k);
  b.deg = c.take<int>(k);
  b.info = c.take<int>(8);
  b.R32 = c.take<char>(nk * 8);
  b.E0 = c.take<char>(nk * 8);
  b.E1 = c.take<char>(nk * 8);
  b.S0 = c.take<char>(split_panel_bytes(k, n));
  b.S1 = c.take<char>(split_panel_bytes(k, n));
  b.colscale = c.take<float>(k);
  b.h16part = c.take<float>(1024);
  b.crtab = c.take<float>((size_t)CR_ROWS * k);
  b.pm = c.take<double>(k);
  b.mlp_p = c.take<float>(MLP_PARAMS);
  b.mlp_x = c.take<float>((size_t)MLP_IN * k);
  b.mlp_y = c.take<float>(k);
  b.ref.mat = c.take<zc>(eig_refine_elems(k));
  b.ref.lam = c.take<double>(k);
  b.ref.stats = c.take<unsigned long long>(4);
  b.ref.pair_cap = 4 * k + 256;
  b.ref.pairs = c.take<int2>(b.ref.pair_cap);
  b.ref.entry_cap = 16 * k + 256;
  b.ref.idx = c.take<int2>(b.ref.entry_cap);
  b.ref.val = c.take<zc>(b.ref.entry_cap);
  b.ref.perm = c.take<int>(k);
}

// ---------------------------------------------------------------------------
// rocSOLVER handle (one per device), used only for the reduced k x k
// Hermitian eigenproblem of Rayleigh-Ritz.

std::mutex g_handle_mu;
rocblas_handle g_handles[64] = {};
// Set by the worker threads of a batched solve: each worker owns a handle,
// so their reduced eigensolves run concurrently on their own streams.
thread_local rocblas_handle tl_handle = nullptr;

int get_handle(rocblas_handle* h) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return CHFSI_DEVICE_ERROR;
  if (!g_handles[dev]) {
    if (rocblas_create_handle(&g_handles[dev]) != rocblas_status_success) return CHFSI_DEVICE_ERROR;
  }
  *h = g_handles[dev];
  return CHFSI_OK;
}

// ---------------------------------------------------------------------------
// event timers per phase

struct Timers {
  hipStream_t s;
  double* acc;                 // may be null
  struct Pending { int phase; hipEvent_t a, b; };
  std::vector<Pending> pend;
  std::vector<hipEvent_t> pool;
  int open_phase = -1;
  hipEvent_t open_ev = nullptr;

  Timers(hipStream_t st, double* a) : s(st), acc(a) {}
  ~Timers() {
    for (auto& p : pend) { pool.push_back(p.a); pool.push_back(p.b); }
    if (open_ev) pool.push_back(open_ev);
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void begin(int phase) {
    if (!acc) return;
    open_ev = get();
    open_phase = phase;
    if (open_ev) (void)hipEventRecord(open_ev, s);
  }
  void end() {
    if (!acc || !open_ev) return;
    hipEvent_t e = get();
    if (e) {
      (void)hipEventRecord(e, s);
      pend.push_back({open_phase, open_ev, e});
    } else {
      pool.push_back(open_ev);
    }
    open_ev = nullptr;
  }
  // call after the stream has been synchronised
  void drain() {
    for (auto& p : pend) {
      float ms = 0.f;
      (void)hipEventSynchronize(p.b);
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) acc[p.phase] += 1e-3 * ms;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pend.clear();
  }
};

// ---------------------------------------------------------------------------
// host helpers

// Number of eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  const int m = (int)a.size();
  for (int i = 0; i < m; ++i) {
    const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    q = (a[i] - x) - (i > 0 ? bb / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Smallest and largest eigenvalue of a symmetric tridiagonal by bisection.
void tridiag_extremes(const std::vector<double>& a, const std::vector<double>& b, double* lo,
                      double* hi) {
  const int m = (int)a.size();
  double gl = 1e300, gu = -1e300;
  for (int i = 0; i < m; ++i) {
    double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
    gl = std::min(gl, a[i] - r);
    gu = std::max(gu, a[i] + r);
  }
  auto kth = [&](int k) {   // k-th smallest, 0-based
    double l = gl, u = gu;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (l + u);
      if (mid == l || mid == u) break;
      if (sturm_count(a, b, mid) > k) u = mid; else l = mid;
    }
    return 0.5 * (l + u);
  };
  *lo = kth(0);
  *hi = kth(m - 1);
}

// ---------------------------------------------------------------------------
// device building blocks

// Blocked right-looking Cholesky of the Hermitian n x n matrix G (lower).
// invd receives the inverses of the diagonal NB-blocks (NB x NB each).
int potrf_blocked(hipStream_t s, int n, zc* G, long ldg, zc* invd, int* info, double rel_tol) {
  for (int jb = 0; jb < n; jb += NB) {
    const int nb = std::min(NB, n - jb);
    zc* inv = invd + (size_t)(jb / NB) * NB * NB;
    CK(potrf_leaf(s, nb, G + jb + (long)jb * ldg, ldg, inv, info, jb, rel_tol));
    const int m2 = n - jb - nb;
    if (m2 > 0) {
      zc* a21 = G + (jb + nb) + (long)jb * ldg;
      // L21 = A21 inv(L11)^H  (in place: each tile owns whole rows of A21)
      CK(zgemm(s, OP_N, OP_C, m2, nb, nb, ONE, a21, ldg, inv, nb, ZERO, a21, ldg, false, nullptr, 0));
      // A22 -= L21 L21^H (lower triangle)
      zc* a22 = G + (jb + nb) + (long)(jb + nb) * ldg;
      CK(zgemm(s, OP_N, OP_C, m2, m2, nb, MONE, a21, ldg, a21, ldg, ONE, a22, ldg, true, nullptr, 0));
    }
  }
  return CHFSI_OK;
}

// X <- L^{-1} X for lower-triangular L (n x n) with inverted diagonal blocks.
// lower_rhs: X is lower triangular (e.g. the identity), so block row j only
// has non-zero columns [0, jb + nb) and the products skip the rest.
int trsm_left_lower(hipStream_t s, int n, int m, const zc* L, long ldl, const zc* invd, zc* X,
                    long ldx, bool lower_rhs = false) {
  for (int jb = 0; jb < n; jb += NB) {
    const int nb = std::min(NB, n - jb);
    const zc* inv = invd + (size_t)(jb / NB) * NB * NB;
    const int cols = lower_rhs ? std::min(m, jb + nb) : m;
    // X_j = inv(L_jj) X_j  (in place: one tile row covers the whole block row)
    CK(zgemm(s, OP_N, OP_N, nb, cols, nb, ONE, inv, nb, X + jb, ldx, ZERO, X + jb, ldx, false,
             nullptr, 0));
    const int m2 = n - jb - nb;
    if (m2 > 0) {
      CK(zgemm(s, OP_N, OP_N, m2, cols, nb, MONE, L + (jb + nb) + (long)jb * ldl, ldl, X + jb,
               ldx, ONE, X + jb + nb, ldx, false, nullptr, 0));
    }
  }
  return CHFSI_OK;
}

// Reduction to standard form (Sec. 3.1) given Linv = L^{-1} for B = L L^H:
// H = Linv A Linv^H from the lower triangle of A: with A = T + T^H (T the
// lower triangle of A, diagonal halved), H = M + M^H for M = (Linv T)
// Linv^H.  Linv T is lower triangular (K range [j, i]) and M needs K <=
// min(i, j), so the two products cost n^3 / 6 + n^3 / 3 complex
// multiply-adds instead of n^3 / 2 + n^3 / 4 for (Linv A) Linv^H.  H (ld)
// first holds T, then M, then the result; W (ld) holds Linv T.  Linv must be
// zero above its diagonal.
int reduce_with_inverse(hipStream_t s, int n, const zc* A, long lda, const zc* Linv, zc* W,
                        zc* H, long ld) {
  CK(lower_half_diag(s, n, A, lda, H, ld));
  // W = Linv T (lower-triangular result: only the tiles meeting the lower
  // triangle are computed; the strict upper part of the diagonal tiles
  // comes out as exact zeros)
  CK(zgemm(s, OP_N, OP_N, n, n, n, ONE, Linv, ld, H, ld, ZERO, W, ld, true, nullptr, 0,
           KTRI_AB_LOWER));
  CK(zgemm(s, OP_N, OP_C, n, n, n, ONE, W, ld, Linv, ld, ZERO, H, ld, false, nullptr, 0,
           KTRI_A_LOWER_B_UPPER));
  CK(add_conj_transpose(s, n, H, ld));
  return CHFSI_OK;
}

int read_info(hipStream_t s, const int* info_dev, int* out) {
  CK(hipMemcpyAsync(out, info_dev, sizeof(int), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  return CHFSI_OK;
}

// One CholeskyQR pass: Yout = Yin R^{-1} with Yin^H Yin = R^H R, after
// normalising the columns of Yin (in place).  shift > 0 adds shift*I to the
// Gram matrix.  Returns CHFSI_NOT_HPD on a failed factorisation.
// offnorm (or null) receives ||G - I||_F of the normalised Gram matrix
// Yin^H Yin (before any shift).
int cholqr_pass(hipStream_t s, int n, int k, zc* Yin, long ldy, zc* Yout, long ldo, StepBufs& b,
                double shift, double* offnorm = nullptr) {
  CK(col_norms(s, n, k, Yin, ldy, b.nrm));
  CK(scale_cols_inv(s, n, k, Yin, ldy, b.nrm));
  CK(zgemm(s, OP_C, OP_N, k, k, n, ONE, Yin, ldy, Yin, ldy, ZERO, b.G, k, true, b.scratch,
           b.scratch_elems));
  CK(herm_from_lower(s, k, b.G, k));
  if (offnorm) CK(gram_offnorm(s, k, b.G, k, b.dummy));
  if (shift > 0.0) CK(add_diag(s, k, b.G, k, shift));
  CK(hipMemsetAsync(b.info, 0, sizeof(int), s));
  zc* invd = b.invk;
  CKS(potrf_blocked(s, k, b.G, k, invd, b.info, GRAM_PIVOT_TOL));
  int info = 0;
  if (offnorm) CK(hipMemcpyAsync(offnorm, b.dummy, sizeof(double), hipMemcpyDeviceToHost, s));
  CKS(read_info(s, b.info, &info));
  if (info != 0) return CHFSI_NOT_HPD;
  CK(set_identity(s, k, b.K2, k));
  CKS(trsm_left_lower(s, k, k, b.G, k, invd, b.K2, k, true));   // K2 = L^{-1}
  // Yout = Yin L^{-H} (upper-triangular right operand)
  CK(zgemm(s, OP_N, OP_C, n, k, k, ONE, Yin, ldy, b.K2, k, ZERO, Yout, ldo, false, nullptr, 0,
           KTRI_B_UPPER));
  return CHFSI_OK;
}

// Orthonormalise Y (n x k) against QL (n x nl) and by CholeskyQR2; result
// in Qout (may equal Y).  Uses b.T1 as the intermediate basis.
int orthonormalize_dev(hipStream_t s, int n, int k, zc* Y, long ldy, int nl, const zc* QL,
                       long ldql, zc* Qout, long ldq, StepBufs& b, int* shifted) {
  if (k <= 0) return CHFSI_OK;
  if (nl > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      // C = QL^H Y (nl x k, ld nl) in T2 (n x k elements, nl < n)
      zc* C = b.T2;
      CK(zgemm(s, OP_C, OP_N, nl, k, n, ONE, QL, ldql, Y, ldy, ZERO, C, nl, false, b.scratch,
               b.scratch_elems));
      CK(zgemm(s, OP_N, OP_N, n, k, nl, MONE, QL, ldql, C, nl, ONE, Y, ldy, false, nullptr, 0));
    }
  }
  zc* Q1 = b.T1;
  // CholeskyQR2; the second pass only when the first one's Gram matrix is
  // not close to the identity.  With ||G - I||_F <= 0.1 (kappa(Y) <= 1.11)
  // one pass already leaves an orthogonality error of the order of the
  // rounding of G (sqrt(n) eps), as the second pass would.
  double offn = HUGE_VAL;
  int st = cholqr_pass(s, n, k, Y, ldy, Q1, n, b, 0.0, &offn);
  if (st == CHFSI_OK && offn <= CHOLQR_ONE_PASS) {
    CK(copy2d(s, n, k, Q1, n, Qout, ldq));
    return CHFSI_OK;
  }
  if (st == CHFSI_OK) st = cholqr_pass(s, n, k, Q1, n, Qout, ldq, b, 0.0);
  if (st != CHFSI_NOT_HPD) return st;
  // Breakdown: shifted CholeskyQR3 (Fukaya et al., SISC 2020).  The shift is
  // 11 (n k + k (k + 1)) u ||Y||_2^2 with ||Y||_2^2 <= ||Y||_F^2 = k after
  // column normalisation.  An exactly rank-deficient block first gets a
  // relative 1e-10 random perturbation (counter-based generator, stream 2).
  const double u = std::ldexp(1.0, -53);
  const double sh = 11.0 * ((double)n * k + (double)k * (k + 1)) * u * (double)k;
  if (shifted) *shifted = 1;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (attempt == 1) {
      CK(col_norms(s, n, k, Y, ldy, b.nrm));
      CK(scale_cols_inv(s, n, k, Y, ldy, b.nrm));
      CK(add_random(s, n, k, Y, ldy, 0x5eedull, 2, 1e-10));
    }
    st = cholqr_pass(s, n, k, Y, ldy, Q1, n, b, sh);
    if (st == CHFSI_OK) st = cholqr_pass(s, n, k, Q1, n, Y, ldy, b, 0.0);
    if (st == CHFSI_OK) st = cholqr_pass(s, n, k, Y, ldy, Q1, n, b, 0.0);
    if (st == CHFSI_OK) {
      CK(copy2d(s, n, k, Q1, n, Qout, ldq));
      return CHFSI_OK;
    }
    if (st != CHFSI_NOT_HPD) return st;
  }
  return CHFSI_NOT_HPD;
}

// The k x k Hermitian eigenproblem of Rayleigh-Ritz on b.G (ld k).
// refine 1: iterative refinement from the identity (eigref.hip), with
// rocSOLVER zheevd as the fallback; 0: zheevd only; 2: refinement only
// (CHFSI_NO_CONVERGENCE when it does not converge).  Eigenvalues go to b.mu
// (ascending); the eigenvectors to b.K2 when refined (*refined = 1), else
// over b.G.
int eigh_projected(hipStream_t s, int k, StepBufs& b, int refine, int* refined) {
  int ok = 0;
  if (refine != 0) {
    int iters = 0;
    CK(eig_refine(s, k, b.G, k, b.K2, k, b.mu, b.ref, &ok, &iters));
    if (!ok && refine == 2) return CHFSI_NO_CONVERGENCE;
  }
  if (refined) *refined = ok;
  if (ok) return CHFSI_OK;
  {
    std::unique_lock<std::mutex> lk(g_handle_mu, std::defer_lock);
    rocblas_handle h = tl_handle;
    if (!h) {
      lk.lock();
      CKS(get_handle(&h));
    }
    CK(rocblas_set_stream(h, s));
    CK(rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_lower, k,
                        (rocblas_double_complex*)b.G, k, b.mu, b.E, b.info));
  }
  int info = 0;
  CK(hipMemcpyAsync(&info, b.info, sizeof(int), hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  CK(info);   // zheevd did not converge
  return CHFSI_OK;
}

// Rayleigh-Ritz on the orthonormal block Q (n x k):
// Z = H Q, G = Q^H Z, G W = W diag(mu), Qout = Q W, Zout = Z W,
// res_j = ||Zout_j - mu_j Qout_j||.  mu_h/res_h are host outputs.  Qout and
// Zout must not overlap Q or Z.
int rayleigh_ritz_dev(hipStream_t s, int n, int k, const zc* H, long ldh, const zc* Q, long ldq,
                      zc* Z, long ldz, zc* Qout, long ldqo, zc* Zout, long ldzo, StepBufs& b,
                      double* mu_h, double* res_h, int refine = 1, int* refined_out = nullptr) {
  // (the filter's partial-sum buffer is free here: split K for long H Q)
  CK(zgemm(s, OP_N, OP_N, n, k, n, ONE, H, ldh, Q, ldq, ZERO, Z, ldz, false, b.fpart,
           b.fpart_elems));
  CK(zgemm(s, OP_C, OP_N, k, k, n, ONE, Q, ldq, Z, ldz, ZERO, b.G, k, true, b.scratch,
           b.scratch_elems));
  CK(herm_from_lower(s, k, b.G, k));
  int refined = 0;
  CKS(eigh_projected(s, k, b, refine, &refined));
  if (refined_out) *refined_out = refined;
  const zc* Wv = refined ? b.K2 : b.G;
  CK(zgemm(s, OP_N, OP_N, n, k, k, ONE, Q, ldq, Wv, k, ZERO, Qout, ldqo, false, nullptr, 0));
  CK(zgemm(s, OP_N, OP_N, n, k, k, ONE, Z, ldz, Wv, k, ZERO, Zout, ldzo, false, nullptr, 0));
  CK(resid_norms(s, n, k, Qout, ldqo, Zout, ldzo, b.mu, b.res));
  CK(hipMemcpyAsync(mu_h, b.mu, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  CK(hipMemcpyAsync(res_h, b.res, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  return CHFSI_OK;
}


// Lanczos with full reorthogonalisation; returns bounds on the host.
// With H32 (fp32(H), n x n contiguous) the mat-vecs read it instead of H
// (half the bytes; products and sums stay FP64): the recurrence then runs
// on fp32(H), and the upper bound is raised by a bound of ||H - fp32(H)||_2
// <= 2^-24 ||H||_F <= 2^-24 sqrt(n) ||H||_2 so that it still bounds H.
int lanczos_dev(hipStream_t s, int n, const zc* H, long ldh, int steps, unsigned long long seed,
                StepBufs& b, double* upper, double* tmin, double* tmax,
                const void* H32 = nullptr) {
  const int m = std::max(1, std::min(steps, std::min(n, b.lanczos_cap)));
  const int gs = gemv_splits(n);
  CK(fill_counter_random(s, n, 1, b.V, n, seed, 0));
  CK(normalize_into(s, n, b.V, b.V, b.dummy));
  for (int j = 0; j < m; ++j) {
    const zc* vj = b.V + (size_t)j * n;
    CK(gemv_n(s, n, H, ldh, vj, b.w, b.gv_part, gs, H32));
    CK(dots_c(s, n, j + 1, b.V, n, b.w, b.h));
    CK(lanczos_axpy(s, n, j, b.V, n, b.h, b.bet, b.w, b.alph));
    for (int pass = 0; pass < 2; ++pass) {
      CK(dots_c(s, n, j + 1, b.V, n, b.w, b.h));
      CK(sub_vh(s, n, j + 1, b.V, n, b.h, b.w));
    }
    CK(normalize_into(s, n, b.w, b.V + (size_t)(j + 1) * n, b.bet + j));
  }
  std::vector<double> a(m), bb(m);
  CK(hipMemcpyAsync(a.data(), b.alph, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  CK(hipMemcpyAsync(bb.data(), b.bet, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  CK(hipStreamSynchronize(s));
  // an invariant subspace ends the recurrence early
  double amax = 0.0;
  for (int j = 0; j < m; ++j) amax = std::max(amax, std::fabs(a[j]));
  int meff = m;
  for (int j = 0; j < m - 1; ++j) {
    if (bb[j] <= 1e-14 * std::max(amax, 1e-300)) { meff = j + 1; break; }
  }
  std::vector<double> aa(a.begin(), a.begin() + meff), be(bb.begin(), bb.begin() + meff);
  double lo, hi;
  tridiag_extremes(aa, be, &lo, &hi);
  *tmin = lo;
  *tmax = hi;
  *upper = hi + std::fabs(bb[meff - 1]);
  if (H32) {
    const double scale = std::max(std::fabs(*upper), std::fabs(lo));
    *upper += std::ldexp(1.0, -24) * std::sqrt((double)n) * scale;
  }
  return CHFSI_OK;
}

// Alg. 2 on device.  P0 holds Y_0 (n x k, columns sorted by ascending
// degree m); on return column j of P[m_j mod 2] holds Y_{m_j}.  flops gets
// the algorithmic count (8 n^2 per column mat-vec), mfma_flops (if given)
// the real flops the MFMAs execute (6 n^2 per column with the 3M split).
int filter_dev(hipStream_t s, int n, int k, const zc* H, long ldh, zc* P0, zc* P1, long ld,
               const std::vector<int>& m, double c, double e, double gamma, zc* part,
               size_t part_elems, double* flops, int* launches, double* mfma_flops = nullptr) {
  if (k <= 0) return CHFSI_OK;
  const double sig1 = e / (gamma - c);
  const double nn = (double)n * (double)n;
  // Y_1 = (sigma_1 / e)(H Y_0 - c Y_0)
  CK(cheb_step(s, n, k, H, ldh, P0, ld, nullptr, ld, P1, ld, c, sig1 / e, 0.0, part, part_elems));
  *flops += 8.0 * nn * k;
  if (mfma_flops) *mfma_flops += 2.0 * filter_step_cm(n, k) * nn * k;
  *launches += 1;
  double sig = sig1;
  int first = 0;
  while (first < k && m[first] <= 1) ++first;
  const int mmax = m[k - 1];
  for (int i = 1; i < mmax; ++i) {
    const double sn = 1.0 / (2.0 / sig1 - sig);
    zc* cur = (i & 1) ? P1 : P0;
    zc* old = (i & 1) ? P0 : P1;
    const int cols = k - first;
    CK(cheb_step(s, n, cols, H, ldh, cur + (size_t)first * ld, ld, old + (size_t)first * ld, ld,
                 old + (size_t)first * ld, ld, c, 2.0 * sn / e, sn * sig, part, part_elems));
    *flops += 8.0 * nn * cols;
    if (mfma_flops) *mfma_flops += 2.0 * filter_step_cm(n, cols) * nn * cols;
    *launches += 1;
    sig = sn;
    while (first < k && m[first] <= i + 1) ++first;
  }
  return CHFSI_OK;
}

template <class T>
int upload(hipStream_t s, T* dst, const std::vector<T>& v) {
  if (v.empty()) return CHFSI_OK;
  CK(hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
  CK(hipStreamSynchronize(s));
  return CHFSI_OK;
}

// Mixed-precision Alg. 2 on the defect of the Ritz vectors (cfilter32.hip).
// Q, Z = H Q (ld) and mu (host) are in the current column order; order[j]
// is the column filtered j-th (ascending degree m[j]).  The filtered block
// goes to Y (ld), and Qs (ld) receives the reordered Q.
//
// Per-step forms of the defect filter besides FP32 (cfilter16.hip):
// sched[i] = 1 runs step i (E_i -> E_{i+1}) in the BF16-split form (needs
// Hs, the BF16 split panel of H), 2 in the FP16-split form (needs Hh, the
// FP16 split panel of 2^s H, and inv_h = 2^-s).  The counters receive the
// algorithmic flops and the number of steps of each split form.
struct SplitSteps {
  const void* Hs = nullptr;
  const void* Hh = nullptr;
  float inv_h = 1.f;
  const std::vector<char>* sched = nullptr;
  double flops_bf16 = 0.0, flops_fp16 = 0.0;
  int steps_bf16 = 0, steps_fp16 = 0;
};

// Host plan of one defect filter: the sigmas of the recurrence, and for
// every step i = 1 .. mmax - 1 (E_i -> E_{i+1}) the first column of its
// window and its form (0 FP32, 1 BF16 split, 2 FP16 split).
struct DefectPlan {
  int n = 0, k = 0, mmax = 0;
  double c = 0.0, e = 0.0;
  std::vector<double> sig;
  std::vector<int> first;
  std::vector<char> kind;
};

// The part of the defect filter before its steps: the coefficient tables
// (uploaded), R32 / E0 / E1 / Qs (defect_setup) and the plan.
int defect_prepare(hipStream_t s, int n, int k, const zc* Q, const zc* Z, long ld,
                   const std::vector<double>& mu, const std::vector<int>& order,
                   const std::vector<int>& m, double c, double e, double gamma, zc* Qs,
                   StepBufs& b, const SplitSteps* sp, DefectPlan& plan) {
  plan = DefectPlan();
  plan.n = n;
  plan.k = k;
  plan.c = c;
  plan.e = e;
  if (k <= 0) return CHFSI_OK;
  const int mmax = m[k - 1];
  if (mmax > CR_ROWS) return CHFSI_INVALID_ARG;
  const double sig1 = e / (gamma - c);
  // p_i(mu_t) for i <= m_j by the scalar form of the recurrence, and the
  // coefficient cr_i[j] = 2 sigma_{i+1} p_i(mu_t_j) / e of step i
  std::vector<float> cr((size_t)mmax * k, 0.f);
  std::vector<double> pm(k);
  std::vector<double> sig(mmax + 1);
  sig[1] = sig1;
  for (int i = 1; i < mmax; ++i) sig[i + 1] = 1.0 / (2.0 / sig1 - sig[i]);
  for (int j = 0; j < k; ++j) {
    const double t = (mu[order[j]] - c) / e;
    double pprev = 1.0, pcur = sig1 * t;
    for (int i = 1; i < m[j]; ++i) {
      cr[(size_t)i * k + j] = (float)(2.0 * sig[i + 1] * pcur / e);
      const double pnext = 2.0 * sig[i + 1] * t * pcur - sig[i + 1] * sig[i] * pprev;
      pprev = pcur;
      pcur = pnext;
    }
    pm[j] = pcur;
  }
  CKS(upload(s, b.mu, mu));
  CKS(upload(s, b.perm, order));
  CKS(upload(s, b.deg, m));
  CKS(upload(s, b.crtab, cr));
  CKS(upload(s, b.pm, pm));
  CK(defect_setup_launch(s, n, k, Q, Z, ld, b.mu, b.perm, Qs, b.R32, b.E0, b.E1,
                         (float)(sig1 / e)));
  plan.mmax = mmax;
  plan.sig = sig;
  plan.first.assign(mmax + 1, 0);
  plan.kind.assign(mmax + 1, 0);
  int first = 0;
  while (first < k && m[first] <= 1) ++first;
  for (int i = 1; i < mmax; ++i) {
    plan.first[i] = first;
    int kd = 0;
    if (sp && sp->sched && i < (int)sp->sched->size()) {
      const int v = (*sp->sched)[i];
      if (v == 1 && sp->Hs) kd = 1;
      if (v == 2 && sp->Hh) kd = 2;
    }
    plan.kind[i] = (char)kd;
    while (first < k && m[first] <= i + 1) ++first;
  }
  return CHFSI_OK;
}

// Scalars of step i of a planned defect filter.
struct DefectStepScalars {
  float shift, sa, sb;
};
DefectStepScalars defect_scalars(const DefectPlan& p, int i) {
  return {(float)p.c, (float)(2.0 * p.sig[i + 1] / p.e), (float)(p.sig[i + 1] * p.sig[i])};
}

// flops32 receives the algorithmic flops of the FP32 steps; sp (or null)
// selects split forms for some steps and counts them.
int defect_filter_dev(hipStream_t s, int n, int k, const void* H32, const zc* Q, const zc* Z,
                      long ld, const std::vector<double>& mu, const std::vector<int>& order,
                      const std::vector<int>& m, double c, double e, double gamma, zc* Qs, zc* Y,
                      StepBufs& b, double* flops32, int* launches, SplitSteps* sp = nullptr) {
  if (k <= 0) return CHFSI_OK;
  DefectPlan plan;
  CKS(defect_prepare(s, n, k, Q, Z, ld, mu, order, m, c, e, gamma, Qs, b, sp, plan));
  const int mmax = plan.mmax;
  const size_t c64 = 8;   // bytes per complex64
  const size_t srow = (size_t)split_kp(n) * 8;   // bytes per split-panel row
  bool split_ready = false;   // the split panel of E_i holds the window
  for (int i = 1; i < mmax; ++i) {
    const int first = plan.first[i];
    const char* cur = (const char*)((i & 1) ? b.E1 : b.E0);
    char* old = (char*)((i & 1) ? b.E0 : b.E1);
    const size_t off = (size_t)first * n * c64;
    const int cols = k - first;
    const DefectStepScalars sc = defect_scalars(plan, i);
    const float shift = sc.shift, sa = sc.sa, sbeta = sc.sb;
    const float* cri = b.crtab + (size_t)i * k + first;
    const int kd = plan.kind[i];
    if (kd == 1) {
      char* scur = (char*)((i & 1) ? b.S1 : b.S0) + first * srow;
      char* snext = (char*)((i & 1) ? b.S0 : b.S1) + first * srow;
      if (!split_ready) CK(cols_to_split(s, n, cols, cur + off, n, scur));
      const bool next16 = i + 1 < mmax && plan.kind[i + 1] == 1;
      CK(defect_step_split(s, n, cols, sp->Hs, scur, cur + off, old + off, old + off,
                           (const char*)b.R32 + off, cri, shift, sa, sbeta,
                           next16 ? snext : nullptr));
      split_ready = next16;
      sp->flops_bf16 += 8.0 * (double)n * n * cols;
      sp->steps_bf16 += 1;
    } else if (kd == 2) {
      char* scur = (char*)b.S0 + first * srow;
      CK(cols_to_split_h16(s, n, cols, cur + off, n, scur, b.colscale + first));
      CK(defect_step_h16(s, n, cols, sp->Hh, sp->inv_h, scur, b.colscale + first, cur + off,
                         old + off, old + off, (const char*)b.R32 + off, cri, shift, sa, sbeta,
                         b.fpart, b.fpart_elems * 2));
      split_ready = false;
      sp->flops_fp16 += 8.0 * (double)n * n * cols;
      sp->steps_fp16 += 1;
    } else {
      CK(defect_step(s, n, cols, H32, cur + off, old + off, old + off, (const char*)b.R32 + off,
                     cri, shift, sa, sbeta, b.fpart, b.fpart_elems * 2));
      split_ready = false;
      *flops32 += 8.0 * (double)n * n * cols;
    }
    *launches += 1;
  }
  CK(defect_assemble_launch(s, n, k, Qs, ld, b.E0, b.E1, b.deg, b.pm, Y, ld));
  return CHFSI_OK;
}

// Whether FP32 rounding in the defect filter stays far below what the
// filter is aiming at, for every wanted vector.  The rounding error of a
// defect step is about eps_fp32 times the defect, i.e. eps_fp32 ||r_j|| /
// ||H|| relative to the column.  Components of that error inside the span
// of the block (the directions the filter amplifies, eq. resl) are removed
// by the Rayleigh-Ritz step that follows; the filter damps the rest.  The
// FP32 form is used when this floor is 100x below the residual the filter
// aims at (the tolerance, or the current residual reduced by rho_j^m).
bool defect_filter_safe(int n_wanted, const std::vector<double>& mu,
                        const std::vector<double>& res, const std::vector<int>& deg, double c,
                        double e, double gamma, double tol, double norm_h) {
  const double eps32 = std::ldexp(1.0, -24);
  auto rho = [](double t) {
    if (std::fabs(t) <= 1.0) return 1.0;
    const double r = std::sqrt(t * t - 1.0);
    return std::max(std::fabs(t + r), std::fabs(t - r));
  };
  (void)gamma;
  for (int j = 0; j < n_wanted; ++j) {
    const double rel = res[j] / norm_h;
    if (!(rel <= 1e-2)) return false;
    const double rj = rho((mu[j] - c) / e);
    const double floor_ = eps32 * rel;
    const double target = std::max(tol, rel * std::pow(rj, -deg[j]));
    if (floor_ > 0.01 * target) return false;
  }
  return true;
}

// Mixed precision: one FP32 defect loop can reduce a residual by about
// 1/(100 eps32) (the bound of defect_filter_safe).  When every wanted
// vector needs at most twice that, cap its degree at one loop's reach so
// that the loop runs in FP32 and the next one finishes; the guards take the
// largest capped degree.  capped[j] marks the capped columns.  Returns
// false (deg unchanged) when the cap does not apply.
bool cap_degrees_fp32(int n_wanted, const std::vector<double>& mu, const std::vector<double>& res,
                      std::vector<int>& deg, double c, double e, double norm_h,
                      std::vector<char>& capped) {
  const double reach_nats = std::log(1.0 / (100.0 * std::ldexp(1.0, -24)));
  const int ka = (int)deg.size();
  const int nw = std::min(n_wanted, ka);
  std::vector<int> d = deg;
  std::vector<char> rate(ka, 0), cap(ka, 0);
  int fill = 0;
  bool any = false, changed = false;
  for (int j = 0; j < nw; ++j) {
    if (!(res[j] / norm_h <= 1e-2)) return false;
    const double t = (mu[j] - c) / e;
    if (!(std::fabs(t) > 1.0)) continue;
    const double lr = std::log(std::fabs(t) + std::sqrt(t * t - 1.0));
    const int reach = (int)std::floor(reach_nats / lr * (1.0 - 1e-12));
    if (reach < 1 || d[j] > 2 * reach) return false;
    if (d[j] > reach) {
      d[j] = reach;
      cap[j] = 1;
      changed = true;
    }
    rate[j] = 1;
    fill = any ? std::max(fill, d[j]) : d[j];
    any = true;
  }
  if (!any || !changed) return false;
  for (int j = 0; j < ka; ++j)
    if (!rate[j]) d[j] = fill;
  deg.swap(d);
  capped.swap(cap);
  return true;
}

// Per-step precision inside an FP32 defect filter (precision 2).  Step i
// (E_i -> E_{i+1}) may use the BF16-split product, whose error is at most
// BF16_SPLIT_EPS times the defect, when for every wanted vector j still
// filtered (m_j > i) that error, damped by the m_j - i - 1 steps after it
// (eq. resl: by rho_j^-(m_j - i - 1) relative to the column), stays
// BF16_SPLIT_MARGIN times below what the filter aims at (the bound of
// defect_filter_safe with the step's own damping).  The bound is a worst
// case: rounding errors of random sign put the measured error near 2^-16,
// a third of it, so the margin of 10 is about 30 in practice; a step taken
// too early only costs convergence (the FP64 residuals decide locking).
// deg is in the current column order; the result has one entry per step
// index 0 .. max degree - 1 (entry 0 unused).
// The FP16-split form (precision 3) takes the same rule with its own
// bound, FP16_SPLIT_EPS = 3 * 2^-22, and marks its steps 2.
constexpr double BF16_SPLIT_EPS = 3.0 / 65536.0;
constexpr double FP16_SPLIT_EPS = 3.0 / 4194304.0;
constexpr double BF16_SPLIT_MARGIN = 10.0;

std::vector<char> split_step_schedule(int n_wanted, const std::vector<double>& mu,
                                      const std::vector<double>& res, const std::vector<int>& deg,
                                      double c, double e, double tol, double norm_h,
                                      double eps, char mark) {
  const int ka = (int)deg.size();
  int mmax = 0;
  for (int j = 0; j < ka; ++j) mmax = std::max(mmax, deg[j]);
  std::vector<char> ok(std::max(mmax, 1), mark);
  ok[0] = 0;
  for (int j = 0; j < std::min(n_wanted, ka); ++j) {
    const double t = (mu[j] - c) / e;
    const double lr = std::fabs(t) > 1.0 ? std::log(std::fabs(t) + std::sqrt(t * t - 1.0)) : 0.0;
    const double rel = res[j] / norm_h;
    const double target = std::max(tol, rel * std::exp(-lr * deg[j]));
    for (int i = 1; i < deg[j]; ++i) {
      const double floor_ = eps * rel * std::exp(-lr * (deg[j] - i - 1));
      if (!(floor_ * BF16_SPLIT_MARGIN <= target)) ok[i] = 0;
    }
  }
  return ok;
}

int upload_ints(hipStream_t s, int* dst, const std::vector<int>& v) {
  if (v.empty()) return CHFSI_OK;
  CK(hipMemcpyAsync(dst, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice, s));
  CK(hipStreamSynchronize(s));
  return CHFSI_OK;
}

double elapsed(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

}  // namespace

// ===========================================================================
// ChFSI solve

namespace {

// Header of the persistent B-factor region at the start of the workspace.
constexpr unsigned long long FACTOR_MAGIC = 0xC4F5100BFAC70001ull;
struct FactorHeader {
  unsigned long long magic, n, hash, pad;
};

struct SolveBufs {
  unsigned long long* header = nullptr;   // FactorHeader (device)
  unsigned long long* hpart = nullptr;    // hash partials + new hash
  zc *H = nullptr, *L = nullptr, *Linv = nullptr, *W = nullptr, *invd = nullptr;
  zc *QL, *QA, *ZA, *P0, *P1, *TMP;
  void* H32 = nullptr;          // fp32(H), mixed precision only
  void* Hs = nullptr;           // BF16 split panel of H's rows, precision 2 only
  void* Hh = nullptr;           // FP16 split panel of 2^s H's rows, precision 3 only
  float inv_hh = 1.f;           // 2^-s
  int* flag;
  StepBufs st;
};

size_t carve_solve(Carver& c, SolveBufs& b, int n, int nev, int nex, bool gen, int lsteps,
                   int precision) {
  const int k = nev + nex;
  const size_t nn = (size_t)n * n, nk = (size_t)n * k;
  if (gen) {
    // persistent factor region first, so its offset does not depend on k
    b.header = c.take<unsigned long long>(4);
    b.L = c.take<zc>(nn);
    b.Linv = c.take<zc>(nn);
    b.hpart = c.take<unsigned long long>(HASH_PARTS + 1);
    b.H = c.take<zc>(nn);
    b.W = c.take<zc>(nn);
    b.invd = c.take<zc>((size_t)((n + NB - 1) / NB) * NB * NB);
  }
  b.QL = c.take<zc>((size_t)n * nev);
  b.QA = c.take<zc>(nk);
  b.ZA = c.take<zc>(nk);
  b.P0 = c.take<zc>(nk);
  b.P1 = c.take<zc>(nk);
  b.TMP = c.take<zc>(nk);
  if (precision >= 1) b.H32 = c.take<char>(nn * 8);
  if (precision == 2) b.Hs = c.take<char>(split_panel_bytes(n, n));
  if (precision == 3) b.Hh = c.take<char>(split_panel_bytes(n, n));
  b.flag = c.take<int>(8);
  carve_step(c, b.st, n, k, nev, lsteps);
  return c.off + ALIGN;
}

int degrees_host(int k, const double* mu, const double* res, int n_wanted, double alpha,
                 double beta, double tol_abs, int deg_max, int* deg) {
  const double c = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
  std::vector<char> def(k, 0);
  int fill = 0;
  bool any = false;
  for (int j = 0; j < std::min(n_wanted, k); ++j) {
    const double t = (mu[j] - c) / e;
    if (std::fabs(t) <= 1.0) continue;
    const double r = std::sqrt(t * t - 1.0);
    const double rho = std::max(std::fabs(t + r), std::fabs(t - r));
    const double ratio = std::max(res[j] / tol_abs, 1.0);
    int m = (int)std::ceil(std::log(ratio) / std::log(rho));
    m = std::min(std::max(m, 1), deg_max);
    deg[j] = m;
    def[j] = 1;
    fill = any ? std::max(fill, m) : m;
    any = true;
  }
  if (!any) fill = deg_max;
  for (int j = 0; j < k; ++j)
    if (!def[j]) deg[j] = fill;
  return CHFSI_OK;
}

// Input features of the degree network (the layout is documented with
// chfsi_degree_features).  Returns false when the vector has no analytic
// rate (|t| <= 1).
bool degree_features(double mu, double res, double gap, double alpha, double beta, double gamma,
                     double norm_h, double tol_abs, int loop, double* f, double* ln_rho) {
  const double c = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
  const double t = (mu - c) / e;
  if (!(std::fabs(t) > 1.0)) return false;
  const double lr = std::log(std::fabs(t) + std::sqrt(t * t - 1.0));
  const double f0 = std::log(std::max(res, tol_abs) / tol_abs);
  f[0] = f0;
  f[1] = std::log(lr);
  f[2] = std::log(std::max(f0 / lr, 0.5));
  f[3] = std::log(std::fabs(t));
  f[4] = (alpha != gamma) ? (mu - gamma) / (alpha - gamma) : 0.0;
  f[5] = std::log(std::max(gap / e, 1e-12));
  f[6] = std::log(std::max(res, 1e-300) / norm_h);
  f[7] = (double)std::min(std::max(loop - 1, 0), 4);
  if (ln_rho) *ln_rho = lr;
  return true;
}

// Distance from mu[j] to the nearest other value of the ascending mu[0..k).
double ritz_gap(int k, const double* mu, int j, double e) {
  double g = std::numeric_limits<double>::infinity();
  if (j > 0) g = std::min(g, mu[j] - mu[j - 1]);
  if (j + 1 < k) g = std::min(g, mu[j + 1] - mu[j]);
  return std::isfinite(g) ? g : e;
}

// SplitMix64 output i of stream `stream` (the generator of the start block
// and Lanczos vector), as a double in [0, 1).
double splitmix_host(unsigned long long seed, int stream, unsigned long long i) {
  unsigned long long z = seed + ((unsigned long long)stream << 48) + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53;
}

constexpr int STREAM_JITTER = 3;
constexpr double MLP_OOD = 6.0;   // standardised features beyond this use the rule

// Sequence-calibrated degrees (degree_mode 3, Multiple Optimization read
// from eq. resl): the rate of vector j is corrected by its speed measured
// earlier in the sequence, speed[j] = observed ln(Res_before / Res_after) /
// (m ln|rho|) (NaN when unknown): m_j = max(rule_j, ceil(m_a,j * f / speed_j))
// with f = SEQ_MARGIN in a loop that can finish every wanted vector (all
// such degrees within deg_max) and 1 otherwise.  Unknown speeds and vectors
// without a rate take the rule.  Guards take the largest wanted degree.
constexpr double SEQ_MARGIN = 1.25;

int sequence_degrees(int k, const double* mu, const double* res, const double* speed,
                     int n_wanted, double alpha, double beta, double tol_abs, int deg_max,
                     int* deg, int* src) {
  std::vector<int> rule(k);
  degrees_host(k, mu, res, n_wanted, alpha, beta, tol_abs, deg_max, rule.data());
  const double c = 0.5 * (alpha + beta), e = 0.5 * (beta - alpha);
  const int nw = std::min(n_wanted, k);
  std::vector<double> need(k, 0.0);
  std::vector<char> rate(k, 0), cal(k, 0);
  bool finishing = true;
  for (int j = 0; j < nw; ++j) {
    const double t = (mu[j] - c) / e;
    if (!(std::fabs(t) > 1.0)) continue;
    rate[j] = 1;
    const double lr = std::log(std::fabs(t) + std::sqrt(t * t - 1.0));
    const double m_a = std::log(std::max(res[j] / tol_abs, 1.0)) / lr;
    const double sp = speed ? speed[j] : NAN;
    cal[j] = std::isfinite(sp) && sp > 0.0;
    need[j] = cal[j] ? m_a / sp : m_a;
    if (!(std::ceil(need[j]) <= (double)deg_max)) finishing = false;
  }
  const double f = finishing ? SEQ_MARGIN : 1.0;
  int fill = 0;
  bool any = false;
  for (int j = 0; j < k; ++j) {
    src[j] = 2;
    if (!rate[j]) continue;
    int m = rule[j];
    if (cal[j]) {
      const double mc = need[j] * f;
      const int mm = std::isfinite(mc) ? (int)std::min<double>(std::ceil(mc), (double)deg_max)
                                       : deg_max;
      m = std::min(std::max(std::max(mm, 1), rule[j]), deg_max);
      src[j] = 1;
    } else {
      src[j] = 0;
    }
    deg[j] = m;
    fill = any ? std::max(fill, m) : m;
    any = true;
  }
  if (!any) fill = deg_max;
  for (int j = 0; j < k; ++j)
    if (src[j] == 2) deg[j] = fill;
  return CHFSI_OK;
}

// Learned degrees (the rule of chfsi_degrees_learned).  prm_host is the
// caller's blob, prm_dev its device copy; x_dev / y_dev hold k rows.
// src (k ints) receives 0 rule fallback, 1 network, 2 guard fill; feats
// (k x 8, may be null) the features of the wanted vectors.
int learned_degrees(hipStream_t s, int k, const double* mu, const double* res, int n_wanted,
                    double alpha, double beta, double gamma, double norm_h, double tol_abs,
                    int loop, int deg_max, const float* prm_host, const float* prm_dev,
                    float* x_dev, float* y_dev, int* deg, float* pred, int* src, double* feats,
                    int finishing_mode = -1, bool* finishing_out = nullptr) {
  std::vector<int> rule(k);
  degrees_host(k, mu, res, n_wanted, alpha, beta, tol_abs, deg_max, rule.data());
  const double e = 0.5 * (beta - alpha);
  const int nw = std::min(n_wanted, k);
  std::vector<int> rows;
  std::vector<float> X;
  std::vector<double> lrho(k, 0.0), m_a(k, 0.0);
  std::vector<char> ood(k, 0);
  for (int j = 0; j < k; ++j) {
    src[j] = 2;
    if (pred) pred[j] = NAN;
  }
  for (int j = 0; j < nw; ++j) {
    double f[MLP_IN];
    if (!degree_features(mu[j], res[j], ritz_gap(k, mu, j, e), alpha, beta, gamma, norm_h,
                         tol_abs, loop, f, &lrho[j]))
      continue;
    if (feats) std::copy(f, f + MLP_IN, feats + (size_t)j * MLP_IN);
    m_a[j] = f[0] / lrho[j];
    for (int i = 0; i < MLP_IN; ++i) {
      const double sd = prm_host[MLP_STD + i] > 0.f ? prm_host[MLP_STD + i] : 1.0;
      const double z = (f[i] - prm_host[MLP_MEAN + i]) / sd;
      if (!(std::fabs(z) <= MLP_OOD)) ood[j] = 1;
      X.push_back((float)f[i]);
    }
    rows.push_back(j);
  }
  std::vector<float> y(rows.size());
  if (!rows.empty()) {
    CK(hipMemcpyAsync(x_dev, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, s));
    CK(mlp_forward(s, (int)rows.size(), x_dev, prm_dev, y_dev));
    CK(hipMemcpyAsync(y.data(), y_dev, sizeof(float) * y.size(), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
  }
  // A loop that can finish every wanted vector (all predicted degrees
  // within deg_max) takes the safety margin: a miss there costs a whole
  // extra loop.  Otherwise some vectors go on anyway and the rest take the
  // predicted degree.
  bool finishing = finishing_mode == 1;
  if (finishing_mode < 0) {
    finishing = true;
    for (size_t r = 0; r < rows.size(); ++r) {
      const int j = rows[r];
      const bool net = !ood[j] && std::isfinite(y[r]);
      const double need = net ? m_a[j] * std::exp(-(double)y[r]) : m_a[j];
      if (!(std::ceil(need) <= (double)deg_max)) finishing = false;
    }
  }
  if (finishing_out) *finishing_out = finishing;
  const double margin = finishing ? (double)prm_host[MLP_MARGIN] : 0.0;
  int fill = 0;
  bool any = false;
  for (size_t r = 0; r < rows.size(); ++r) {
    const int j = rows[r];
    if (pred) pred[j] = y[r];
    int m;
    if (ood[j] || !std::isfinite(y[r])) {
      m = rule[j];
      src[j] = 0;
    } else {
      const double mc = m_a[j] * std::exp(margin - (double)y[r]);
      m = std::isfinite(mc) ? (int)std::min<double>(std::ceil(mc), (double)deg_max) : deg_max;
      // the rule's degree is the floor: the network only adds degree where
      // the analytic model is too optimistic
      m = std::min(std::max(std::max(m, 1), rule[j]), deg_max);
      src[j] = 1;
    }
    deg[j] = m;
    fill = any ? std::max(fill, m) : m;
    any = true;
  }
  if (!any) fill = deg_max;
  for (int j = 0; j < k; ++j)
    if (src[j] == 2) deg[j] = fill;
  return CHFSI_OK;
}

// One chfsi_solve call as a state machine over the phases of Alg. 1:
// setup (input checks, reduction, Lanczos bound, start block), then loops
// of begin_loop (degrees, precision, degree order), the filter, end_loop
// (QR, Rayleigh-Ritz, residuals, locking, next degrees), and finish
// (output).  A single solve runs the filter itself (filter_own); a batch of
// solves runs its FP64 filters together in grouped launches.
struct Solve {
  // arguments
  int n = 0, nev = 0, nex = 0, k = 0;
  const zc* A = nullptr;
  int lda = 0;
  const zc* B = nullptr;
  int ldb = 0;
  double tol = 0.0;
  const zc* X0 = nullptr;
  int ldx0 = 0;
  const double* Lambda0 = nullptr;
  double* Lambda = nullptr;
  zc* X = nullptr;
  int ldx = 0;
  void* work = nullptr;
  size_t work_bytes = 0;
  chfsi_opts o = {};
  hipStream_t s = nullptr;
  chfsi_info* info = nullptr;

  // state across loops
  std::chrono::steady_clock::time_point t_start;
  bool gen = false;
  SolveBufs b;
  Timers tm{nullptr, nullptr};
  long ld = 0;
  const zc* H = nullptr;
  long ldh = 0;
  double beta = 0.0, tmin = 0.0, tmax = 0.0, norm_h = 0.0, tol_abs = 0.0;
  long long matvecs = 0, filter_mv = 0;
  int shifted = 0;
  std::vector<double> mu, res;
  double alpha = 0.0, gamma = 0.0;
  // per position: degree, where it came from (0 rule, 1 network, 2 guard,
  // 3 fixed deg0), the rule's degree, jittered or not
  std::vector<int> deg, dsrc, rule_deg;
  std::vector<char> jittered;
  int learned_cols = 0, fallback_cols = 0, learned_raised = 0, log_records = 0;
  int nl = 0;
  std::vector<double> lam_locked;
  double max_locked_res = 0.0;
  int it = 0;
  int status = CHFSI_NO_CONVERGENCE;
  double filter_flops = 0.0, filter_sec = 0.0, flops32 = 0.0, sec32 = 0.0, flops16 = 0.0;
  double flopsh = 0.0, flops64_mfma = 0.0;
  int iters32 = 0, launches = 0, steps16 = 0, stepsh = 0, rr_refined = 0, rr_dense = 0;
  bool have_res = false;   // residuals of the current block known
  hipEvent_t fe0 = nullptr, fe1 = nullptr;
  bool done = false;
  // batch: this loop's defect filter runs in its group's launches (prepared
  // on this problem's stream; end_loop assembles the filtered block)
  DefectPlan dplan;
  bool grouped_defect = false;

  // the current loop
  int ka = 0, nw_loop = 0;
  double c = 0.0, e = 0.0;
  bool use32 = false, logging = false, own_filter = false, res_known_before = false;
  std::vector<char> capped;
  std::vector<double> pending;
  std::vector<int> order, msort;
  // per active position: convergence speed of the vector relative to the
  // analytic model (measured in this call, or carried in from the previous
  // problem through opts.seq_rates; NaN when unknown), and this loop's
  // residual and ln|rho| before the filter
  std::vector<double> speed, res_before, lnrho;
  std::vector<double> speed_locked;

  ~Solve() {
    if (fe0) (void)hipEventDestroy(fe0);
    if (fe1) (void)hipEventDestroy(fe1);
  }

  double alpha_of(int nl_, int ka_) const {
    if (o.alpha_rule == 1) return mu[std::min(nev - nl_, ka_ - 1)];
    return mu[ka_ - 1];
  }

  int setup() {
    t_start = std::chrono::steady_clock::now();
    k = nev + nex;
    gen = B != nullptr;
    Carver cv(work);
    const size_t need = carve_solve(cv, b, n, nev, nex, gen, o.lanczos_steps, o.precision);
    if (work_bytes < need) return CHFSI_INVALID_ARG;
    StepBufs& sb = b.st;
    tm.s = s;
    tm.acc = info ? info->step_seconds : nullptr;
    ld = n;

    // non-finite inputs
    CK(hipMemsetAsync(b.flag, 0, sizeof(int), s));
    CK(check_finite(s, n, n, A, lda, b.flag));
    if (gen) CK(check_finite(s, n, n, B, ldb, b.flag));
    if (X0) CK(check_finite(s, n, k, X0, ldx0, b.flag));
    int flag = 0;
    CKS(read_info(s, b.flag, &flag));
    if (flag) return CHFSI_NONFINITE;

    // reduction to standard form (Sec. 3.1): B = L L^H, H = L^{-1} A L^{-H};
    // the start block in the new coordinates is Y0 = L^H X0
    H = A;
    ldh = lda;
    if (gen) {
      tm.begin(0);
      // reuse the factor of B when the workspace holds the factor of this B
      FactorHeader hdr = {};
      unsigned long long hnew = 0;
      CK(matrix_hash(s, n, n, B, ldb, b.hpart, b.hpart + HASH_PARTS));
      CK(hipMemcpyAsync(&hdr, b.header, sizeof(hdr), hipMemcpyDeviceToHost, s));
      CK(hipMemcpyAsync(&hnew, b.hpart + HASH_PARTS, sizeof(hnew), hipMemcpyDeviceToHost, s));
      CK(hipStreamSynchronize(s));
      const bool reuse = o.reuse_b_factor && hdr.magic == FACTOR_MAGIC &&
                         hdr.n == (unsigned long long)n && hdr.hash == hnew;
      if (info) info->b_factor_reused = reuse ? 1 : 0;
      if (!reuse) {
        FactorHeader inval = {0, 0, 0, 0};
        CK(hipMemcpyAsync(b.header, &inval, sizeof(inval), hipMemcpyHostToDevice, s));
        CK(copy2d(s, n, n, B, ldb, b.L, ld));
        CK(hipMemsetAsync(sb.info, 0, sizeof(int), s));
        CKS(potrf_blocked(s, n, b.L, ld, b.invd, sb.info, 0.0));
        int pinfo = 0;
        CKS(read_info(s, sb.info, &pinfo));
        if (pinfo != 0) return CHFSI_NOT_HPD;
        CK(zero_upper(s, n, b.L, ld));
        CK(set_identity(s, n, b.Linv, ld));
        CKS(trsm_left_lower(s, n, n, b.L, ld, b.invd, b.Linv, ld, true));
        FactorHeader valid = {FACTOR_MAGIC, (unsigned long long)n, hnew, 0};
        CK(hipMemcpyAsync(b.header, &valid, sizeof(valid), hipMemcpyHostToDevice, s));
        CK(hipStreamSynchronize(s));
      }
      if (X0) {
        CK(zgemm(s, OP_C, OP_N, n, k, n, ONE, b.L, ld, X0, ldx0, ZERO, b.QA, ld, false, nullptr,
                 0, KTRI_A_UPPER));
      }
      CKS(reduce_with_inverse(s, n, A, lda, b.Linv, b.W, b.H, ld));
      tm.end();
      H = b.H;
      ldh = ld;
    } else if (X0) {
      CK(copy2d(s, n, k, X0, ldx0, b.QA, ld));
    }
    if (!X0) CK(fill_counter_random(s, n, k, b.QA, ld, o.seed, 1));

    // Lanczos bound (the LANCZOS step of Alg. 1); the mixed-precision modes
    // need fp32(H) anyway and run its mat-vecs on that copy
    if (o.precision >= 1) CK(matrix_to_fp32(s, n, H, ldh, b.H32));
    tm.begin(1);
    CKS(lanczos_dev(s, n, H, ldh, o.lanczos_steps, o.seed, sb, &beta, &tmin, &tmax,
                    o.precision >= 1 ? b.H32 : nullptr));
    tm.end();
    norm_h = std::max(std::fabs(beta), std::fabs(tmin));
    tol_abs = tol * norm_h;
    matvecs = std::min(o.lanczos_steps, n);

    // Start.  With the previous problem's Ritz values (Alg. 1 inputs) the
    // first filter takes its bounds from them and filters X0 directly;
    // otherwise one QR + Rayleigh-Ritz of the start block supplies them.
    mu.assign(k, 0.0);
    res.assign(k, 0.0);
    if (X0 && Lambda0) {
      for (int j = 0; j < k; ++j) mu[j] = Lambda0[j];
    } else {
      tm.begin(3);
      CK(copy2d(s, n, k, b.QA, ld, b.TMP, ld));
      CKS(orthonormalize_dev(s, n, k, b.TMP, ld, 0, nullptr, ld, b.QA, ld, sb, &shifted));
      tm.end();
      tm.begin(4);
      int refined = 0;
      CKS(rayleigh_ritz_dev(s, n, k, H, ldh, b.QA, ld, b.ZA, ld, b.P0, ld, b.P1, ld, sb,
                            mu.data(), res.data(), o.rr_refine, &refined));
      ++(refined ? rr_refined : rr_dense);
      std::swap(b.QA, b.P0);
      std::swap(b.ZA, b.P1);
      tm.end();
      tm.drain();
      matvecs += k;
    }
    alpha = alpha_of(0, k);
    gamma = std::min(mu[0], tmin);
    deg.assign(k, o.deg0);
    dsrc.assign(k, 3);
    rule_deg.assign(k, o.deg0);
    jittered.assign(k, 0);
    if (o.degree_mode == 2)
      CK(hipMemcpyAsync(sb.mlp_p, o.mlp, sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice, s));
    have_res = !(X0 && Lambda0);
    speed.assign(k, NAN);
    if (X0 && o.seq_rates)
      for (int j = 0; j < k; ++j) speed[j] = o.seq_rates[j];
    if (o.precision == 2) CK(matrix_to_split(s, n, H, ldh, b.Hs));
    if (o.precision == 3)
      CK(matrix_to_split_h16(s, n, H, ldh, b.H32, b.Hh, b.st.h16part, &b.inv_hh));
    CK(hipEventCreate(&fe0));
    CK(hipEventCreate(&fe1));
    return CHFSI_OK;
  }

  // Degrees of the active block for loop `loop` (Sec. 3.1.1, or learned,
  // then the optional jitter); needs the residuals of the block.
  int choose_degrees(int ka_, int loop) {
    StepBufs& sb = b.st;
    const int nw = std::min(nev - nl, ka_);
    deg.assign(ka_, o.deg0);
    dsrc.assign(ka_, 3);
    jittered.assign(ka_, 0);
    if (o.degree_mode == 1) return CHFSI_OK;
    std::vector<int> rule(ka_);
    degrees_host(ka_, mu.data(), res.data(), nev - nl, alpha, beta, tol_abs, o.deg_max,
                 rule.data());
    if (o.degree_mode == 3) {
      CKS(sequence_degrees(ka_, mu.data(), res.data(), speed.data(), nev - nl, alpha, beta,
                           tol_abs, o.deg_max, deg.data(), dsrc.data()));
      for (int j = 0; j < nw; ++j) {
        if (dsrc[j] == 1) ++learned_cols;
        if (dsrc[j] == 1 && deg[j] > rule[j]) ++learned_raised;
        if (dsrc[j] == 0) ++fallback_cols;
      }
    } else if (o.degree_mode == 2) {
      bool finishing = false;
      CKS(learned_degrees(s, ka_, mu.data(), res.data(), nev - nl, alpha, beta, gamma, norm_h,
                          tol_abs, loop, o.deg_max, o.mlp, sb.mlp_p, sb.mlp_x, sb.mlp_y,
                          deg.data(), nullptr, dsrc.data(), nullptr, -1, &finishing));
      if (finishing && o.precision >= 1) {
        // a loop whose degrees get capped to the reach of FP32 cannot finish
        const double cc = 0.5 * (alpha + beta), ee = 0.5 * (beta - alpha);
        std::vector<int> d2 = deg;
        std::vector<char> cp(ka_, 0);
        if (!defect_filter_safe(nev - nl, mu, res, deg, cc, ee, gamma, tol, norm_h) &&
            cap_degrees_fp32(nev - nl, mu, res, d2, cc, ee, norm_h, cp))
          CKS(learned_degrees(s, ka_, mu.data(), res.data(), nev - nl, alpha, beta, gamma,
                              norm_h, tol_abs, loop, o.deg_max, o.mlp, sb.mlp_p, sb.mlp_x,
                              sb.mlp_y, deg.data(), nullptr, dsrc.data(), nullptr, 0, nullptr));
      }
      for (int j = 0; j < nw; ++j) {
        if (dsrc[j] == 1) ++learned_cols;
        if (dsrc[j] == 1 && deg[j] > rule[j]) ++learned_raised;
        if (dsrc[j] == 0) ++fallback_cols;
      }
    } else {
      deg = rule;
      dsrc.assign(ka_, 0);
    }
    if (o.degree_jitter > 0.0) {
      const double cc = 0.5 * (alpha + beta), ee = 0.5 * (beta - alpha);
      int fill = 0;
      bool any = false;
      std::vector<char> rate(ka_, 0);
      for (int j = 0; j < nw; ++j) {
        if (!(std::fabs((mu[j] - cc) / ee) > 1.0)) continue;
        rate[j] = 1;
        const double u = 2.0 * splitmix_host(o.seed, STREAM_JITTER,
                                             (unsigned long long)(loop - 1) * k + j) - 1.0;
        int m = (int)std::lround(deg[j] * std::exp(o.degree_jitter * u));
        deg[j] = std::min(std::max(m, 1), o.deg_max);
        jittered[j] = 1;
        fill = any ? std::max(fill, deg[j]) : deg[j];
        any = true;
      }
      if (!any) fill = o.deg_max;
      for (int j = 0; j < ka_; ++j)
        if (!rate[j]) deg[j] = fill;
    }
    return CHFSI_OK;
  }

  // Start of an outer loop: degrees, precision, degree order; for an FP64
  // filter the active block is gathered into P0 in that order.  Sets done
  // when the loop cap is reached.
  int begin_loop() {
    StepBufs& sb = b.st;
    own_filter = false;
    if (it >= o.max_iter) {
      done = true;
      return CHFSI_OK;
    }
    ++it;
    ka = k - nl;
    c = 0.5 * (alpha + beta);
    e = 0.5 * (beta - alpha);
    // A warm start with Lambda0 may take its first degrees from the rule
    // once the residuals of X0 are known (first_rule).
    const bool warm_rule = it == 1 && X0 && Lambda0 && o.first_rule && o.degree_mode != 1;
    if (!have_res && (o.precision >= 1 || warm_rule)) {
      // one product gives Z = H Q and the residuals of the warm start block
      tm.begin(4);
      CK(zgemm(s, OP_N, OP_N, n, ka, n, ONE, H, ldh, b.QA, ld, ZERO, b.ZA, ld, false, sb.fpart,
               sb.fpart_elems));
      CKS(upload(s, sb.mu, std::vector<double>(mu.begin(), mu.begin() + ka)));
      CK(resid_norms(s, n, ka, b.QA, ld, b.ZA, ld, sb.mu, sb.res));
      CK(hipMemcpyAsync(res.data(), sb.res, sizeof(double) * ka, hipMemcpyDeviceToHost, s));
      CK(hipStreamSynchronize(s));
      tm.end();
      matvecs += ka;
      have_res = true;
    }
    if (warm_rule) CKS(choose_degrees(ka, 1));
    // the rule's degrees of this loop (for the log)
    nw_loop = std::min(nev - nl, ka);
    if (have_res)
      degrees_host(ka, mu.data(), res.data(), nev - nl, alpha, beta, tol_abs, o.deg_max,
                   rule_deg.data());
    // precision of this filter: the FP32 defect form needs the residual
    // block of the current Ritz pairs and small enough residuals
    use32 = false;
    capped.assign(ka, 0);
    if (o.precision >= 1) {
      use32 = defect_filter_safe(nev - nl, mu, res, deg, c, e, gamma, tol, norm_h);
      if (!use32) {
        std::vector<int> d2 = deg;
        if (cap_degrees_fp32(nev - nl, mu, res, d2, c, e, norm_h, capped) &&
            defect_filter_safe(nev - nl, mu, res, d2, c, e, gamma, tol, norm_h)) {
          deg.swap(d2);
          use32 = true;
        } else {
          capped.assign(ka, 0);
        }
      }
    }
    res_known_before = have_res;
    logging = o.log && log_records < o.log_capacity && have_res;
    pending.clear();
    if (logging) {
      pending.assign((size_t)nw_loop * CHFSI_LOG_FIELDS, NAN);
      for (int j = 0; j < nw_loop; ++j) {
        double* r = &pending[(size_t)j * CHFSI_LOG_FIELDS];
        const double gap = ritz_gap(ka, mu.data(), j, e);
        r[0] = it; r[1] = j; r[2] = nev - nl; r[3] = ka;
        r[4] = mu[j]; r[5] = res[j]; r[6] = gap;
        r[7] = alpha; r[8] = beta; r[9] = gamma; r[10] = norm_h; r[11] = tol_abs;
        r[12] = deg[j]; r[13] = rule_deg[j];
        int flags = 0;
        if (dsrc[j] == 1) flags |= 2;
        if (dsrc[j] == 0 && o.degree_mode == 2) flags |= 4;
        if (jittered[j]) flags |= 8;
        if (use32) flags |= 1;
        if (capped[j]) flags |= 16;
        r[15] = flags;
        degree_features(mu[j], res[j], gap, alpha, beta, gamma, norm_h, tol_abs, it, r + 16,
                        nullptr);
      }
    }
    res_before.assign(res.begin(), res.begin() + ka);
    lnrho.assign(ka, 0.0);
    for (int j = 0; j < ka; ++j) {
      const double t = (mu[j] - c) / e;
      if (std::fabs(t) > 1.0) lnrho[j] = std::log(std::fabs(t) + std::sqrt(t * t - 1.0));
    }
    // columns sorted by ascending degree (stable)
    order.resize(ka);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return deg[x] < deg[y]; });
    msort.resize(ka);
    for (int j = 0; j < ka; ++j) msort[j] = deg[order[j]];
    if (!use32) {
      tm.begin(6);
      CKS(upload_ints(s, sb.perm, order));
      CKS(upload_ints(s, sb.deg, msort));
      CK(gather_cols(s, n, ka, b.QA, ld, b.P0, ld, sb.perm));
      tm.end();
    }
    return CHFSI_OK;
  }

  // The filter of this loop on this problem alone (Alg. 2, or its FP32
  // defect form), timed with events on the stream.
  int filter_own() {
    StepBufs& sb = b.st;
    CK(hipEventRecord(fe0, s));
    if (use32) {
      tm.begin(2);
      double f32 = 0.0;
      std::vector<char> sched;
      SplitSteps sp;
      if (o.precision >= 2) {
        const bool h16 = o.precision == 3;
        sched = split_step_schedule(nev - nl, mu, res,
                                    std::vector<int>(deg.begin(), deg.begin() + ka), c, e, tol,
                                    norm_h, h16 ? FP16_SPLIT_EPS : BF16_SPLIT_EPS, h16 ? 2 : 1);
        sp.Hs = b.Hs;
        sp.Hh = b.Hh;
        sp.inv_h = b.inv_hh;
        sp.sched = &sched;
      }
      CKS(defect_filter_dev(s, n, ka, b.H32, b.QA, b.ZA, ld,
                            std::vector<double>(mu.begin(), mu.begin() + ka), order, msort, c, e,
                            gamma, b.P0, b.TMP, sb, &f32, &launches, &sp));
      flops16 += sp.flops_bf16;
      steps16 += sp.steps_bf16;
      flopsh += sp.flops_fp16;
      stepsh += sp.steps_fp16;
      tm.end();
      flops32 += f32;
      iters32 += 1;
      for (int j = 0; j < ka; ++j) filter_flops += 8.0 * (double)n * n * msort[j];
    } else {
      // Chebyshev filter (Alg. 2)
      tm.begin(2);
      CKS(filter_dev(s, n, ka, H, ldh, b.P0, b.P1, ld, msort, c, e, gamma, sb.fpart,
                     sb.fpart_elems, &filter_flops, &launches, &flops64_mfma));
      tm.end();
    }
    CK(hipEventRecord(fe1, s));
    own_filter = true;
    return CHFSI_OK;
  }

  // Batch: the defect filter's preparation on this problem's stream (tables,
  // residual block, E_0, E_1); its steps run in the group's launches.
  int defect_prepare_own() {
    StepBufs& sb = b.st;
    tm.begin(2);
    std::vector<char> sched;
    SplitSteps sp;
    if (o.precision >= 2) {
      const bool h16 = o.precision == 3;
      sched = split_step_schedule(nev - nl, mu, res,
                                  std::vector<int>(deg.begin(), deg.begin() + ka), c, e, tol,
                                  norm_h, h16 ? FP16_SPLIT_EPS : BF16_SPLIT_EPS, h16 ? 2 : 1);
      sp.Hs = b.Hs;
      sp.Hh = b.Hh;
      sp.inv_h = b.inv_hh;
      sp.sched = &sched;
    }
    CKS(defect_prepare(s, n, ka, b.QA, b.ZA, ld,
                       std::vector<double>(mu.begin(), mu.begin() + ka), order, msort, c, e,
                       gamma, b.P0, sb, &sp, dplan));
    tm.end();
    grouped_defect = true;
    iters32 += 1;
    for (int j = 0; j < ka; ++j) filter_flops += 8.0 * (double)n * n * msort[j];
    return CHFSI_OK;
  }

  // End of an outer loop: QR, Rayleigh-Ritz, residuals, log, locking and
  // the next loop's degrees.  Sets done on convergence.
  int end_loop() {
    StepBufs& sb = b.st;
    if (grouped_defect) {
      // Y = Qs diag(p_m(mu)) + E_m of the grouped defect filter
      tm.begin(2);
      CK(defect_assemble_launch(s, n, ka, b.P0, ld, sb.E0, sb.E1, sb.deg, sb.pm, b.TMP, ld));
      tm.end();
      grouped_defect = false;
    }
    for (int j = 0; j < ka; ++j) filter_mv += msort[j];
    matvecs += std::accumulate(msort.begin(), msort.end(), 0LL);
    if (!use32) {
      tm.begin(6);
      CK(gather_parity(s, n, ka, b.P0, b.P1, ld, b.TMP, ld, sb.deg));
      tm.end();
    }
    // orthonormalise against the locked vectors (the QR step of Alg. 1)
    tm.begin(3);
    int sh = 0;
    CKS(orthonormalize_dev(s, n, ka, b.TMP, ld, nl, b.QL, ld, b.QA, ld, sb, &sh));
    shifted += sh;
    tm.end();
    // Rayleigh-Ritz (the RAYLEIGH-RITZ steps of Alg. 1) and residuals
    tm.begin(4);
    int refined = 0;
    CKS(rayleigh_ritz_dev(s, n, ka, H, ldh, b.QA, ld, b.ZA, ld, b.P0, ld, b.P1, ld, sb,
                          mu.data(), res.data(), o.rr_refine, &refined));
    ++(refined ? rr_refined : rr_dense);
    std::swap(b.QA, b.P0);
    std::swap(b.ZA, b.P1);
    tm.end();
    matvecs += ka;
    if (own_filter) {
      float ms = 0.f;
      CK(hipEventElapsedTime(&ms, fe0, fe1));
      filter_sec += 1e-3 * ms;
      if (use32) sec32 += 1e-3 * ms;
    }
    // measured speed of each wanted vector; residuals below 1e-2 tol count
    // as that; an FP32 loop counts only where the residual stayed far above
    // its rounding floor (about eps32 times the residual before)
    const bool measured = res_known_before;
    have_res = true;
    tm.drain();
    if (measured) {
      const double floor32 = 1e3 * std::ldexp(1.0, -24);
      for (int j = 0; j < nw_loop; ++j) {
        if (!(lnrho[j] > 0.0) || !(res_before[j] > tol_abs) || deg[j] < 1) continue;
        if (use32 && !(res[j] > floor32 * res_before[j])) continue;
        const double after = std::max(res[j], 1e-2 * tol_abs);
        const double sp = std::log(res_before[j] / after) / (deg[j] * lnrho[j]);
        speed[j] = std::min(std::max(sp, 0.05), 8.0);
      }
    }
    if (logging) {
      for (int j = 0; j < nw_loop && log_records < o.log_capacity; ++j) {
        double* r = &pending[(size_t)j * CHFSI_LOG_FIELDS];
        r[14] = res[j];
        std::copy(r, r + CHFSI_LOG_FIELDS, o.log + (size_t)log_records * CHFSI_LOG_FIELDS);
        ++log_records;
      }
    }
    // locking (the LOCKING step): the lowest nev - nl active pairs are candidates
    const int ncand = nev - nl;
    std::vector<int> lock_idx, keep_idx;
    for (int j = 0; j < ka; ++j) {
      if (j < ncand && res[j] <= tol_abs) lock_idx.push_back(j);
      else keep_idx.push_back(j);
    }
    if (!lock_idx.empty()) {
      tm.begin(6);
      CKS(upload_ints(s, sb.perm, lock_idx));
      CK(gather_cols(s, n, (int)lock_idx.size(), b.QA, ld, b.QL + (size_t)nl * ld, ld, sb.perm));
      CKS(upload_ints(s, sb.perm, keep_idx));
      CK(gather_cols(s, n, (int)keep_idx.size(), b.QA, ld, b.P0, ld, sb.perm));
      CK(gather_cols(s, n, (int)keep_idx.size(), b.ZA, ld, b.P1, ld, sb.perm));
      std::swap(b.QA, b.P0);
      std::swap(b.ZA, b.P1);
      tm.end();
      for (int j : lock_idx) {
        lam_locked.push_back(mu[j]);
        speed_locked.push_back(speed[j]);
        max_locked_res = std::max(max_locked_res, res[j]);
      }
      std::vector<double> mu2, res2, sp2;
      for (int j : keep_idx) {
        mu2.push_back(mu[j]);
        res2.push_back(res[j]);
        sp2.push_back(speed[j]);
      }
      mu.assign(k, 0.0);
      res.assign(k, 0.0);
      speed.assign(k, NAN);
      std::copy(mu2.begin(), mu2.end(), mu.begin());
      std::copy(res2.begin(), res2.end(), res.begin());
      std::copy(sp2.begin(), sp2.end(), speed.begin());
      nl += (int)lock_idx.size();
    }
    if (nl >= nev) {
      status = CHFSI_OK;
      done = true;
      return CHFSI_OK;
    }
    const int ka2 = k - nl;
    alpha = alpha_of(nl, ka2);
    gamma = std::min(gamma, mu[0]);
    CKS(choose_degrees(ka2, it + 1));
    return CHFSI_OK;
  }

  // Output: all k pairs ascending; X = L^{-H} Y for the generalized
  // problem.  Returns the solve's status.
  int finish() {
    StepBufs& sb = b.st;
    const int kact = k - nl;
    std::vector<double> lam_all(k);
    std::vector<int> src(k);   // index into [QL | QA]
    for (int j = 0; j < nl; ++j) {
      lam_all[j] = lam_locked[j];
      src[j] = j;
    }
    for (int j = 0; j < kact; ++j) {
      lam_all[nl + j] = mu[j];
      src[nl + j] = nl + j;
    }
    std::vector<int> ord(k);
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return lam_all[x] < lam_all[y]; });
    tm.begin(7);
    // [QL | QA] side by side in P1, then one gather into X in ascending order
    CK(copy2d(s, n, nl, b.QL, ld, b.P1, ld));
    CK(copy2d(s, n, kact, b.QA, ld, b.P1 + (size_t)nl * ld, ld));
    std::vector<int> gperm(k);
    for (int j = 0; j < k; ++j) gperm[j] = src[ord[j]];
    CKS(upload_ints(s, sb.perm, gperm));
    if (gen) {
      // X = L^{-H} Y (upper-triangular operand)
      CK(gather_cols(s, n, k, b.P1, ld, b.TMP, ld, sb.perm));
      CK(zgemm(s, OP_C, OP_N, n, k, n, ONE, b.Linv, ld, b.TMP, ld, ZERO, X, ldx, false, nullptr,
               0, KTRI_A_UPPER));
    } else {
      CK(gather_cols(s, n, k, b.P1, ld, X, ldx, sb.perm));
    }
    tm.end();
    CK(hipStreamSynchronize(s));
    tm.drain();
    for (int j = 0; j < k; ++j) Lambda[j] = lam_all[ord[j]];
    if (o.seq_rates) {
      std::vector<double> sp_all(k, NAN);
      for (int j = 0; j < nl; ++j) sp_all[j] = speed_locked[j];
      for (int j = 0; j < kact; ++j) sp_all[nl + j] = speed[j];
      for (int j = 0; j < k; ++j) o.seq_rates[j] = sp_all[ord[j]];
    }

    if (info) {
      info->iters = it;
      info->converged = std::min(nl, nev);
      info->filter_launches = launches;
      info->cholqr_shifted = shifted;
      info->matvecs = matvecs;
      info->filter_matvecs = filter_mv;
      info->filter_flops = filter_flops;
      info->filter_seconds = filter_sec;
      info->filter_iters_fp32 = iters32;
      info->filter_flops_fp32 = flops32;
      info->filter_flops_bf16 = flops16;
      info->filter_steps_bf16 = steps16;
      info->filter_flops_fp16 = flopsh;
      info->filter_flops_fp64_mfma = flops64_mfma;
      info->filter_steps_fp16 = stepsh;
      info->filter_seconds_fp32 = sec32;
      info->beta = beta;
      info->norm_h = norm_h;
      info->max_resid = norm_h > 0.0 ? max_locked_res / norm_h : max_locked_res;
      info->log_records = log_records;
      info->learned_cols = learned_cols;
      info->fallback_cols = fallback_cols;
      info->learned_raised = learned_raised;
      info->rr_refined = rr_refined;
      info->rr_dense = rr_dense;
      info->total_seconds = elapsed(t_start);
    }
    return status;
  }
};

int solve_impl(int n, int nev, int nex, const zc* A, int lda, const zc* B, int ldb, double tol,
               const zc* X0, int ldx0, const double* Lambda0, double* Lambda, zc* X, int ldx,
               void* work, size_t work_bytes, const chfsi_opts& o, hipStream_t s,
               chfsi_info* info) {
  Solve S;
  S.n = n; S.nev = nev; S.nex = nex;
  S.A = A; S.lda = lda; S.B = B; S.ldb = ldb; S.tol = tol;
  S.X0 = X0; S.ldx0 = ldx0; S.Lambda0 = Lambda0; S.Lambda = Lambda; S.X = X; S.ldx = ldx;
  S.work = work; S.work_bytes = work_bytes; S.o = o; S.s = s; S.info = info;
  CKS(S.setup());
  for (;;) {
    CKS(S.begin_loop());
    if (S.done) break;
    CKS(S.filter_own());
    CKS(S.end_loop());
    if (S.done) break;
  }
  return S.finish();
}

// FP64 filters (Alg. 2) of a group of solves: step i of every solve whose
// highest degree exceeds i runs in one grouped launch.  launch() builds the
// launch arguments of all steps in pinned host memory, copies them to the
// device and queues the steps on the stream (optionally captured as one HIP
// graph) without waiting; finish() waits for them and shares the device
// time out by flops.
struct FilterGroup {
  GemmArgs* dlist = nullptr;   // device argument lists (batch workspace)
  int* dslots = nullptr;
  GemmArgs* hlist = nullptr;   // pinned staging
  int* hslots = nullptr;
  size_t cap_entries = 0, cap_slots = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<Solve*> jobs;
  std::vector<double> fl;
  int cm = 4;                  // real products per complex multiply-add of the launches
  bool pending = false;

  ~FilterGroup() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (hlist) (void)hipHostFree(hlist);
    if (hslots) (void)hipHostFree(hslots);
  }

  int init(GemmArgs* dl, int* ds, size_t ce, size_t cs) {
    dlist = dl;
    dslots = ds;
    cap_entries = ce;
    cap_slots = cs;
    CK(hipHostMalloc((void**)&hlist, sizeof(GemmArgs) * std::max<size_t>(ce, 1)));
    CK(hipHostMalloc((void**)&hslots, sizeof(int) * std::max<size_t>(cs, 1)));
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    return CHFSI_OK;
  }

  int launch(hipStream_t s, const std::vector<Solve*>& js, bool use_graph) {
    jobs = js;
    const int count = (int)jobs.size();
    int steps = 0;
    for (Solve* j : jobs) steps = std::max(steps, j->msort.back());
    std::vector<int> step_entry(steps + 1, 0), step_slot(steps + 1, 0), step_count(steps),
        step_total(steps);
    std::vector<double> sig(count), sig1(count);
    std::vector<int> first(count, 0);
    fl.assign(count, 0.0);
    for (int q = 0; q < count; ++q) {
      Solve& S = *jobs[q];
      sig1[q] = S.e / (S.gamma - S.c);
      sig[q] = sig1[q];
      while (first[q] < S.ka && S.msort[first[q]] <= 1) ++first[q];
    }
    size_t ne = 0, ns = 0;
    for (int i = 0; i < steps; ++i) {
      step_entry[i] = (int)ne;
      step_slot[i] = (int)ns;
      int total = 0, cnt = 0;
      if (ns >= cap_slots) return CHFSI_INVALID_ARG;
      hslots[ns++] = 0;
      for (int q = 0; q < count; ++q) {
        Solve& S = *jobs[q];
        if (S.msort.back() <= i) continue;
        if (ne >= cap_entries || ns >= cap_slots) return CHFSI_INVALID_ARG;
        int sl = 0;
        const double nn = (double)S.n * S.n;
        if (i == 0) {
          // Y_1 = (sigma_1 / e)(H Y_0 - c Y_0)
          hlist[ne++] = cheb_group_args(S.n, S.ka, S.H, S.ldh, S.b.P0, S.ld, nullptr, S.ld,
                                        S.b.P1, S.ld, S.c, sig1[q] / S.e, 0.0, &sl);
          fl[q] += 8.0 * nn * S.ka;
        } else {
          const double sn = 1.0 / (2.0 / sig1[q] - sig[q]);
          zc* cur = (i & 1) ? S.b.P1 : S.b.P0;
          zc* old = (i & 1) ? S.b.P0 : S.b.P1;
          const int cols = S.ka - first[q];
          const size_t off = (size_t)first[q] * S.ld;
          hlist[ne++] = cheb_group_args(S.n, cols, S.H, S.ldh, cur + off, S.ld, old + off, S.ld,
                                        old + off, S.ld, S.c, 2.0 * sn / S.e, sn * sig[q], &sl);
          fl[q] += 8.0 * nn * cols;
          sig[q] = sn;
          while (first[q] < S.ka && S.msort[first[q]] <= i + 1) ++first[q];
        }
        S.launches += 1;
        total += sl;
        hslots[ns++] = total;
        ++cnt;
      }
      step_count[i] = cnt;
      step_total[i] = total;
    }
    CK(hipMemcpyAsync(dlist, hlist, sizeof(GemmArgs) * ne, hipMemcpyHostToDevice, s));
    CK(hipMemcpyAsync(dslots, hslots, sizeof(int) * ns, hipMemcpyHostToDevice, s));
    // one tile variant per grouped launch: the tuned choice carrying the
    // most flops among the problems
    double w[FILTER_VARIANTS] = {};
    for (int q = 0; q < count; ++q) {
      const int v = filter_variant(jobs[q]->n, jobs[q]->ka);
      w[v == 2 ? DEFAULT_FILTER_VARIANT : v] += fl[q];
    }
    int variant = DEFAULT_FILTER_VARIANT;
    for (int v = 1; v < FILTER_VARIANTS; ++v)
      if (w[v] > w[variant]) variant = v;
    cm = variant_cm(variant);
    CK(hipEventRecord(e0, s));
    if (use_graph) {
      CK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      int err = 0;
      for (int i = 0; i < steps && !err; ++i)
        err = cheb_step_group(s, dlist + step_entry[i], dslots + step_slot[i], step_count[i],
                              step_total[i], variant);
      const int cap_err = (int)hipStreamEndCapture(s, &graph);
      if (err || cap_err) return CHFSI_DEVICE_ERROR;
      CK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
      CK(hipGraphLaunch(gexec, s));
    } else {
      for (int i = 0; i < steps; ++i)
        CK(cheb_step_group(s, dlist + step_entry[i], dslots + step_slot[i], step_count[i],
                           step_total[i], variant));
    }
    CK(hipEventRecord(e1, s));
    pending = true;
    return CHFSI_OK;
  }

  int finish() {
    if (!pending) return CHFSI_OK;
    pending = false;
    CK(hipEventSynchronize(e1));
    if (gexec) {
      (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    }
    if (graph) {
      (void)hipGraphDestroy(graph);
      graph = nullptr;
    }
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    double ftot = 0.0;
    for (double f : fl) ftot += f;
    for (size_t q = 0; q < jobs.size(); ++q) {
      jobs[q]->filter_flops += fl[q];
      jobs[q]->flops64_mfma += fl[q] * cm / 4.0;
      if (ftot > 0.0) jobs[q]->filter_sec += 1e-3 * ms * fl[q] / ftot;
    }
    return CHFSI_OK;
  }
};

// The mixed-precision defect filters of a group's problems in grouped
// launches: per recurrence step one launch per form present at that step
// (FP16-split, BF16-split, FP32) over all those problems' windows, each
// split form preceded by one launch that splits the problems' E_i columns
// (where the previous step did not leave the split).  The problems'
// preparation (tables, residual blocks) and assembly run on their own
// streams; every launch argument of a loop is built on the host and
// uploaded once.  No split-K (the problems together fill the GPU).
struct DefectGroup {
  char* dargs = nullptr;   // device argument arrays (batch workspace)
  int* dslots = nullptr;
  char* hargs = nullptr;   // pinned staging
  int* hslots = nullptr;
  size_t cap_bytes = 0, cap_slots = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<Solve*> jobs;
  std::vector<double> fl;
  bool pending = false;
  // one launch: form (0 FP32 step, 1 BF16 step, 2 FP16 step, 3 BF16 column
  // split, 4 FP16 column split), tile, argument and slot offsets, size
  struct Launch {
    int form;
    bool wide;
    size_t arg_off, slot_off;
    int count, total;
  };
  std::vector<Launch> plan;

  ~DefectGroup() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (hargs) (void)hipHostFree(hargs);
    if (hslots) (void)hipHostFree(hslots);
  }

  int init(char* da, int* ds, size_t cb, size_t cs) {
    dargs = da;
    dslots = ds;
    cap_bytes = cb;
    cap_slots = cs;
    CK(hipHostMalloc((void**)&hargs, std::max<size_t>(cb, 1)));
    CK(hipHostMalloc((void**)&hslots, sizeof(int) * std::max<size_t>(cs, 1)));
    CK(hipEventCreate(&e0));
    CK(hipEventCreate(&e1));
    return CHFSI_OK;
  }

  int launch(hipStream_t s, const std::vector<Solve*>& js) {
    jobs = js;
    plan.clear();
    const int count = (int)jobs.size();
    fl.assign(count, 0.0);
    int steps = 0;
    for (Solve* j : jobs) steps = std::max(steps, j->dplan.mmax);
    const size_t arg_sz[5] = {defect_group_arg_bytes(), split_group_arg_bytes(),
                              split_group_arg_bytes(), colsplit_group_arg_bytes(),
                              colsplit_group_arg_bytes()};
    size_t ab = 0, ns = 0;
    std::vector<char> ready(count, 0);   // split panel of E_i holds the window (BF16)
    const int wide_min = split_wide_min_cols();
    for (int i = 1; i < steps; ++i) {
      // the step's entries per form, in the order they are launched
      struct Ent {
        int q, cols, first;
        bool next;
      };
      std::vector<Ent> by[5];
      for (int q = 0; q < count; ++q) {
        const DefectPlan& p = jobs[q]->dplan;
        if (i >= p.mmax) continue;
        const int first = p.first[i], cols = p.k - first;
        const int kd = p.kind[i];
        if (kd == 2) {
          by[4].push_back({q, cols, first, false});
          by[2].push_back({q, cols, first, false});
          ready[q] = 0;
        } else if (kd == 1) {
          const bool next = i + 1 < p.mmax && p.kind[i + 1] == 1;
          if (!ready[q]) by[3].push_back({q, cols, first, false});
          by[1].push_back({q, cols, first, next});
          ready[q] = next;
        } else {
          by[0].push_back({q, cols, first, false});
          ready[q] = 0;
        }
      }
      const int order[5] = {4, 3, 2, 1, 0};
      for (int f : order) {
        if (by[f].empty()) continue;
        Launch L = {};
        L.form = f;
        ab = (ab + 255) / 256 * 256;
        L.arg_off = ab;
        L.slot_off = ns;
        L.count = (int)by[f].size();
        if (ab + arg_sz[f] * L.count > cap_bytes || ns + L.count + 1 > cap_slots)
          return CHFSI_INVALID_ARG;
        if (f == 1 || f == 2) {   // tile: the one carrying more of the flops
          double w = 0.0, tot = 0.0;
          for (const Ent& x : by[f]) {
            const double fx = (double)jobs[x.q]->n * jobs[x.q]->n * x.cols;
            tot += fx;
            if (x.cols >= wide_min) w += fx;
          }
          L.wide = 2.0 * w > tot;
        }
        int total = 0;
        hslots[ns] = 0;
        for (int e = 0; e < L.count; ++e) {
          const Ent& x = by[f][e];
          Solve& S = *jobs[x.q];
          StepBufs& sb = S.b.st;
          const int n = S.n, k = S.dplan.k;
          const size_t off = (size_t)x.first * n * 8;   // complex64 window offset
          const size_t srow = (size_t)split_kp(n) * 8;
          const char* cur = (const char*)((i & 1) ? sb.E1 : sb.E0);
          char* old = (char*)((i & 1) ? sb.E0 : sb.E1);
          const float* cri = sb.crtab + (size_t)i * k + x.first;
          const DefectStepScalars sc = defect_scalars(S.dplan, i);
          void* out = hargs + L.arg_off + arg_sz[f] * e;
          int wg = 0;
          if (f == 0) {
            wg = defect_group_fill(n, x.cols, S.b.H32, cur + off, old + off, old + off,
                                   (const char*)sb.R32 + off, cri, sc.shift, sc.sa, sc.sb, out);
            S.flops32 += 8.0 * (double)n * n * x.cols;
          } else if (f == 1 || f == 2) {
            const bool h16 = f == 2;
            char* scur = (char*)((h16 || !(i & 1)) ? sb.S0 : sb.S1) + x.first * srow;
            char* snext = (char*)((i & 1) ? sb.S0 : sb.S1) + x.first * srow;
            wg = split_group_fill(h16, L.wide, n, x.cols, h16 ? S.b.Hh : S.b.Hs, S.b.inv_hh,
                                  scur, sb.colscale + x.first, cur + off, old + off, old + off,
                                  (const char*)sb.R32 + off, cri, sc.shift, sc.sa, sc.sb,
                                  x.next ? snext : nullptr, out);
            if (h16) {
              S.flopsh += 8.0 * (double)n * n * x.cols;
              S.stepsh += 1;
            } else {
              S.flops16 += 8.0 * (double)n * n * x.cols;
              S.steps16 += 1;
            }
          } else {
            const bool h16 = f == 4;
            char* scur = (char*)((h16 || !(i & 1)) ? sb.S0 : sb.S1) + x.first * srow;
            colsplit_group_fill(n, cur + off, n, scur, sb.colscale + x.first, out);
            wg = x.cols;
          }
          if (f <= 2) {
            fl[x.q] += 8.0 * (double)n * n * x.cols;
            S.launches += 1;
          }
          total += wg;
          hslots[ns + e + 1] = total;
        }
        L.total = total;
        ns += L.count + 1;
        ab += arg_sz[f] * L.count;
        plan.push_back(L);
      }
    }
    if (ab) CK(hipMemcpyAsync(dargs, hargs, ab, hipMemcpyHostToDevice, s));
    if (ns) CK(hipMemcpyAsync(dslots, hslots, sizeof(int) * ns, hipMemcpyHostToDevice, s));
    CK(hipEventRecord(e0, s));
    for (const Launch& L : plan) {
      const char* a = dargs + L.arg_off;
      const int* sl = dslots + L.slot_off;
      if (L.form == 0) CK(defect_group_launch(s, a, sl, L.count, L.total));
      else if (L.form <= 2) CK(split_group_launch(s, L.form == 2, L.wide, a, sl, L.count, L.total));
      else CK(colsplit_group_launch(s, L.form == 4, a, sl, L.count, L.total));
    }
    CK(hipEventRecord(e1, s));
    pending = true;
    return CHFSI_OK;
  }

  int finish() {
    if (!pending) return CHFSI_OK;
    pending = false;
    CK(hipEventSynchronize(e1));
    float ms = 0.f;
    CK(hipEventElapsedTime(&ms, e0, e1));
    double ftot = 0.0;
    for (double f : fl) ftot += f;
    for (size_t q = 0; q < jobs.size(); ++q) {
      if (ftot <= 0.0) break;
      const double t = 1e-3 * ms * fl[q] / ftot;
      jobs[q]->filter_sec += t;
      jobs[q]->sec32 += t;
    }
    return CHFSI_OK;
  }
};

// Launch-argument capacity of the batch workspace for `count` solves (two
// groups): the grouped FP64 filter (one entry per problem and step) and the
// grouped defect filter (per step, at most two launches per problem: its
// column split and its step).
void batch_caps(int count, const chfsi_opts& o, size_t* entries, size_t* slots) {
  const size_t steps = (size_t)std::max(std::max(o.deg0, o.deg_max), 1);
  *entries = steps * (size_t)count;
  *slots = steps * ((size_t)count + 1);
}

void batch_defect_caps(int count, const chfsi_opts& o, size_t* bytes, size_t* slots) {
  const size_t steps = (size_t)std::max(std::max(o.deg0, o.deg_max), 1);
  const size_t a = std::max(defect_group_arg_bytes(),
                            std::max(split_group_arg_bytes(), colsplit_group_arg_bytes()));
  *bytes = steps * (2 * (size_t)count * a + 5 * 256);
  *slots = steps * 5 * ((size_t)count + 1);
}

size_t batch_bytes(int count, const chfsi_opts& o) {
  size_t entries = 0, slots = 0, dbytes = 0, dslots = 0;
  batch_caps(count, o, &entries, &slots);
  batch_defect_caps(count, o, &dbytes, &dslots);
  Carver c(nullptr);
  for (int g = 0; g < 2; ++g) {
    c.take<GemmArgs>(entries);
    c.take<int>(slots);
    c.take<char>(dbytes);
    c.take<int>(dslots);
  }
  return c.off + ALIGN;
}

// Solves of a batch, run as two pipelined groups.  Every problem runs on one
// of up to 8 worker streams, driven by a host thread of its group with its
// own rocSOLVER handle, so the per-problem phases -- reduction, Lanczos, QR,
// Rayleigh-Ritz with its latency-bound reduced eigensolve, locking -- of
// different problems overlap on the GPU.  Each group runs its loops in
// lockstep: begin_loop on its unfinished problems (FP32 defect filters run
// right there, on the problem's stream), its FP64 filters in grouped
// launches on the caller's stream, end_loop.  The two groups alternate on
// the caller's stream, so one group's QR / Rayleigh-Ritz / locking run while
// the other group's filter occupies the matrix cores.  With `serial`, one
// group, one stream, no threads.  status[q] receives each problem's result.
constexpr int BATCH_WORKERS = 8;

int solve_batch_impl(std::vector<std::unique_ptr<Solve>>& S, hipStream_t s, void* bwork,
                     size_t bbytes, bool graph, bool serial, bool own_defect,
                     std::vector<int>& status) {
  const int count = (int)S.size();
  size_t cap_entries = 0, cap_slots = 0, cap_dbytes = 0, cap_dslots = 0;
  batch_caps(count, S[0]->o, &cap_entries, &cap_slots);
  batch_defect_caps(count, S[0]->o, &cap_dbytes, &cap_dslots);
  if (bbytes < batch_bytes(count, S[0]->o)) return CHFSI_INVALID_ARG;
  int dev = 0;
  CK(hipGetDevice(&dev));
  const int ngroups = (serial || count < 2) ? 1 : 2;
  const int T = serial ? 1 : std::min(count, BATCH_WORKERS);

  // groups: problems by decreasing n dealt alternately; worker threads and
  // streams split between the groups
  std::vector<int> byn(count);
  std::iota(byn.begin(), byn.end(), 0);
  std::stable_sort(byn.begin(), byn.end(), [&](int a, int b) { return S[a]->n > S[b]->n; });
  std::vector<std::vector<int>> members(ngroups);
  for (int i = 0; i < count; ++i) members[i % ngroups].push_back(byn[i]);
  std::vector<int> t0(ngroups), tn(ngroups);
  for (int g = 0; g < ngroups; ++g) {
    tn[g] = ngroups == 1 ? T : std::max(1, T / 2);
    t0[g] = g * (T / ngroups);
    tn[g] = std::min(tn[g], (int)members[g].size());
  }

  // resources of the call, released on every path
  struct Res {
    std::vector<hipStream_t> st;
    std::vector<rocblas_handle> h;
    std::vector<hipEvent_t> ev;
    ~Res() {
      for (auto x : st) if (x) { (void)hipStreamSynchronize(x); (void)hipStreamDestroy(x); }
      for (auto x : h) if (x) rocblas_destroy_handle(x);
      for (auto x : ev) if (x) (void)hipEventDestroy(x);
    }
  } r;
  r.st.assign(T, nullptr);
  r.h.assign(T, nullptr);
  r.ev.assign(T + 1, nullptr);
  for (int t = 0; t < T; ++t) {
    CK(hipStreamCreateWithFlags(&r.st[t], hipStreamNonBlocking));
    if (rocblas_create_handle(&r.h[t]) != rocblas_status_success) return CHFSI_DEVICE_ERROR;
  }
  for (auto& e : r.ev) CK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  hipEvent_t ev_main = r.ev[T];
  std::vector<FilterGroup> fg(ngroups);
  std::vector<DefectGroup> dg(ngroups);
  Carver cv(bwork);
  for (int g = 0; g < ngroups; ++g) {
    GemmArgs* dl = cv.take<GemmArgs>(cap_entries);
    int* ds = cv.take<int>(cap_slots);
    CKS(fg[g].init(dl, ds, cap_entries, cap_slots));
    char* da = cv.take<char>(cap_dbytes);
    int* dd = cv.take<int>(cap_dslots);
    CKS(dg[g].init(da, dd, cap_dbytes, cap_dslots));
  }
  // inputs written on the caller's stream are visible to the workers
  CK(hipEventRecord(ev_main, s));
  for (int t = 0; t < T; ++t) CK(hipStreamWaitEvent(r.st[t], ev_main, 0));
  std::vector<int> thread_of(count, 0);
  for (int g = 0; g < ngroups; ++g)
    for (size_t i = 0; i < members[g].size(); ++i) {
      const int q = members[g][i];
      thread_of[q] = t0[g] + (int)(i % tn[g]);
      S[q]->s = r.st[thread_of[q]];
    }

  status.assign(count, CHFSI_OK);
  std::vector<char> failed(count, 0), active(count, 0);
  // run fn(q) for the group's problems, each on its worker's host thread
  auto parallel = [&](int g, auto fn) {
    auto work = [&](int t) {
      if (hipSetDevice(dev) != hipSuccess) {
        for (int q : members[g])
          if (thread_of[q] == t) {
            status[q] = CHFSI_DEVICE_ERROR;
            failed[q] = 1;
          }
        return;
      }
      tl_handle = r.h[t];
      for (int q : members[g]) {
        if (thread_of[q] != t) continue;
        try {
          fn(q);
        } catch (const std::bad_alloc&) {
          status[q] = CHFSI_ALLOC_ERROR;
          failed[q] = 1;
        } catch (...) {
          status[q] = CHFSI_DEVICE_ERROR;
          failed[q] = 1;
        }
      }
      tl_handle = nullptr;
    };
    if (serial) {            // the calling thread drives the one worker stream
      work(0);
      return;
    }
    std::vector<std::thread> th;
    for (int t = t0[g]; t < t0[g] + tn[g]; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  };
  // begin_loop on the group's unfinished problems, then its grouped filter
  // queued on the caller's stream after their workers' work; returns whether
  // the group still has work
  auto begin_and_launch = [&](int g, bool& live) -> int {
    parallel(g, [&](int q) {
      active[q] = 0;
      if (failed[q] || S[q]->done) return;
      status[q] = S[q]->begin_loop();
      if (status[q] == CHFSI_OK && !S[q]->done && S[q]->use32 && S[q]->ka > 0)
        status[q] = own_defect ? S[q]->filter_own() : S[q]->defect_prepare_own();
      if (status[q] != CHFSI_OK) {
        failed[q] = 1;
        return;
      }
      if (!S[q]->done) active[q] = 1;
    });
    std::vector<Solve*> fp64, mixed;
    live = false;
    for (int q : members[g]) {
      if (!active[q]) continue;
      live = true;
      if (!S[q]->use32 && S[q]->ka > 0) fp64.push_back(S[q].get());
      if (S[q]->grouped_defect) mixed.push_back(S[q].get());
    }
    if (fp64.empty() && mixed.empty()) return CHFSI_OK;
    for (int t = t0[g]; t < t0[g] + tn[g]; ++t) {
      CK(hipEventRecord(r.ev[t], r.st[t]));
      CK(hipStreamWaitEvent(s, r.ev[t], 0));
    }
    if (!fp64.empty()) CKS(fg[g].launch(s, fp64, graph));
    if (!mixed.empty()) CKS(dg[g].launch(s, mixed));
    // the group's workers continue after its filters
    hipEvent_t done_ev = !mixed.empty() ? dg[g].e1 : fg[g].e1;
    for (int t = t0[g]; t < t0[g] + tn[g]; ++t) CK(hipStreamWaitEvent(r.st[t], done_ev, 0));
    return CHFSI_OK;
  };

  for (int g = 0; g < ngroups; ++g)
    parallel(g, [&](int q) {
      status[q] = S[q]->setup();
      if (status[q] != CHFSI_OK) failed[q] = 1;
    });
  std::vector<char> live(ngroups, 0);
  for (int g = 0; g < ngroups; ++g) {
    bool l = false;
    CKS(begin_and_launch(g, l));
    live[g] = l;
  }
  for (;;) {
    bool any = false;
    for (int g = 0; g < ngroups; ++g) {
      if (!live[g]) continue;
      CKS(fg[g].finish());
      CKS(dg[g].finish());
      parallel(g, [&](int q) {
        if (!active[q]) return;
        status[q] = S[q]->end_loop();
        if (status[q] != CHFSI_OK) failed[q] = 1;
      });
      bool l = false;
      CKS(begin_and_launch(g, l));
      live[g] = l;
      any = any || l;
    }
    if (!any) break;
  }
  for (int g = 0; g < ngroups; ++g)
    parallel(g, [&](int q) {
      if (!failed[q]) status[q] = S[q]->finish();
    });
  // outputs complete on the workers before the caller's stream goes on
  for (int t = 0; t < T; ++t) {
    CK(hipEventRecord(r.ev[t], r.st[t]));
    CK(hipStreamWaitEvent(s, r.ev[t], 0));
  }
  CK(hipStreamSynchronize(s));
  return CHFSI_OK;
}

int check_ptr(const void* p) { return (p && aligned16(p)) ? CHFSI_OK : CHFSI_INVALID_ARG; }

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// Argument checks of chfsi_solve (no device calls).
int validate_solve(int n, int nev, int nex, const void* A, int lda, const void* B, int ldb,
                   double tol, const void* X0, int ldx0, const double* Lambda0, double* Lambda,
                   void* X, int ldx, void* work, const chfsi_opts& o) {
    const int k = nev + nex;
    if (n < 1 || nev < 1 || nex < 1 || k > n || !(tol > 0.0) || lda < n || ldx < n) return CHFSI_INVALID_ARG;
    if (check_ptr(A) || check_ptr(X) || check_ptr(work) || !Lambda) return CHFSI_INVALID_ARG;
    if (B && (ldb < n || !aligned16(B))) return CHFSI_INVALID_ARG;
    if (X0 && (ldx0 < n || !aligned16(X0))) return CHFSI_INVALID_ARG;
    if (o.deg0 < 1 || o.deg_max < 1 || o.max_iter < 1 || o.lanczos_steps < 1) return CHFSI_INVALID_ARG;
    if (o.precision < 0 || o.precision > 3) return CHFSI_INVALID_ARG;
    if (o.rr_refine < 0 || o.rr_refine > 1) return CHFSI_INVALID_ARG;
    if (o.degree_mode < 0 || o.degree_mode > 3 || o.first_rule < 0 || o.first_rule > 1)
      return CHFSI_INVALID_ARG;
    if (o.degree_mode == 3 && !o.seq_rates) return CHFSI_INVALID_ARG;
    if (!(o.degree_jitter >= 0.0) || !std::isfinite(o.degree_jitter)) return CHFSI_INVALID_ARG;
    if (o.log_capacity < 0 || (o.log_capacity > 0 && !o.log)) return CHFSI_INVALID_ARG;
    if (o.degree_mode == 2) {
      if (!o.mlp) return CHFSI_INVALID_ARG;
      for (int i = 0; i < MLP_PARAMS; ++i)
        if (!std::isfinite(o.mlp[i])) return CHFSI_NONFINITE;
    }
    if (o.precision >= 1 && (o.deg0 > CR_ROWS || o.deg_max > CR_ROWS)) return CHFSI_INVALID_ARG;
    if (X0 == X && ldx0 != ldx) return CHFSI_INVALID_ARG;
    if (Lambda0) {
      if (!X0) return CHFSI_INVALID_ARG;
      for (int j = 0; j < k; ++j) {
        if (!std::isfinite(Lambda0[j])) return CHFSI_NONFINITE;
        if (j > 0 && Lambda0[j] < Lambda0[j - 1]) return CHFSI_INVALID_ARG;
      }
      if (!(Lambda0[k - 1] > Lambda0[0])) return CHFSI_INVALID_ARG;
    }
    return CHFSI_OK;
}


}  // namespace
}  // namespace chfsi

using namespace chfsi;

// Device scratch of chfsi_filter_noalloc: one copy per GPU, held until the
// process ends.  Host code never uses this name as an address (on the host
// it is only a stand-in for the symbol): the device address of each GPU's
// copy comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char scratch[CHFSI_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the current GPU's scratch (looked up on the first call
// on that device, with the device current); status code.
int noalloc_scratch(void** out) {
  int dev = 0;
  CK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return CHFSI_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    CK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return CHFSI_DEVICE_ERROR;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CHFSI_OK;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" {

size_t chfsi_filter_noalloc_need_bytes(int n, int k) {
  if (n < 1 || k < 1) return 0;
  const size_t nk = (size_t)n * (size_t)k;
  return 2 * round256(nk * sizeof(zc)) + round256(sizeof(int) * (size_t)k);
}

int chfsi_default_opts(chfsi_opts* o) {
  if (!o) return CHFSI_INVALID_ARG;
  o->tol = 1e-10;
  o->deg0 = 10;
  o->deg_max = 40;
  o->max_iter = 100;
  o->lanczos_steps = 20;
  o->alpha_rule = 0;
  o->degree_mode = 0;
  o->reuse_b_factor = 1;
  o->precision = 0;
  o->seed = 0;
  o->degree_jitter = 0.0;
  o->first_rule = 0;
  o->log_capacity = 0;
  o->log = nullptr;
  o->mlp = nullptr;
  o->seq_rates = nullptr;
  o->rr_refine = 1;
  return CHFSI_OK;
}

size_t chfsi_batch_workspace_bytes(int count, const chfsi_opts* opts) {
  if (count < 1) return 0;
  chfsi_opts o;
  chfsi_default_opts(&o);
  if (opts) o = *opts;
  return batch_bytes(count, o);
}

int chfsi_solve_batch(int count, const int* n, const int* nev, const int* nex,
                      const void* const* A, const int* lda, const void* const* B, const int* ldb,
                      double tol, const void* const* X0, const int* ldx0,
                      const double* const* Lambda0, double* const* Lambda, void* const* X,
                      const int* ldx, void* const* work, const size_t* work_bytes,
                      void* batch_work, size_t batch_work_bytes, const chfsi_opts* opts, int flags,
                      void* stream, chfsi_info* info, int* status) {
  try {
    if (count < 1 || !n || !nev || !nex || !A || !lda || !Lambda || !X || !ldx || !work ||
        !work_bytes || !status || check_ptr(batch_work) || (flags & ~7))
      return CHFSI_INVALID_ARG;
    if ((B && !ldb) || (X0 && !ldx0)) return CHFSI_INVALID_ARG;
    if ((flags & 1) && !stream) return CHFSI_INVALID_ARG;   // no capture on the null stream
    chfsi_opts o;
    chfsi_default_opts(&o);
    if (opts) o = *opts;
    o.tol = tol;
    if (o.log_capacity != 0 || o.seq_rates) return CHFSI_INVALID_ARG;   // no shared host arrays
    for (int q = 0; q < count; ++q) {
      const void* bq = B ? B[q] : nullptr;
      const void* xq = X0 ? X0[q] : nullptr;
      const double* lq = Lambda0 ? Lambda0[q] : nullptr;
      CKS(validate_solve(n[q], nev[q], nex[q], A[q], lda[q], bq, bq ? ldb[q] : 0, tol, xq,
                         xq ? ldx0[q] : 0, lq, Lambda[q], X[q], ldx[q], work[q], o));
      for (int r = 0; r < q; ++r)
        if (work[r] == work[q]) return CHFSI_INVALID_ARG;   // workspaces must be distinct
    }
    if (batch_work_bytes < batch_bytes(count, o)) return CHFSI_INVALID_ARG;
    std::vector<std::unique_ptr<Solve>> S(count);
    for (int q = 0; q < count; ++q) {
      S[q].reset(new Solve());
      Solve& v = *S[q];
      v.n = n[q]; v.nev = nev[q]; v.nex = nex[q];
      v.A = (const zc*)A[q]; v.lda = lda[q];
      v.B = B ? (const zc*)B[q] : nullptr; v.ldb = v.B ? ldb[q] : 0;
      v.tol = tol;
      v.X0 = X0 ? (const zc*)X0[q] : nullptr; v.ldx0 = v.X0 ? ldx0[q] : 0;
      v.Lambda0 = Lambda0 ? Lambda0[q] : nullptr;
      v.Lambda = Lambda[q]; v.X = (zc*)X[q]; v.ldx = ldx[q];
      v.work = work[q]; v.work_bytes = work_bytes[q];
      v.o = o; v.s = as_stream(stream);
      v.info = info ? &info[q] : nullptr;
      if (v.info) std::memset(v.info, 0, sizeof(chfsi_info));
    }
    std::vector<int> st;
    CKS(solve_batch_impl(S, as_stream(stream), batch_work, batch_work_bytes, (flags & 1) != 0,
                         (flags & 2) != 0, (flags & 4) != 0, st));
    int worst = CHFSI_OK;
    for (int q = 0; q < count; ++q) {
      status[q] = st[q];
      if (st[q] != CHFSI_OK && (worst == CHFSI_OK || worst == CHFSI_NO_CONVERGENCE)) worst = st[q];
    }
    return worst;
  } catch (const std::bad_alloc&) {
    return CHFSI_ALLOC_ERROR;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

const char* chfsi_status_string(int status) {
  switch (status) {
    case CHFSI_OK: return "success";
    case CHFSI_INVALID_ARG: return "invalid argument";
    case CHFSI_NOT_HPD: return "matrix is not Hermitian positive definite";
    case CHFSI_NO_CONVERGENCE: return "no convergence within max_iter";
    case CHFSI_NONFINITE: return "non-finite input";
    case CHFSI_DEVICE_ERROR: return "device error";
    case CHFSI_ALLOC_ERROR: return "host allocation failure";
    default: return "unknown status";
  }
}

size_t chfsi_workspace_bytes(int n, int nev, int nex, int generalized, const chfsi_opts* opts) {
  if (n < 1 || nev < 1 || nex < 1 || nev + nex > n) return 0;
  chfsi_opts o;
  chfsi_default_opts(&o);
  if (opts) o = *opts;
  SolveBufs b;
  Carver c(nullptr);
  return carve_solve(c, b, n, nev, nex, generalized != 0, std::max(o.lanczos_steps, 1),
                     o.precision);
}


int chfsi_solve(int n, int nev, int nex, const void* A, int lda, const void* B, int ldb, double tol,
                const void* X0, int ldx0, const double* Lambda0, double* Lambda, void* X, int ldx,
                void* work, size_t work_bytes, const chfsi_opts* opts, void* stream,
                chfsi_info* info) {
  try {
    chfsi_opts o;
    chfsi_default_opts(&o);
    if (opts) o = *opts;
    o.tol = tol;
    CKS(validate_solve(n, nev, nex, A, lda, B, ldb, tol, X0, ldx0, Lambda0, Lambda, X, ldx, work,
                       o));
    if (info) std::memset(info, 0, sizeof(*info));
    return solve_impl(n, nev, nex, (const zc*)A, lda, (const zc*)B, ldb, tol, (const zc*)X0, ldx0,
                      Lambda0, Lambda, (zc*)X, ldx, work, work_bytes, o, as_stream(stream), info);
  } catch (const std::bad_alloc&) {
    return CHFSI_ALLOC_ERROR;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

size_t chfsi_step_workspace_bytes(int n, int k) {
  if (n < 1 || k < 1) return 0;
  StepBufs b;
  Carver c(nullptr);
  carve_step(c, b, n, k, k, 20);
  return c.off + ALIGN;
}

size_t chfsi_eigh_workspace_bytes(int k) { return chfsi_step_workspace_bytes(k, k); }

int chfsi_eigh_projected(int k, const void* G, int ldg, void* W, int ldw, double* mu, int mode,
                         void* work, size_t work_bytes, void* stream, int* refined_out) {
  try {
    if (k < 1 || ldg < k || ldw < k || !mu || mode < 0 || mode > 2) return CHFSI_INVALID_ARG;
    if (check_ptr(G) || check_ptr(W) || check_ptr(work)) return CHFSI_INVALID_ARG;
    if (work_bytes < chfsi_eigh_workspace_bytes(k)) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    StepBufs b;
    Carver cv(work);
    carve_step(cv, b, k, k, k, 20);
    CK(copy2d(s, k, k, (const zc*)G, ldg, b.G, k));
    int refined = 0;
    CKS(eigh_projected(s, k, b, mode, &refined));
    CK(copy2d(s, k, k, refined ? b.K2 : b.G, k, (zc*)W, ldw));
    CK(hipMemcpyAsync(mu, b.mu, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (refined_out) *refined_out = refined;
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_filter(int n, int k, const void* H, int ldh, void* Y, int ldy, const int* degrees,
                 double c, double e, double gamma, void* work, size_t work_bytes, void* stream,
                 double* flops_out, int* launches_out) {
  try {
    if (n < 1 || k < 1 || ldh < n || ldy < n || !degrees || !(e > 0.0) || gamma == c)
      return CHFSI_INVALID_ARG;
    if (check_ptr(H) || check_ptr(Y) || check_ptr(work)) return CHFSI_INVALID_ARG;
    for (int j = 0; j < k; ++j) {
      if (degrees[j] < 1 || (j > 0 && degrees[j] < degrees[j - 1])) return CHFSI_INVALID_ARG;
    }
    if (work_bytes < chfsi_step_workspace_bytes(n, k)) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    StepBufs b;
    Carver cv(work);
    carve_step(cv, b, n, k, k, 20);
    std::vector<int> m(degrees, degrees + k);
    // P0 = a packed copy of Y, P1 = T2
    CK(copy2d(s, n, k, (const zc*)Y, ldy, b.T1, n));
    double fl = 0.0;
    int ln = 0;
    CKS(filter_dev(s, n, k, (const zc*)H, ldh, b.T1, b.T2, n, m, c, e, gamma, b.fpart,
                   b.fpart_elems, &fl, &ln));
    CKS(upload_ints(s, b.deg, m));
    CK(gather_parity(s, n, k, b.T1, b.T2, n, (zc*)Y, ldy, b.deg));
    CK(hipStreamSynchronize(s));
    if (flops_out) *flops_out = fl;
    if (launches_out) *launches_out = ln;
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_filter_noalloc(int n, int k, const void* H, int ldh, void* Y, int ldy,
                         const int* degrees, double c, double e, double gamma, void* stream,
                         double* flops_out, int* launches_out) {
  try {
    if (n < 1 || k < 1 || ldh < n || ldy < n || !degrees || !(e > 0.0) || gamma == c)
      return CHFSI_INVALID_ARG;
    if (check_ptr(H) || check_ptr(Y)) return CHFSI_INVALID_ARG;
    for (int j = 0; j < k; ++j) {
      if (degrees[j] < 1 || (j > 0 && degrees[j] < degrees[j - 1])) return CHFSI_INVALID_ARG;
    }
    const size_t need = chfsi_filter_noalloc_need_bytes(n, k);
    if (need > (size_t)CHFSI_NOALLOC_SCRATCH_BYTES) return CHFSI_INVALID_ARG;
    void* base = nullptr;
    CKS(noalloc_scratch(&base));
    hipStream_t s = as_stream(stream);
    // scratch: ping-pong blocks P0, P1 (packed n x k), the degrees, and the
    // rest for split-K partial sums (up to CHEB_MAX_SPLITS blocks; fewer
    // splits when less room is left)
    const size_t nk = (size_t)n * (size_t)k;
    char* p = (char*)base;
    zc* P0 = (zc*)p;
    p += round256(nk * sizeof(zc));
    zc* P1 = (zc*)p;
    p += round256(nk * sizeof(zc));
    int* deg = (int*)p;
    p += round256(sizeof(int) * (size_t)k);
    zc* part = (zc*)p;
    const size_t left = (size_t)CHFSI_NOALLOC_SCRATCH_BYTES - need;
    const size_t part_elems = std::min(left / sizeof(zc), (size_t)CHEB_MAX_SPLITS * nk);
    std::vector<int> m(degrees, degrees + k);
    CK(copy2d(s, n, k, (const zc*)Y, ldy, P0, n));
    double fl = 0.0;
    int ln = 0;
    CKS(filter_dev(s, n, k, (const zc*)H, ldh, P0, P1, n, m, c, e, gamma,
                   part_elems >= 2 * nk ? part : nullptr, part_elems, &fl, &ln));
    CKS(upload_ints(s, deg, m));
    CK(gather_parity(s, n, k, P0, P1, n, (zc*)Y, ldy, deg));
    CK(hipStreamSynchronize(s));
    if (flops_out) *flops_out = fl;
    if (launches_out) *launches_out = ln;
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

size_t chfsi_defect_workspace_bytes(int n, int k) {
  if (n < 1 || k < 1) return 0;
  StepBufs b;
  Carver c(nullptr);
  carve_step(c, b, n, k, k, 20);
  c.take<char>((size_t)n * n * 8);
  return c.off + ALIGN;
}

int chfsi_filter_defect(int n, int k, const void* H, int ldh, const void* Q, int ldq,
                        const void* Z, int ldz, const double* mu, const int* degrees, double c,
                        double e, double gamma, void* Y, int ldy, void* work, size_t work_bytes,
                        void* stream, double* flops_out) {
  try {
    if (n < 1 || k < 1 || k > n || ldh < n || ldq != n || ldz != n || ldy < n || !mu ||
        !degrees || !(e > 0.0) || gamma == c)
      return CHFSI_INVALID_ARG;
    if (check_ptr(H) || check_ptr(Q) || check_ptr(Z) || check_ptr(Y) || check_ptr(work))
      return CHFSI_INVALID_ARG;
    for (int j = 0; j < k; ++j) {
      if (degrees[j] < 1 || degrees[j] > CR_ROWS || (j > 0 && degrees[j] < degrees[j - 1]))
        return CHFSI_INVALID_ARG;
    }
    if (work_bytes < chfsi_defect_workspace_bytes(n, k)) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    StepBufs b;
    Carver cv(work);
    carve_step(cv, b, n, k, k, 20);
    void* H32 = cv.take<char>((size_t)n * n * 8);
    CK(matrix_to_fp32(s, n, (const zc*)H, ldh, H32));
    std::vector<int> order(k), m(degrees, degrees + k);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> muv(mu, mu + k);
    double f32 = 0.0;
    int launches = 0;
    // Qs -> T1 (packed); Y written with its own leading dimension
    CKS(defect_filter_dev(s, n, k, H32, (const zc*)Q, (const zc*)Z, n, muv, order, m, c, e, gamma,
                          b.T1, b.T2, b, &f32, &launches));
    CK(copy2d(s, n, k, b.T2, n, (zc*)Y, ldy));
    CK(hipStreamSynchronize(s));
    if (flops_out) *flops_out = f32;
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

size_t chfsi_defect_split_workspace_bytes(int n, int k) {
  if (n < 1 || k < 1) return 0;
  return chfsi_defect_workspace_bytes(n, k) + split_panel_bytes(n, n) + ALIGN;
}

namespace {

// The defect filter with its first split_steps steps in a split form (mark
// 1: BF16, 2: FP16), the rest FP32 (the workspace of both entry points).
int filter_defect_split_impl(int n, int k, const void* H, int ldh, const void* Q, int ldq,
                             const void* Z, int ldz, const double* mu, const int* degrees,
                             double c, double e, double gamma, int split_steps, char mark,
                             void* Y, int ldy, void* work, size_t work_bytes, void* stream,
                             double* flops_split_out, double* flops_fp32_out) {
  if (n < 1 || k < 1 || k > n || ldh < n || ldq != n || ldz != n || ldy < n || !mu ||
      !degrees || !(e > 0.0) || gamma == c || split_steps < 0)
    return CHFSI_INVALID_ARG;
  if (check_ptr(H) || check_ptr(Q) || check_ptr(Z) || check_ptr(Y) || check_ptr(work))
    return CHFSI_INVALID_ARG;
  for (int j = 0; j < k; ++j) {
    if (degrees[j] < 1 || degrees[j] > CR_ROWS || (j > 0 && degrees[j] < degrees[j - 1]))
      return CHFSI_INVALID_ARG;
  }
  if (work_bytes < chfsi_defect_split_workspace_bytes(n, k)) return CHFSI_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  StepBufs b;
  Carver cv(work);
  carve_step(cv, b, n, k, k, 20);
  void* H32 = cv.take<char>((size_t)n * n * 8);
  void* Hsp = cv.take<char>(split_panel_bytes(n, n));
  CK(matrix_to_fp32(s, n, (const zc*)H, ldh, H32));
  SplitSteps sp;
  if (mark == 1) {
    CK(matrix_to_split(s, n, (const zc*)H, ldh, Hsp));
    sp.Hs = Hsp;
  } else {
    CK(matrix_to_split_h16(s, n, (const zc*)H, ldh, H32, Hsp, b.h16part, &sp.inv_h));
    sp.Hh = Hsp;
  }
  std::vector<int> order(k), m(degrees, degrees + k);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> muv(mu, mu + k);
  const int mmax = m[k - 1];
  std::vector<char> sched(std::max(mmax, 1), 0);
  for (int i = 1; i < mmax; ++i) sched[i] = i <= split_steps ? mark : 0;
  sp.sched = &sched;
  double f32 = 0.0;
  int launches = 0;
  CKS(defect_filter_dev(s, n, k, H32, (const zc*)Q, (const zc*)Z, n, muv, order, m, c, e, gamma,
                        b.T1, b.T2, b, &f32, &launches, &sp));
  CK(copy2d(s, n, k, b.T2, n, (zc*)Y, ldy));
  CK(hipStreamSynchronize(s));
  if (flops_split_out) *flops_split_out = mark == 1 ? sp.flops_bf16 : sp.flops_fp16;
  if (flops_fp32_out) *flops_fp32_out = f32;
  return CHFSI_OK;
}

}  // namespace

int chfsi_filter_defect_split(int n, int k, const void* H, int ldh, const void* Q, int ldq,
                              const void* Z, int ldz, const double* mu, const int* degrees,
                              double c, double e, double gamma, int bf16_steps, void* Y, int ldy,
                              void* work, size_t work_bytes, void* stream,
                              double* flops_bf16_out, double* flops_fp32_out) {
  try {
    return filter_defect_split_impl(n, k, H, ldh, Q, ldq, Z, ldz, mu, degrees, c, e, gamma,
                                    bf16_steps, 1, Y, ldy, work, work_bytes, stream,
                                    flops_bf16_out, flops_fp32_out);
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_filter_defect_fp16(int n, int k, const void* H, int ldh, const void* Q, int ldq,
                             const void* Z, int ldz, const double* mu, const int* degrees,
                             double c, double e, double gamma, int fp16_steps, void* Y, int ldy,
                             void* work, size_t work_bytes, void* stream,
                             double* flops_fp16_out, double* flops_fp32_out) {
  try {
    return filter_defect_split_impl(n, k, H, ldh, Q, ldq, Z, ldz, mu, degrees, c, e, gamma,
                                    fp16_steps, 2, Y, ldy, work, work_bytes, stream,
                                    flops_fp16_out, flops_fp32_out);
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_orthonormalize(int n, int k, void* Y, int ldy, int nl, const void* QL, int ldql,
                         void* work, size_t work_bytes, void* stream, int* shifted_out) {
  try {
    if (n < 1 || k < 1 || ldy < n || nl < 0 || nl + k > n) return CHFSI_INVALID_ARG;
    if (check_ptr(Y) || check_ptr(work)) return CHFSI_INVALID_ARG;
    if (nl > 0 && (check_ptr(QL) || ldql < n)) return CHFSI_INVALID_ARG;
    // the projection coefficients need nl x k elements of T2 (n x k): fine
    if (work_bytes < chfsi_step_workspace_bytes(n, std::max(k, nl))) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    StepBufs b;
    Carver cv(work);
    carve_step(cv, b, n, std::max(k, nl), std::max(k, nl), 20);
    int sh = 0;
    CKS(orthonormalize_dev(s, n, k, (zc*)Y, ldy, nl, (const zc*)QL, ldql, (zc*)Y, ldy, b, &sh));
    CK(hipStreamSynchronize(s));
    if (shifted_out) *shifted_out = sh;
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_rayleigh_ritz(int n, int k, const void* H, int ldh, void* Q, int ldq, void* Z, int ldz,
                        double* mu, double* res, void* work, size_t work_bytes, void* stream) {
  try {
    if (n < 1 || k < 1 || k > n || ldh < n || ldq < n || ldz < n || !mu || !res)
      return CHFSI_INVALID_ARG;
    if (check_ptr(H) || check_ptr(Q) || check_ptr(Z) || check_ptr(work)) return CHFSI_INVALID_ARG;
    if (work_bytes < chfsi_step_workspace_bytes(n, k)) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    StepBufs b;
    Carver cv(work);
    carve_step(cv, b, n, k, k, 20);
    // packed copy of Q in T1, H Q in T2; the rotated basis goes to the
    // caller's Q and Z
    CK(copy2d(s, n, k, (const zc*)Q, ldq, b.T1, n));
    CKS(rayleigh_ritz_dev(s, n, k, (const zc*)H, ldh, b.T1, n, b.T2, n, (zc*)Q, ldq, (zc*)Z, ldz, b,
                          mu, res));
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_lanczos_bounds(int n, const void* H, int ldh, int steps, unsigned long long seed,
                         void* work, size_t work_bytes, void* stream, double* upper,
                         double* theta_min, double* theta_max) {
  try {
    if (n < 1 || ldh < n || steps < 1 || steps > 20 || !upper || !theta_min || !theta_max)
      return CHFSI_INVALID_ARG;
    if (check_ptr(H) || check_ptr(work)) return CHFSI_INVALID_ARG;
    if (work_bytes < chfsi_step_workspace_bytes(n, 1)) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    StepBufs b;
    Carver cv(work);
    carve_step(cv, b, n, 1, 1, 20);
    return lanczos_dev(s, n, (const zc*)H, ldh, steps, seed, b, upper, theta_min, theta_max);
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

size_t chfsi_reduce_workspace_bytes(int n) {
  if (n < 1) return 0;
  Carver c(nullptr);
  c.take<zc>((size_t)n * n);
  c.take<zc>((size_t)n * n);
  c.take<zc>((size_t)n * n);
  c.take<zc>((size_t)((n + NB - 1) / NB) * NB * NB);
  c.take<int>(8);
  return c.off + ALIGN;
}

int chfsi_reduce_standard(int n, const void* A, int lda, const void* B, int ldb, void* H, int ldh,
                          void* L, int ldl, void* work, size_t work_bytes, void* stream) {
  try {
    if (n < 1 || lda < n || ldb < n || ldh < n || ldl < n) return CHFSI_INVALID_ARG;
    if (check_ptr(A) || check_ptr(B) || check_ptr(H) || check_ptr(L) || check_ptr(work))
      return CHFSI_INVALID_ARG;
    if (work_bytes < chfsi_reduce_workspace_bytes(n)) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    Carver cv(work);
    zc* Linv = cv.take<zc>((size_t)n * n);
    zc* W = cv.take<zc>((size_t)n * n);
    zc* Hp = cv.take<zc>((size_t)n * n);
    zc* invd = cv.take<zc>((size_t)((n + NB - 1) / NB) * NB * NB);
    int* dinfo = cv.take<int>(8);
    zc* Lm = (zc*)L;
    CK(copy2d(s, n, n, (const zc*)B, ldb, Lm, ldl));
    CK(hipMemsetAsync(dinfo, 0, sizeof(int), s));
    CKS(potrf_blocked(s, n, Lm, ldl, invd, dinfo, 0.0));
    int pinfo = 0;
    CKS(read_info(s, dinfo, &pinfo));
    if (pinfo != 0) return CHFSI_NOT_HPD;
    CK(zero_upper(s, n, Lm, ldl));
    CK(set_identity(s, n, Linv, n));
    CKS(trsm_left_lower(s, n, n, Lm, ldl, invd, Linv, n, true));
    CKS(reduce_with_inverse(s, n, (const zc*)A, lda, Linv, W, Hp, n));
    CK(copy2d(s, n, n, Hp, n, (zc*)H, ldh));
    CK(hipStreamSynchronize(s));
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_degrees(int k, const double* mu, const double* res, int n_wanted, double alpha,
                  double beta, double tol_abs, int deg_max, int* deg) {
  if (k < 1 || !mu || !res || !deg || !(beta > alpha) || !(tol_abs > 0.0) || deg_max < 1)
    return CHFSI_INVALID_ARG;
  return degrees_host(k, mu, res, n_wanted, alpha, beta, tol_abs, deg_max, deg);
}

int chfsi_split_schedule(int n_wanted, int ka, const double* mu, const double* res,
                         const int* deg, double c, double e, double tol, double norm_h, int form,
                         signed char* steps) {
  if (ka < 1 || !mu || !res || !deg || !steps || (form != 1 && form != 2) || !(e > 0.0) ||
      !(tol > 0.0) || !(norm_h > 0.0))
    return CHFSI_INVALID_ARG;
  for (int j = 0; j < ka; ++j)
    if (deg[j] < 1) return CHFSI_INVALID_ARG;
  const std::vector<char> sched = split_step_schedule(
      n_wanted, std::vector<double>(mu, mu + ka), std::vector<double>(res, res + ka),
      std::vector<int>(deg, deg + ka), c, e, tol, norm_h,
      form == 2 ? FP16_SPLIT_EPS : BF16_SPLIT_EPS, (char)form);
  for (size_t i = 0; i < sched.size(); ++i) steps[i] = (signed char)sched[i];
  return CHFSI_OK;
}

int chfsi_degree_features(double mu, double res, double gap, double alpha, double beta,
                          double gamma, double norm_h, double tol_abs, int loop, double* f) {
  if (!f || !(beta > alpha) || !(tol_abs > 0.0) || !(norm_h > 0.0)) return CHFSI_INVALID_ARG;
  return degree_features(mu, res, gap, alpha, beta, gamma, norm_h, tol_abs, loop, f, nullptr)
             ? CHFSI_OK
             : CHFSI_INVALID_ARG;
}

int chfsi_degrees_sequence(int k, const double* mu, const double* res, const double* speed,
                           int n_wanted, double alpha, double beta, double tol_abs, int deg_max,
                           int* deg, int* src) {
  if (k < 1 || !mu || !res || !deg || !(beta > alpha) || !(tol_abs > 0.0) || deg_max < 1 ||
      n_wanted < 0)
    return CHFSI_INVALID_ARG;
  std::vector<int> sv(k);
  CKS(sequence_degrees(k, mu, res, speed, n_wanted, alpha, beta, tol_abs, deg_max, deg,
                       sv.data()));
  if (src) std::copy(sv.begin(), sv.end(), src);
  return CHFSI_OK;
}

size_t chfsi_mlp_workspace_bytes(int n) {
  if (n < 1) n = 1;
  // parameters, Adam moments and gradient, inputs/outputs for inference,
  // and the gradient scratch
  const size_t floats =
      3 * (size_t)MLP_PARAMS + 4096 + (size_t)n * (MLP_IN + 1) + mlp_grad_work_floats(n);
  return floats * sizeof(float) + 8 * ALIGN;
}

int chfsi_degrees_learned(int k, const double* mu, const double* res, int n_wanted, double alpha,
                          double beta, double gamma, double norm_h, double tol_abs, int loop,
                          int deg_max, const float* params, void* work, size_t work_bytes,
                          void* stream, int* deg, float* pred, int* src) {
  try {
    if (k < 1 || !mu || !res || !deg || !params || !(beta > alpha) || !(tol_abs > 0.0) ||
        !(norm_h > 0.0) || deg_max < 1 || n_wanted < 0 || check_ptr(work) ||
        work_bytes < chfsi_mlp_workspace_bytes(k))
      return CHFSI_INVALID_ARG;
    for (int i = 0; i < MLP_PARAMS; ++i)
      if (!std::isfinite(params[i])) return CHFSI_NONFINITE;
    hipStream_t s = as_stream(stream);
    Carver cv(work);
    float* p = cv.take<float>(MLP_PARAMS);
    float* x = cv.take<float>((size_t)MLP_IN * k);
    float* y = cv.take<float>(k);
    CK(hipMemcpyAsync(p, params, sizeof(float) * MLP_PARAMS, hipMemcpyHostToDevice, s));
    std::vector<int> sv(k);
    CKS(learned_degrees(s, k, mu, res, n_wanted, alpha, beta, gamma, norm_h, tol_abs, loop,
                        deg_max, params, p, x, y, deg, pred, sv.data(), nullptr));
    if (src) std::copy(sv.begin(), sv.end(), src);
    return CHFSI_OK;
  } catch (const std::bad_alloc&) {
    return CHFSI_ALLOC_ERROR;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_mlp_forward(int n, const float* X, const float* params, float* y, void* stream) {
  if (n < 0 || (n > 0 && (!X || !params || !y))) return CHFSI_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  CK(mlp_forward(s, n, X, params, y));
  CK(hipStreamSynchronize(s));
  return CHFSI_OK;
}

int chfsi_mlp_gradient(int n, const float* X, const float* T, const float* params, float* grad,
                       float* loss, void* work, size_t work_bytes, void* stream) {
  if (n < 1 || !X || !T || !params || !grad || !loss || check_ptr(work) ||
      work_bytes < chfsi_mlp_workspace_bytes(n))
    return CHFSI_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  CK(mlp_gradient(s, n, X, T, params, grad, loss, (float*)work));
  CK(hipStreamSynchronize(s));
  return CHFSI_OK;
}

int chfsi_mlp_adam(float* params, const float* grad, float* m, float* v, float lr, int t,
                   void* stream) {
  if (!params || !grad || !m || !v || t < 1 || !(lr > 0.f)) return CHFSI_INVALID_ARG;
  hipStream_t s = as_stream(stream);
  CK(mlp_adam(s, params, grad, m, v, lr, t));
  CK(hipStreamSynchronize(s));
  return CHFSI_OK;
}

int chfsi_mlp_train(int n, const float* X, const float* T, float* params, int steps, float lr,
                    void* work, size_t work_bytes, void* stream, float* loss_out) {
  try {
    if (n < 1 || !X || !T || !params || steps < 0 || !(lr > 0.f) || check_ptr(work) ||
        work_bytes < chfsi_mlp_workspace_bytes(n))
      return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    Carver cv(work);
    float* G = cv.take<float>(MLP_PARAMS);
    float* M = cv.take<float>(MLP_PARAMS);
    float* V = cv.take<float>(MLP_PARAMS);
    float* loss = cv.take<float>(4096);
    float* scratch = cv.take<float>(mlp_grad_work_floats(n));
    CK(hipMemsetAsync(M, 0, sizeof(float) * MLP_PARAMS, s));
    CK(hipMemsetAsync(V, 0, sizeof(float) * MLP_PARAMS, s));
    // the losses of up to LB steps stay on the device between copies
    constexpr int LB = 4096;
    std::vector<float> hl(steps);
    int done = 0;
    for (int t = 1; t <= steps; ++t) {
      CK(mlp_gradient(s, n, X, T, params, G, loss + (t - 1) % LB, scratch));
      CK(mlp_adam(s, params, G, M, V, lr, t));
      if (loss_out && (t % LB == 0 || t == steps)) {
        CK(hipMemcpyAsync(hl.data() + done, loss, sizeof(float) * (t - done), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        done = t;
      }
    }
    CK(hipStreamSynchronize(s));
    if (loss_out)
      for (int t = 0; t < steps; ++t) loss_out[t] = hl[t] / (float)n;
    return CHFSI_OK;
  } catch (const std::bad_alloc&) {
    return CHFSI_ALLOC_ERROR;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

size_t chfsi_autotune_workspace_bytes(int n_max, int N_max) {
  if (n_max < 1 || N_max < 1) return 0;
  Carver c(nullptr);
  c.take<zc>((size_t)n_max * n_max);
  c.take<zc>((size_t)n_max * N_max);
  c.take<zc>((size_t)n_max * N_max);
  return c.off + ALIGN;
}

int chfsi_autotune_filter(int count, const int* n, const int* N, void* work, size_t work_bytes,
                          void* stream, int* variant, double* tflops) {
  try {
    if (count < 0 || (count > 0 && (!n || !N || !variant)) || check_ptr(work)) return CHFSI_INVALID_ARG;
    int nmax = 1, Nmax = 1;
    for (int i = 0; i < count; ++i) {
      if (n[i] < 1 || N[i] < 1 || N[i] > n[i]) return CHFSI_INVALID_ARG;
      nmax = std::max(nmax, n[i]);
      Nmax = std::max(Nmax, N[i]);
    }
    if (work_bytes < chfsi_autotune_workspace_bytes(nmax, Nmax)) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    Carver cv(work);
    zc* H = cv.take<zc>((size_t)nmax * nmax);
    zc* Y0 = cv.take<zc>((size_t)nmax * Nmax);
    zc* Y1 = cv.take<zc>((size_t)nmax * Nmax);
    CK(fill_counter_random(s, nmax, nmax, H, nmax, 1, 1));
    for (int i = 0; i < count; ++i) {
      CK(fill_counter_random(s, n[i], N[i], Y0, n[i], 2, 1));
      CK(fill_counter_random(s, n[i], N[i], Y1, n[i], 3, 1));
      double tf[FILTER_VARIANTS] = {};
      CK(tune_filter_shape(s, n[i], N[i], H, Y0, Y1, &variant[i], tf));
      if (tflops)
        for (int v = 0; v < FILTER_VARIANTS; ++v) tflops[FILTER_VARIANTS * i + v] = tf[v];
    }
    CK(hipStreamSynchronize(s));
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

int chfsi_autotune_set(int n, int N, int variant) {
  if (n < 1 || N < 1 || variant < 0 || variant >= FILTER_VARIANTS) return CHFSI_INVALID_ARG;
  tune_set(n, N, variant);
  return CHFSI_OK;
}

int chfsi_autotune_reset(void) {
  tune_reset();
  return CHFSI_OK;
}

int chfsi_zgemm(char opa, char opb, int M, int N, int K, const double* alpha, const void* A,
                int lda, const void* B, int ldb, const double* beta, void* C, int ldc, void* work,
                size_t work_bytes, void* stream) {
  try {
    if (M < 0 || N < 0 || K < 0 || !alpha || !beta) return CHFSI_INVALID_ARG;
    const Op oa = (opa == 'N' || opa == 'n') ? OP_N : ((opa == 'C' || opa == 'c') ? OP_C : (Op)-1);
    const Op ob = (opb == 'N' || opb == 'n') ? OP_N : ((opb == 'C' || opb == 'c') ? OP_C : (Op)-1);
    if ((int)oa < 0 || (int)ob < 0) return CHFSI_INVALID_ARG;
    const int arows = oa == OP_N ? M : K, brows = ob == OP_N ? K : N;
    if (lda < std::max(1, arows) || ldb < std::max(1, brows) || ldc < std::max(1, M))
      return CHFSI_INVALID_ARG;
    if (M == 0 || N == 0) return CHFSI_OK;
    if (check_ptr(C) || (K > 0 && (check_ptr(A) || check_ptr(B)))) return CHFSI_INVALID_ARG;
    hipStream_t s = as_stream(stream);
    const size_t need = zgemm_work_elems(M, N, K);
    zc* w = nullptr;
    size_t we = 0;
    if (need > 0 && work && aligned16(work) && work_bytes >= need * sizeof(zc)) {
      w = (zc*)work;
      we = work_bytes / sizeof(zc);
    }
    CK(zgemm(s, oa, ob, M, N, K, zc{alpha[0], alpha[1]}, (const zc*)A, lda, (const zc*)B, ldb,
             zc{beta[0], beta[1]}, (zc*)C, ldc, false, w, we));
    CK(hipStreamSynchronize(s));
    return CHFSI_OK;
  } catch (const std::exception& ex) {
    report_failure(ex.what(), __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  } catch (...) {
    report_failure("unknown exception", __LINE__, -1);
    return CHFSI_DEVICE_ERROR;
  }
}

}  // extern "C"
