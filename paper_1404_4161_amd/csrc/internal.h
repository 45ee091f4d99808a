// Internal declarations shared by the HIP sources of libchfsi.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace chfsi {

typedef double2 zc;   // complex128: x = real, y = imaginary

enum Op { OP_N = 0, OP_C = 1 };

// Epilogues of the complex GEMM.
enum Epi {
  EPI_STORE = 0,     // C = alpha * acc + beta * C
  EPI_CHEB = 1,      // Yout = sa * (acc - shift * Ycur) - sb * Yold  (three-term step)
  EPI_PARTIAL = 2,   // raw partial sums of a split-K launch
  EPI_PARTIAL_CHEB = 3,   // the same for a filter step (a kernel name of its own)
};

struct GemmArgs {
  int M, N, K;
  const zc* A; long lda;
  const zc* B; long ldb;
  zc* C; long ldc;
  zc alpha, beta;
  // Chebyshev epilogue
  const zc* Ycur; long ldyc;
  const zc* Yold; long ldyo;
  double shift, sa, sb;
  // split-K
  int splits;        // number of K chunks (grid dimension)
  int kchunk;        // K elements per chunk (multiple of the K tile)
  zc* part;          // partial buffer: split s, element (i, j) at part[s*M*N + i + j*M]
  // tiling / scheduling
  int tiles_m, tiles_n;
  int lower_only;    // compute only tiles that meet the lower triangle (incl. diagonal)
  int total_tiles;   // tiles per split (after the lower-only mask)
  int rows_desc;     // visit tile rows in descending order (set by the launcher)
  int ktri;          // triangular operands: 0 none, 1 op(A) lower (k < m0 + BM),
                     // 2 op(B) upper (k < n0 + BN), 3 op(A) upper (k >= m0),
                     // 4 op(A) and op(B) lower (n0 <= k < m0 + BM),
                     // 5 op(A) lower, op(B) upper (k < min(m0 + BM, n0 + BN))
};

enum KTri {
  KTRI_NONE = 0,
  KTRI_A_LOWER = 1,
  KTRI_B_UPPER = 2,
  KTRI_A_UPPER = 3,
  KTRI_AB_LOWER = 4,
  KTRI_A_LOWER_B_UPPER = 5
};

// ----- launchers (return hipError_t as int) -------------------------------
// General complex GEMM C = alpha op(A) op(B) + beta C.  work/work_elems is
// scratch for split-K partial sums (may be null: no split-K).
// ktri skips the K range where a triangular operand is zero (the memory
// there must hold zeros or is not read at all).
int zgemm(hipStream_t s, Op opa, Op opb, int M, int N, int K, zc alpha,
          const zc* A, long lda, const zc* B, long ldb, zc beta, zc* C, long ldc,
          bool lower_only, zc* work, size_t work_elems, int ktri = KTRI_NONE);

// Scratch elements zgemm may use for a given shape (0 if no split-K).
size_t zgemm_work_elems(int M, int N, int K);

// One step of the scaled three-term Chebyshev recurrence on columns [0, N):
// Yout = sa * (H Ycur - shift Ycur) - sb * Yold   (Yold read only if sb != 0)
// Yout may alias Yold (in-place update of Y_{i-1} into Y_{i+1}).
// With part != null (part_elems complex elements of scratch) the step may
// split K over several workgroups per tile to fill the resident slots
// evenly; the partial sums are then combined, with the same epilogue, by a
// second kernel.
constexpr int CHEB_MAX_SPLITS = 4;
int cheb_step(hipStream_t s, int n, int N, const zc* H, long ldh,
              const zc* Ycur, long ldyc, const zc* Yold, long ldyo,
              zc* Yout, long ldyout, double shift, double sa, double sb,
              zc* part, size_t part_elems);

// Batched form of cheb_step: the launch arguments of one problem's step
// (no split-K), and the number of workgroups it needs (a multiple of 8).
GemmArgs cheb_group_args(int n, int N, const zc* H, long ldh, const zc* Ycur, long ldyc,
                         const zc* Yold, long ldyo, zc* Yout, long ldyout, double shift, double sa,
                         double sb, int* slots);
// One launch running `count` steps; list (device) holds their arguments and
// slot_begin (device, count + 1 ints, multiples of 8) their workgroup ranges.
// variant: the filter variant (below); the wide variant 2 of single steps
// runs as the default here.
int cheb_step_group(hipStream_t s, const GemmArgs* list, const int* slot_begin, int count,
                    int total_slots, int variant);

// Filter tile autotuner (zgemm.hip).  Variants of the FP64 filter step:
// 0 / 1: 64 x 64 tiles with the 4M complex split, K staged 8 / 16 deep
// (four / two workgroups per CU); 2: 128 x 128 tiles (4M, one workgroup
// per CU, windows of N >= 256); 3 / 4: as 0 / 1 with the 3M split (three
// real products per complex multiply-add; three / two workgroups per CU);
// 5 / 6: operands loaded straight into LDS, 3M with a three-stage ring
// (three workgroups per CU) / 4M with two stages (four per CU).
// filter_variant: the variant for an n x n by n x N step (nearest measured
// shape; DEFAULT_FILTER_VARIANT when none).  tune_filter_shape: times the
// variants of a step on the given buffers (H n x n, Y0 and Y1 n x N, ld n;
// Y1 is overwritten), records the fastest (another than the default only
// when 2 % faster) and returns it
// with the complex-equivalent TFLOP/s of each (tf[2] = 0 for N < 256).
// tune_set / tune_reset edit the table directly.
constexpr int FILTER_VARIANTS = 7;
constexpr int DEFAULT_FILTER_VARIANT = 5;   // with no measurement for a shape
constexpr int variant_cm(int variant) {
  return variant == 3 || variant == 4 || variant == 5 ? 3 : 4;
}
int filter_variant(int n, int N);
// real products per complex multiply-add (3 or 4) of a filter step of n x n
// by n x N
inline int filter_step_cm(int n, int N) { return variant_cm(filter_variant(n, N)); }
int tune_filter_shape(hipStream_t s, int n, int N, const zc* H, zc* Y0, zc* Y1, int* variant,
                      double tf[FILTER_VARIANTS]);
void tune_set(int n, int N, int variant);
void tune_reset();

// ----- small kernels (blas1.hip) -----
int col_norms(hipStream_t s, int n, int k, const zc* X, long ldx, double* out);
int resid_norms(hipStream_t s, int n, int k, const zc* Q, long ldq, const zc* Z, long ldz,
                const double* mu, double* out);
int scale_cols_inv(hipStream_t s, int n, int k, zc* X, long ldx, const double* nrm);
int gather_cols(hipStream_t s, int n, int cnt, const zc* src, long lds, zc* dst, long ldd,
                const int* perm);
int gather_parity(hipStream_t s, int n, int k, const zc* P0, const zc* P1, long ldp,
                  zc* dst, long ldd, const int* deg);
int copy2d(hipStream_t s, int rows, int cols, const zc* src, long lds, zc* dst, long ldd);
int herm_from_lower(hipStream_t s, int k, zc* G, long ldg);
int symmetrize(hipStream_t s, int n, zc* H, long ldh);
// H <- H + H^H in place (exactly Hermitian result).
int add_conj_transpose(hipStream_t s, int n, zc* H, long ldh);
// out[0] = ||G - I||_F (device double), G k x k.
int gram_offnorm(hipStream_t s, int k, const zc* G, long ldg, double* out);
// D = lower triangle of A with the diagonal halved, zero above (D != A).
int lower_half_diag(hipStream_t s, int n, const zc* A, long lda, zc* D, long ldd);
int conj_transpose(hipStream_t s, int n, const zc* src, long lds, zc* dst, long ldd);
int zero_upper(hipStream_t s, int n, zc* L, long ldl);
int set_identity(hipStream_t s, int n, zc* X, long ldx);
int add_diag(hipStream_t s, int n, zc* G, long ldg, double v);
int check_finite(hipStream_t s, int rows, int cols, const zc* X, long ldx, int* flag);
int fill_counter_random(hipStream_t s, int n, int k, zc* X, long ldx,
                        unsigned long long seed, int stream_id);
int fill_zero(hipStream_t s, size_t count, zc* X);
// 64-bit fingerprint of a rows x cols matrix into out[0] (device); part
// holds HASH_PARTS partial sums.
constexpr int HASH_PARTS = 1024;
int matrix_hash(hipStream_t s, int rows, int cols, const zc* X, long ldx,
                unsigned long long* part, unsigned long long* out);

// Cholesky leaf: factor the nb x nb block at G (lower, in place) and write
// inv(L_block) (nb x nb, ld nb) to inv.  info (device) receives the
// 1-based global column of the first pivot <= rel_tol * |original diagonal|
// (or non-positive), with col_offset added.
int potrf_leaf(hipStream_t s, int nb, zc* G, long ldg, zc* inv, int* info, int col_offset,
               double rel_tol);
// X += eps * (SplitMix64 uniform in [-1/2, 1/2]^2) per entry
int add_random(hipStream_t s, int n, int k, zc* X, long ldx, unsigned long long seed,
               int stream_id, double eps);

// Lanczos helpers
// H32 (or null): fp32(H), n x n contiguous, read instead of H (FP64 sums).
int gemv_n(hipStream_t s, int n, const zc* H, long ldh, const zc* x, zc* y, zc* part, int splits,
           const void* H32 = nullptr);
int dots_c(hipStream_t s, int n, int cnt, const zc* V, long ldv, const zc* w, zc* h);
int sub_vh(hipStream_t s, int n, int cnt, const zc* V, long ldv, const zc* h, zc* w);
int lanczos_axpy(hipStream_t s, int n, int j, const zc* V, long ldv, const zc* h,
                 const double* betas, zc* w, double* alphas);
int normalize_into(hipStream_t s, int n, const zc* w, zc* v, double* beta_out);

// ----- mixed-precision (FP32 defect) filter, cfilter32.hip -----
// H32 receives fp32(H) as a packed n x n complex64 matrix.
int matrix_to_fp32(hipStream_t s, int n, const zc* H, long ldh, void* H32);
// Columns j < k in degree order: Qs[:, j] = Q[:, perm[j]], R32[:, j] =
// fp32(Z[:, perm[j]] - mu[perm[j]] Q[:, perm[j]]), E0 = 0, E1 = s1 R32.
// Q, Z, Qs have leading dimension ld; R32, E0, E1 are packed (ld n).
int defect_setup_launch(hipStream_t s, int n, int k, const zc* Q, const zc* Z, long ld,
                        const double* mu, const int* perm, zc* Qs, void* R32, void* E0, void* E1,
                        float s1);
// One defect step on N columns (pointers already offset to the window):
// Eout = sa (H32 Ecur - shift Ecur) + cr[j] R32_j - sb Eold.
int defect_step(hipStream_t s, int n, int N, const void* H32, const void* Ecur, const void* Eold,
                void* Eout, const void* R32, const float* cr, float shift, float sa, float sb,
                void* part, size_t part_elems);
// Y[:, j] = pm[j] Qs[:, j] + E_{deg[j]}[:, j] (E_m in E1 for odd m).
int defect_assemble_launch(hipStream_t s, int n, int k, const zc* Qs, long ld, const void* E0,
                           const void* E1, const int* deg, const double* pm, zc* Y, long ldy);

// Grouped defect steps of several independent problems in one launch (k-point
// batches).  *_fill writes one problem's kernel arguments (arg_bytes of them)
// to host memory `out` and returns its workgroup count (a multiple of 8);
// the caller lays the problems' ranges out in slots (prefix sums, slots[0]
// = 0, slots[count] = total), uploads both, and launches once per step.
// FP32 form (64 x 64 tiles, no split-K):
size_t defect_group_arg_bytes();
int defect_group_fill(int n, int N, const void* H32, const void* Ecur, const void* Eold,
                      void* Eout, const void* R32, const float* cr, float shift, float sa,
                      float sb, void* out);
int defect_group_launch(hipStream_t s, const void* dargs, const int* dslots, int count,
                        int total);

// Sum of split-K partials part[p * M * N + i + j * M] (p < splits) followed
// by the defect step's epilogue (the form of defect_step), into Eout.
int defect_reduce_launch(hipStream_t s, int M, int N, int splits, const void* part,
                         const void* Ecur, const void* Eold, void* Eout, long lde, const void* R,
                         long ldr, const float* cr, float shift, float sa, float sb);

// ----- BF16- and FP16-split defect steps, cfilter16.hip -----
// Split panels: rows of a reduction index padded to split_kp(K) (a multiple
// of 32), 8 bytes per complex value (BF16 hi/lo of the real and imaginary
// parts, grouped by 8 k).
int split_kp(int K);
size_t split_panel_bytes(int rows, int K);
// Hs row m = split(fp32(H[m, :])).
int matrix_to_split(hipStream_t s, int n, const zc* H, long ldh, void* Hs);
// S row j = split(E[:, j]) for j < cols (E complex64, leading dimension lde).
int cols_to_split(hipStream_t s, int K, int cols, const void* E, long lde, void* S);
// The defect step of defect_step with H Ecur from the splits Hs and Es (the
// window's rows of the E_i panel); Es_next (or null) receives the split of
// Eout for a following BF16 step.  No split-K.
int defect_step_split(hipStream_t s, int n, int N, const void* Hs, const void* Es,
                      const void* Ecur, const void* Eold, void* Eout, const void* R32,
                      const float* cr, float shift, float sa, float sb, void* Es_next);
// Grouped BF16- (h16 false) or FP16-split (h16 true) defect steps, 64 x 64
// or (wide) 128 x 128 tiles, no split-K; arguments as defect_step_split /
// defect_step_h16 (Es_next: BF16 only).
// windows of at least this many columns take the 128 x 128 tile
int split_wide_min_cols();
size_t split_group_arg_bytes();
int split_group_fill(bool h16, bool wide, int n, int N, const void* Hs, float inv_h,
                     const void* Es, const float* inv_e, const void* Ecur, const void* Eold,
                     void* Eout, const void* R32, const float* cr, float shift, float sa,
                     float sb, void* Es_next, void* out);
int split_group_launch(hipStream_t s, bool h16, bool wide, const void* dargs, const int* dslots,
                       int count, int total);
// Grouped column splits (cols_to_split / cols_to_split_h16 of several
// problems): one workgroup per column, problem p owning the columns
// [cols[p], cols[p+1]); colsplit_group_fill returns 0.
size_t colsplit_group_arg_bytes();
int colsplit_group_fill(int K, const void* E, long lde, void* S, float* inv, void* out);
int colsplit_group_launch(hipStream_t s, bool h16, const void* dargs, const int* dcols, int count,
                          int total_cols);
// FP16 form (same panel geometry, FP16 words of scaled values).  Hs row m =
// split(2^s fp32(H[m, :])) with one power of two s from the largest
// magnitude of H32 (= fp32(H), n x n contiguous; part: 1024 floats of
// device scratch; synchronises the stream); *inv_out = 2^-s.
int matrix_to_split_h16(hipStream_t s, int n, const zc* H, long ldh, const void* H32,
                        void* Hs, float* part, float* inv_out);
// S row j = split(2^s_j E[:, j]) with s_j from column j's largest magnitude;
// inv[j] = 2^-s_j (device).
int cols_to_split_h16(hipStream_t s, int K, int cols, const void* E, long lde, void* S,
                      float* inv);
// The defect step with H Ecur from the FP16 splits (inv_h, inv_e undo the
// scaling).  Windows narrower than 257 columns split K (up to 8 ways,
// chunks of at least 512) when that fills the GPU better, with partials in
// part (part_elems complex64 values; no split-K when it is too small).
int defect_step_h16(hipStream_t s, int n, int N, const void* Hs, float inv_h, const void* Es,
                    const float* inv_e, const void* Ecur, const void* Eold, void* Eout,
                    const void* R32, const float* cr, float shift, float sa, float sb,
                    void* part, size_t part_elems);

// ----- projected eigenproblem by iterative refinement, eigref.hip -----
struct EigRefineBufs {
  zc* mat;                    // 7 k x k work matrices
  double* lam;                // k
  unsigned long long* stats;  // 4
  int2* pairs;                // pair_cap strongly coupled pairs
  int pair_cap;
  int2* idx;                  // entry_cap cluster-block entries
  zc* val;
  int entry_cap;
  int* perm;                  // k
};
size_t eig_refine_elems(int k);
// Eigenvectors W (k x k, ld ldw, columns ascending) and eigenvalues mu
// (device, k, ascending) of the Hermitian G (ld ldg, read-only) by
// refinement from the identity.  *refined = 0 (and W, mu untouched) when
// G is too far from diagonal or the refinement does not converge: the
// caller then uses a dense eigensolver.  Returns a HIP error code.
int eig_refine(hipStream_t s, int k, const zc* G, long ldg, zc* W, long ldw, double* mu,
               EigRefineBufs& rb, int* refined, int* iterations);

// ----- degree network (mlp.hip) -----
// Parameter blob layout (floats); the same layout is documented in chfsi.h.
constexpr int MLP_IN = 8, MLP_H = 64;
constexpr int MLP_MEAN = 0;
constexpr int MLP_STD = MLP_MEAN + MLP_IN;
constexpr int MLP_W1 = MLP_STD + MLP_IN;          // MLP_H x MLP_IN, row-major
constexpr int MLP_B1 = MLP_W1 + MLP_H * MLP_IN;
constexpr int MLP_W2 = MLP_B1 + MLP_H;            // MLP_H x MLP_H, row-major
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_W3 = MLP_B2 + MLP_H;
constexpr int MLP_B3 = MLP_W3 + MLP_H;
constexpr int MLP_MARGIN = MLP_B3 + 1;
constexpr int MLP_PARAMS = MLP_MARGIN + 1;
// Samples per partial sum of the gradient reduction.
constexpr int MLP_CHUNK = 256;

// Device floats used by mlp_gradient for n samples.
size_t mlp_grad_work_floats(int n);
// y[s] = net(X[s, :]) for n samples (X row-major n x MLP_IN).
int mlp_forward(hipStream_t s, int n, const float* X, const float* prm, float* Y);
// Gradient of (1/n) sum_s (net(X_s) - T_s)^2 with respect to every entry of
// the blob (zero for the non-trained ones) into G; the loss into loss_dev[0].
int mlp_gradient(hipStream_t s, int n, const float* X, const float* T, const float* prm,
                 float* G, float* loss_dev, float* work);
// One Adam step (t >= 1) on the trained entries.
int mlp_adam(hipStream_t s, float* prm, const float* G, float* M, float* V, float lr, int t);

}  // namespace chfsi
