/*
 * chfsi.h -- C ABI of the MI355X (gfx950) Chebyshev Filtered Subspace
 * Iteration library (libchfsi.so).
 *
 * Method: Berljafa, Wortmann, Di Napoli, "An optimized and scalable
 * eigensolver for sequences of eigenvalue problems" -- Alg. 1 (ChFSI) with
 * Alg. 2 (the Chebyshev filter) at its core, Sec. 3.1 and 3.1.1.
 *
 * Conventions shared by every entry point
 *   - Complex matrices are complex128 (two IEEE doubles, real part first),
 *     COLUMN-MAJOR, with a leading dimension ld >= rows.  Passing a
 *     row-major Hermitian matrix instead reads conj(A): same eigenvalues,
 *     conjugated eigenvectors.
 *   - Pointers documented as "device" are HIP device pointers on the
 *     current device; "host" pointers are ordinary host memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device
 *     work is ordered on it.  Every entry point returns after its results
 *     are complete (it synchronises the stream).
 *   - The caller owns every buffer.  The library never frees caller
 *     memory.  Inputs documented as read-only are not modified.
 *   - Scratch memory: `work` is a caller-owned device buffer of at least
 *     the size reported by the matching *_workspace_bytes query.  The
 *     rocSOLVER/rocBLAS handle used for the reduced eigenproblem manages
 *     its own device memory.
 *   - Errors are reported by the returned status; no entry point aborts,
 *     prints or throws.  Calls with distinct workspaces on distinct streams
 *     are independent.
 */
#ifndef CHFSI_H
#define CHFSI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define CHFSI_OK              0  /* success                                              */
#define CHFSI_INVALID_ARG     1  /* bad size, leading dimension, pointer or workspace    */
#define CHFSI_NOT_HPD         2  /* B (or a Gram matrix) is not Hermitian positive def.  */
#define CHFSI_NO_CONVERGENCE  3  /* max_iter reached; outputs hold the best so far       */
#define CHFSI_NONFINITE       4  /* NaN or Inf in an input                               */
#define CHFSI_DEVICE_ERROR    5  /* a HIP / rocSOLVER call failed                        */
#define CHFSI_ALLOC_ERROR     6  /* internal host allocation failed                      */

/* Options of the solver.  Field meanings (paper references in brackets):
 *   tol           residual target: a Ritz pair locks when ||H y - mu y|| <=
 *                 tol * ||H|| with ||H|| estimated by Lanczos [Sec. 3.1.1,
 *                 eq. resl; Sec. 4]; default 1e-10.
 *   deg0          filter degree of the first loop [Alg. 1 input DEG]; 10.
 *   deg_max       degree cap of the optimisation [Sec. 3.1.1]; 40.
 *   max_iter      cap on outer loops (the paper has none); 100.
 *   lanczos_steps steps of the upper-bound estimate [Sec. 3.1]; 20.
 *   alpha_rule    lower end of the damped interval: 0 = largest Ritz value
 *                 of the block, 1 = the (nev+1)-th Ritz value [Sec. 3.1].
 *   degree_mode   0 = per-vector analytic degrees [Sec. 3.1.1], 1 = fixed
 *                 deg0 for every vector and loop, 2 = learned: a network
 *                 predicts how fast each vector converges compared with
 *                 the analytic model and the degree is scaled to match
 *                 (see chfsi_degrees_learned); the analytic degree stays
 *                 the floor of every learned degree and the fallback for
 *                 inputs outside the network's training range.
 *                 3 = sequence-calibrated (Multiple Optimization): the
 *                 rule's rate of each vector is divided by its speed
 *                 measured earlier in the sequence (seq_rates), m_j =
 *                 max(rule_j, ceil(m_a,j * f / speed_j)) with f = 1.25 in a
 *                 loop that can finish every wanted vector and 1 otherwise;
 *                 vectors without a measured speed take the rule.
 *   reuse_b_factor  1 (default): keep the Cholesky factor of B and its
 *                 inverse in the workspace and reuse them on the next call
 *                 with the same workspace when B is bitwise unchanged (a
 *                 64-bit fingerprint of B is checked on every call); 0:
 *                 always factor B.  For sequences whose B is fixed the
 *                 factor is then computed once per sequence.
 *   precision     0 (default): FP64 filter.  1: mixed -- when the current
 *                 Ritz pairs' residuals are small enough that FP32 rounding
 *                 cannot limit the filter (checked per outer loop: the
 *                 floor eps_fp32 * residual must be 100x below the
 *                 residual the filter aims at), the
 *                 filter runs in complex FP32 on the defect
 *                 E = p(Ht) Q - Q p(mu_t) of the Ritz vectors Q; QR,
 *                 Rayleigh-Ritz, residuals and locking stay FP64.  The
 *                 Lanczos mat-vecs of precisions 1-3 read fp32(H) (FP64
 *                 sums), and the upper bound is raised by 2^-24 sqrt(n)
 *                 max(|bound|, |theta_min|), a bound of ||H - fp32(H)||_2.
 *                 2: as 1, and inside such a filter each recurrence step
 *                 whose rounding is damped enough by the steps after it
 *                 runs its product in BF16 (two-term BF16 splits of H and
 *                 E, three v_mfma_f32_16x16x32_bf16 products, FP32
 *                 accumulation; error about 3 * 2^-16 of the defect): per
 *                 step i and wanted vector j with m_j > i, the floor
 *                 3 * 2^-16 * rel_j * |rho_j|^-(m_j - i - 1) must be 10x
 *                 below max(tol, rel_j |rho_j|^-m_j), rel_j = residual /
 *                 norm_h (eq. resl).  Needs n^2 * 8 more bytes of work.
 *                 3: as 1, with the FP16-split product instead: two-term
 *                 FP16 splits of 2^s H (one power of two for H) and of
 *                 2^s_j E_j (one per column of E, both from the largest
 *                 magnitude, into [2^14, 2^15)), three
 *                 v_mfma_f32_16x16x32_f16 products, FP32 accumulation,
 *                 the scaling undone in the epilogue; error about
 *                 3 * 2^-22 of the defect, so the rule of precision 2
 *                 with 3 * 2^-22 in place of 3 * 2^-16 admits nearly
 *                 every step of an FP32 defect filter.  Needs n^2 * 8
 *                 more bytes of work.
 *   seed          seed of the SplitMix64 counter-based generator used for
 *                 the Lanczos start vector and a random start block.
 *   degree_jitter 0 (default), or s > 0: every wanted vector's degree m is
 *                 replaced by round(m * exp(s * u)), u uniform in [-1, 1]
 *                 from the counter generator (stream 3, counter = loop *
 *                 k + column), clamped to [1, deg_max].  Used to collect
 *                 convergence logs over a range of degrees.
 *   first_rule    0 (default): the first loop uses deg0 [Alg. 1].  1: in a
 *                 warm start with Lambda0, the residuals of X0 are computed
 *                 first (one product H X0) and the first loop's degrees
 *                 come from the degree rule in force (Sec. 3.1.1 applies
 *                 once the residuals are known).  The mixed path computes
 *                 those residuals anyway.
 *   log, log_capacity  HOST buffer of log_capacity records of
 *                 CHFSI_LOG_FIELDS doubles, or NULL: one record per
 *                 filtered wanted vector and loop (layout below).  The
 *                 number written is info->log_records.
 *   mlp           HOST, CHFSI_MLP_PARAMS floats: the degree network used by
 *                 degree_mode 2 (required then; read once per call).
 *   seq_rates     HOST, k doubles in/out, or NULL (required by degree_mode
 *                 3): per eigenvector (in the order of X0 / Lambda), its
 *                 convergence speed relative to the analytic model of
 *                 eq. (resl), ln(Res_before / Res_after) / (m ln|rho|),
 *                 last measured (NaN when unknown; an FP32 loop counts only
 *                 where Res_after > 1e3 eps32 Res_before).  On
 *                 input (with X0) the speeds of the previous problem; on
 *                 output this problem's, in the order of Lambda.  Passing
 *                 the array along a sequence carries the calibration.
 *   rr_refine     1 (default): the k x k eigenproblem of Rayleigh-Ritz is
 *                 solved by iterative refinement from the identity (the
 *                 projected matrix is nearly diagonal once the block is
 *                 close to eigenvectors; close Ritz values are rotated as
 *                 clusters), with rocSOLVER zheevd as the fallback when it
 *                 is far from diagonal; 0: zheevd always.  Both give the
 *                 eigenpairs to rounding (see chfsi_eigh_projected). */
typedef struct chfsi_opts {
  double tol;
  int deg0;
  int deg_max;
  int max_iter;
  int lanczos_steps;
  int alpha_rule;
  int degree_mode;
  int reuse_b_factor;
  int precision;
  unsigned long long seed;
  double degree_jitter;
  int first_rule;
  int log_capacity;
  double* log;
  const float* mlp;
  double* seq_rates;
  int rr_refine;
} chfsi_opts;

/* Per-solve statistics (all optional to read).
 *   step_seconds: device time per phase, indices
 *     0 reduction, 1 lanczos, 2 filter, 3 orthonormalisation,
 *     4 rayleigh-ritz, 5 residuals, 6 locking/permutations, 7 back-transform */
typedef struct chfsi_info {
  int iters;               /* outer loops                                        */
  int converged;           /* locked wanted pairs (== nev on success)            */
  int filter_launches;     /* filter-step kernel launches                        */
  int cholqr_shifted;      /* orthonormalisations that needed the shifted pass   */
  int b_factor_reused;     /* 1 when B's factor came from the workspace          */
  int filter_iters_fp32;   /* outer loops whose filter ran in FP32 defect form   */
  long long matvecs;       /* column mat-vecs with H (filter + RR + Lanczos)     */
  long long filter_matvecs;/* sum over loops of the degrees of the filtered cols */
  double filter_flops;     /* 8 n^2 per column mat-vec of the filter             */
  double filter_seconds;   /* device time of the filter-step launches            */
  double total_seconds;    /* host wall time of the call                         */
  double max_resid;        /* max ||H y - lambda y|| / ||H|| over the nev pairs  */
  double beta;             /* Lanczos upper bound of the spectrum of H           */
  double norm_h;           /* max(|beta|, |theta_min|), the scale of `tol`       */
  double step_seconds[8];
  double filter_flops_fp32;   /* FP32 GEMM flops executed by defect filters      */
  double filter_seconds_fp32; /* device time of the defect filters               */
  int log_records;         /* records written to opts->log                       */
  int learned_cols;        /* wanted column degrees taken from the network       */
  int fallback_cols;       /* wanted column degrees that fell back to the rule   */
  int learned_raised;      /* network degrees above the rule's degree            */
  int filter_steps_bf16;   /* defect-filter steps run with BF16-split products   */
  double filter_flops_bf16;/* 8 n^2 per column of those steps                    */
  int rr_refined;          /* Rayleigh-Ritz eigenproblems solved by refinement   */
  int rr_dense;            /* ... and by the dense eigensolver (zheevd)          */
  int filter_steps_fp16;   /* defect-filter steps run with FP16-split products   */
  double filter_flops_fp16;/* 8 n^2 per column of those steps                    */
  double filter_flops_fp64_mfma; /* real flops the MFMAs of the FP64 filter steps
                            executed: 8 n^2 per column mat-vec with the 4M
                            complex split, 6 n^2 with 3M (filter_flops counts
                            8 n^2 for both)                                   */
} chfsi_info;

/* Convergence log record (CHFSI_LOG_FIELDS doubles), one per wanted vector
 * j of the active block filtered in a loop:
 *   0 loop (1-based)       1 j (position in the active block, ascending mu)
 *   2 wanted columns left  3 active block size
 *   4 mu_j before          5 res_j before (||H q - mu q||)
 *   6 gap_j = distance to the nearest other Ritz value of the block
 *   7 alpha  8 beta  9 gamma   10 norm_h   11 tol * norm_h
 *   12 degree used         13 degree of the analytic rule
 *   14 res at position j after the loop's Rayleigh-Ritz
 *   15 flags: 1 FP32 defect filter, 2 degree from the network,
 *             4 network fallback to the rule, 8 jittered, 16 capped at
 *             the reach of one FP32 loop
 *   16..23 the network's input features (chfsi_degree_features). */
#define CHFSI_LOG_FIELDS 24

/* Degree network: an 8 -> 64 -> 64 -> 1 perceptron with tanh activations
 * in FP32.  Parameter blob (CHFSI_MLP_PARAMS floats):
 *   [0, 8) feature means, [8, 16) feature scales (inputs are standardised
 *   as (x - mean) / scale), [16, 528) W1 (64 x 8 row-major), [528, 592) b1,
 *   [592, 4688) W2 (64 x 64 row-major), [4688, 4752) b2, [4752, 4816) w3,
 *   [4816] b3, [4817] margin.
 * Output: y ~ ln(observed log-reduction of the residual per degree /
 * ln|rho_j|), the log of the vector's convergence speed relative to the
 * analytic model of Sec. 3.1.1 (eq. resl). */
#define CHFSI_MLP_FEATURES 8
#define CHFSI_MLP_PARAMS 4818

/* Fill *o with the defaults listed above.  Returns CHFSI_OK, or
 * CHFSI_INVALID_ARG for o == NULL. */
int chfsi_default_opts(chfsi_opts* o);

/* Bytes of device workspace chfsi_solve needs for this problem
 * (generalized != 0 when B is given).  opts may be NULL.  For a generalized
 * problem the workspace starts with B's factor (see reuse_b_factor); keep
 * passing the same workspace along a sequence to reuse it. */
size_t chfsi_workspace_bytes(int n, int nev, int nex, int generalized, const chfsi_opts* opts);

/* Solve the nev lowest eigenpairs of A x = lambda B x (B == NULL: B = I)
 * with ChFSI, Alg. 1 of the paper:
 *   reduction to H = L^{-1} A L^{-H}, B = L L^H [Sec. 3.1], Lanczos bound,
 *   then loops of {Chebyshev filter (Alg. 2, per-vector degrees, columns
 *   sorted by degree [Sec. 3.2]), orthonormalisation (CholeskyQR2 against
 *   the locked vectors), Rayleigh-Ritz, residuals, locking, degree
 *   optimisation} until nev pairs have converged.
 * Arguments
 *   n, nev, nex  problem size, wanted pairs, extra (guard) vectors; the
 *                block has k = nev + nex columns; 1 <= nev, 1 <= nex,
 *                k <= n.
 *   A, lda       device, n x n Hermitian, read-only.  A standard problem
 *                uses A as given (both triangles); the reduction of a
 *                generalized problem reads the lower triangle only.
 *   B, ldb       device, n x n Hermitian positive definite, read-only, or
 *                NULL for a standard problem.
 *   tol          residual target (overrides opts->tol); > 0.
 *   X0, ldx0     device, n x k start block (e.g. the previous problem's
 *                Ritz vectors, in the coordinates of A, B), read-only, or
 *                NULL for a seeded random block.
 *   Lambda0      HOST, k doubles ascending, or NULL: the Ritz values that go
 *                with X0 (the previous problem's eigenvalues, the inputs
 *                lambda_1 and lambda_{nev+1} of Alg. 1).  When given, the
 *                first filter takes its interval from them and filters X0
 *                directly; when NULL, one QR + Rayleigh-Ritz of the start
 *                block supplies them.  Requires X0.
 *   Lambda       HOST, k doubles: all k Ritz values, ascending; the first
 *                nev are the converged eigenvalues.
 *   X, ldx       device, n x k output Ritz vectors (X^H B X = I), in the
 *                order of Lambda.  May alias X0 (same pointer and ld).
 *   work, work_bytes  device workspace, >= chfsi_workspace_bytes(...).
 *   opts         NULL for defaults.
 *   stream       hipStream_t or NULL.
 *   info         NULL or statistics out.
 * Returns a status code; on CHFSI_NO_CONVERGENCE Lambda and X hold the
 * current pairs. */
int chfsi_solve(int n, int nev, int nex,
                const void* A, int lda,
                const void* B, int ldb,
                double tol,
                const void* X0, int ldx0,
                const double* Lambda0,
                double* Lambda,
                void* X, int ldx,
                void* work, size_t work_bytes,
                const chfsi_opts* opts,
                void* stream,
                chfsi_info* info);

/* Batched solve of independent problems (e.g. the k-points of one
 * self-consistency step, Sec. 1 / Sec. 4: every k-point gives its own
 * sequence): `count` problems, each with the arguments of chfsi_solve given
 * by index q (arrays of count entries), run their outer loops in lockstep.
 * The problems form two groups that alternate on `stream`; every loop's
 * filters of a group share grouped launches on `stream`: the FP64 filters
 * one launch per recurrence step (a grouped MFMA kernel over all its
 * problems' tiles), the mixed-precision defect filters one launch per
 * recurrence step and step form (with one grouped column-split launch
 * before a split step); the per-problem phases (reduction, Lanczos, QR,
 * Rayleigh-Ritz, the defect filters' set-up and assembly) run on up to 8
 * internal streams, each driven by a host thread of
 * the library with its own rocSOLVER handle, so that different problems'
 * phases overlap.  Event dependencies order everything after the work
 * already queued on `stream`, and the call returns when all is done.  Each
 * problem runs the same algorithm as chfsi_solve with the same arguments;
 * only the summation order of the filter products may differ (the grouped
 * launch does not split K).
 *   B, X0, Lambda0 may be NULL (no problem has one) or hold NULL entries;
 *   ldb / ldx0 are then read only for the non-NULL entries.
 *   work[q], work_bytes[q]  per-problem workspaces (chfsi_workspace_bytes),
 *               pairwise distinct; B's factor is reused per workspace.
 *   batch_work  device, >= chfsi_batch_workspace_bytes(count, opts): the
 *               launch arguments of the grouped filters.
 *   opts        shared by all problems; log_capacity must be 0 and
 *               seq_rates NULL (degree_mode 3 is not available here).
 *   flags       bit 0: capture each loop's grouped filter launches as one
 *               HIP graph and launch it (needs a non-NULL stream).
 *               bit 1: serial -- one internal stream driven by the calling
 *               thread (no worker threads; the per-problem phases of
 *               different problems do not overlap).
 *               bit 2: run each problem's mixed-precision defect filter on
 *               its own stream, one problem at a time (by default the
 *               defect filters of a group share, per recurrence step, one
 *               launch per step form: FP16-split, BF16-split or FP32).
 *   info        NULL or count statistics records.
 *   status      HOST, count ints out: each problem's status.
 * Returns CHFSI_OK when every problem converged, else the first error
 * (or CHFSI_NO_CONVERGENCE). */
size_t chfsi_batch_workspace_bytes(int count, const chfsi_opts* opts);
int chfsi_solve_batch(int count, const int* n, const int* nev, const int* nex,
                      const void* const* A, const int* lda, const void* const* B, const int* ldb,
                      double tol, const void* const* X0, const int* ldx0,
                      const double* const* Lambda0, double* const* Lambda, void* const* X,
                      const int* ldx, void* const* work, const size_t* work_bytes,
                      void* batch_work, size_t batch_work_bytes, const chfsi_opts* opts, int flags,
                      void* stream, chfsi_info* info, int* status);

/* Static, human-readable text for a status code. */
const char* chfsi_status_string(int status);

/* ------------------------------------------------------------------------
 * Step-level entry points (each one row of the hot path), device buffers.
 * ---------------------------------------------------------------------- */

/* Workspace bytes for the step-level calls below on an n x k block
 * (covers chfsi_filter, chfsi_orthonormalize, chfsi_rayleigh_ritz,
 * chfsi_lanczos_bounds, chfsi_zgemm split-K). */
size_t chfsi_step_workspace_bytes(int n, int k);

/* Chebyshev filter, Alg. 2: Y <- p_{m_j}(Ht) Y_j for every column j, with
 * Ht = (H - cI)/e, p_m(t) = C_m(t) / C_m((gamma - c)/e) and the scaled
 * three-term recurrence of eq. (3term).
 *   H, ldh      device n x n Hermitian, read-only.
 *   Y, ldy      device n x k, in/out.
 *   degrees     HOST, k ints >= 1, ascending (columns sorted by degree as in
 *               Sec. 3.2); CHFSI_INVALID_ARG otherwise.
 *   c, e, gamma centre and half-width of the damped interval and the
 *               estimate of lambda_1 (e > 0, gamma != c).
 *   flops_out   NULL or the algorithmic flops (8 n^2 per column mat-vec).
 *   launches_out NULL or number of filter-step kernel launches. */
int chfsi_filter(int n, int k, const void* H, int ldh, void* Y, int ldy,
                 const int* degrees, double c, double e, double gamma,
                 void* work, size_t work_bytes, void* stream,
                 double* flops_out, int* launches_out);

/* chfsi_filter without a workspace argument and without any device
 * allocation, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same operation, arguments, degree order and result as chfsi_filter; the
 * library keeps the filter's ping-pong blocks, the degrees and the split-K
 * partial sums in a static device array of CHFSI_NOALLOC_SCRATCH_BYTES per
 * GPU (held by each GPU the library runs on until the process ends).
 *   Limit: chfsi_filter_noalloc_need_bytes(n, k) = 2 n k 16 bytes plus the
 *   degrees, rounded to 256-byte blocks, must not exceed
 *   CHFSI_NOALLOC_SCRATCH_BYTES (n k up to about 2.09e6), else
 *   CHFSI_INVALID_ARG before any device work.  The split-K partial sums use
 *   what is left of the array (fewer splits than chfsi_filter when little is
 *   left: the same result up to the order of the sums).
 *   Every call on one GPU shares that GPU's array and leaves its contents
 *   behind; calls that overlap on one GPU (several host threads or streams)
 *   race and must be serialised by the caller. */
#define CHFSI_NOALLOC_SCRATCH_BYTES (64u << 20)
size_t chfsi_filter_noalloc_need_bytes(int n, int k);
int chfsi_filter_noalloc(int n, int k, const void* H, int ldh, void* Y, int ldy,
                         const int* degrees, double c, double e, double gamma, void* stream,
                         double* flops_out, int* launches_out);

/* Mixed-precision form of chfsi_filter (same result, FP32 GEMMs): filters
 * the Ritz vectors Q (n x k, ascending degrees as in chfsi_filter) given
 * Z = H Q and the Ritz values mu (HOST, k doubles), by running the
 * recurrence on the defect p_i(Ht) Q - Q diag(p_i((mu - c)/e)) in complex
 * FP32 (v_mfma_f32_16x16x4_f32).  The rounding error scales with the
 * residuals ||Z_j - mu_j Q_j|| instead of ||Q_j||.  Q and Z must be packed
 * (ldq = ldz = n); degrees <= 256; work >= chfsi_defect_workspace_bytes.
 *   Y, ldy    device n x k out (must not overlap Q or Z).
 *   flops_out NULL or the executed FP32 GEMM flops. */
size_t chfsi_defect_workspace_bytes(int n, int k);
int chfsi_filter_defect(int n, int k, const void* H, int ldh, const void* Q, int ldq,
                        const void* Z, int ldz, const double* mu, const int* degrees, double c,
                        double e, double gamma, void* Y, int ldy, void* work, size_t work_bytes,
                        void* stream, double* flops_out);

/* chfsi_filter_defect with its first bf16_steps recurrence steps (E_i ->
 * E_{i+1}, i = 1 .. bf16_steps) run in BF16-split form (precision 2 of
 * chfsi_opts: H and E_i each split into two BF16 words, three
 * v_mfma_f32_16x16x32_bf16 products per real product, FP32 accumulation,
 * E kept in FP32 between steps); the later steps run in FP32.  bf16_steps
 * = 0 gives chfsi_filter_defect's result.  Same arguments and limits as
 * chfsi_filter_defect; work >= chfsi_defect_split_workspace_bytes(n, k).
 *   flops_bf16_out, flops_fp32_out  NULL or the algorithmic flops (8 n^2
 *               per column and step) of the BF16 and of the FP32 steps. */
size_t chfsi_defect_split_workspace_bytes(int n, int k);
int chfsi_filter_defect_split(int n, int k, const void* H, int ldh, const void* Q, int ldq,
                              const void* Z, int ldz, const double* mu, const int* degrees,
                              double c, double e, double gamma, int bf16_steps, void* Y, int ldy,
                              void* work, size_t work_bytes, void* stream,
                              double* flops_bf16_out, double* flops_fp32_out);

/* chfsi_filter_defect_split with FP16-split steps (precision 3 of
 * chfsi_opts) in place of the BF16 ones: the first fp16_steps steps take
 * two-term FP16 splits of 2^s H and of 2^s_j E_i[:, j] (powers of two from
 * the largest magnitudes; one reduction over H, whose result is read on the
 * host, so the call synchronises the stream once more), three
 * v_mfma_f32_16x16x32_f16 products per real product and FP32
 * accumulation; the later steps run in FP32.  Same arguments, limits and
 * workspace as chfsi_filter_defect_split.
 *   flops_fp16_out, flops_fp32_out  NULL or the algorithmic flops of the
 *               FP16 and of the FP32 steps. */
int chfsi_filter_defect_fp16(int n, int k, const void* H, int ldh, const void* Q, int ldq,
                             const void* Z, int ldz, const double* mu, const int* degrees,
                             double c, double e, double gamma, int fp16_steps, void* Y, int ldy,
                             void* work, size_t work_bytes, void* stream,
                             double* flops_fp16_out, double* flops_fp32_out);

/* The k x k Hermitian eigenproblem of Rayleigh-Ritz, G W = W diag(mu)
 * with mu ascending and W unitary (Alg. 1, RAYLEIGH-RITZ).
 *   mode 0: rocSOLVER zheevd.  1: iterative refinement from W = I (each
 *   step: S = W^H G W, R = I - W^H W, lam_i = s_ii / (1 - r_ii), W <- W (I
 *   + F) with f_ii = r_ii / 2, f_ij = (s_ij + lam_j r_ij) / (lam_j - lam_i)
 *   and f_ji = r_ji - conj(f_ij) for i < j when the coupling is below 0.1
 *   of the gap; pairs coupled more strongly are grouped into clusters whose
 *   blocks are diagonalised by Jacobi rotations), falling back to zheevd
 *   when G is far from diagonal (clusters over 32 columns or over half the
 *   block, or no convergence in 10 steps).  2: refinement only
 *   (CHFSI_NO_CONVERGENCE instead of the fallback).
 *   G, ldg      device k x k Hermitian (read-only; both triangles used).
 *   W, ldw      device k x k out.   mu  HOST, k doubles out.
 *   refined_out NULL or 1 when the refinement gave the result.
 *   work        device, >= chfsi_eigh_workspace_bytes(k). */
size_t chfsi_eigh_workspace_bytes(int k);
int chfsi_eigh_projected(int k, const void* G, int ldg, void* W, int ldw, double* mu, int mode,
                         void* work, size_t work_bytes, void* stream, int* refined_out);

/* Orthonormalise the n x k block Y against the n x nl locked block QL
 * (two projection passes, QL^H QL = I assumed) and then by CholeskyQR2,
 * falling back to a shifted CholeskyQR3 when the Gram matrix is not
 * numerically positive definite.  Implements the QR step of Alg. 1.
 *   Y, ldy     device, in/out: on return an orthonormal basis of the
 *              projected span (same column order).
 *   QL, ldql   device n x nl, read-only (NULL when nl == 0).
 *   shifted_out NULL or 1 when the shifted pass was used. */
int chfsi_orthonormalize(int n, int k, void* Y, int ldy, int nl, const void* QL, int ldql,
                         void* work, size_t work_bytes, void* stream, int* shifted_out);

/* Rayleigh-Ritz (Alg. 1) plus residual norms (eq. resl):
 *   Z = H Q, G = Q^H Z, G W = W diag(mu) ascending, Q <- Q W, Z <- Z W,
 *   res_j = ||Z_j - mu_j Q_j||_2.
 *   Q, ldq   device n x k orthonormal, in/out.
 *   Z, ldz   device n x k out (H times the new Q).
 *   mu, res  HOST, k doubles out each. */
int chfsi_rayleigh_ritz(int n, int k, const void* H, int ldh, void* Q, int ldq,
                        void* Z, int ldz, double* mu, double* res,
                        void* work, size_t work_bytes, void* stream);

/* Lanczos estimate of the spectrum of H (Sec. 3.1): `steps` steps with full
 * reorthogonalisation from the SplitMix64 start vector of `seed` (stream
 * 0).  Outputs (HOST): upper = theta_max + |b_steps| (the bound used for
 * beta), theta_min, theta_max. */
int chfsi_lanczos_bounds(int n, const void* H, int ldh, int steps, unsigned long long seed,
                         void* work, size_t work_bytes, void* stream,
                         double* upper, double* theta_min, double* theta_max);

/* Reduction of A x = lambda B x to standard form (Sec. 3.1):
 * B = L L^H (Cholesky), H = L^{-1} A L^{-H}, formed as M + M^H with M =
 * (L^{-1} T) L^{-H}, T the lower triangle of A with its diagonal halved
 * (exactly Hermitian; only the lower triangles of A and B are read).
 *   H, ldh  device n x n out.    L, ldl  device n x n out (lower; the
 *   strictly upper part is set to zero).  A and B are read-only.
 * Returns CHFSI_NOT_HPD when the Cholesky factorisation breaks down. */
size_t chfsi_reduce_workspace_bytes(int n);
int chfsi_reduce_standard(int n, const void* A, int lda, const void* B, int ldb,
                          void* H, int ldh, void* L, int ldl,
                          void* work, size_t work_bytes, void* stream);

/* Per-vector filter degrees of Single Optimization (Sec. 3.1.1), host only:
 * m_j = ceil(ln(res_j / tol_abs) / ln|rho_j|) clamped to [1, deg_max], with
 * |rho_j| from t_j = (mu_j - c)/e, c = (alpha+beta)/2, e = (beta-alpha)/2.
 * Vectors j >= n_wanted (guards) and vectors with |t_j| <= 1 get the largest
 * degree among the others (deg_max if there is none).
 *   mu, res  HOST, k doubles.   deg  HOST, k ints out. */
int chfsi_degrees(int k, const double* mu, const double* res, int n_wanted,
                  double alpha, double beta, double tol_abs, int deg_max, int* deg);

/* Which recurrence steps of an FP32 defect filter the solver runs in a
 * split form (host only; precision 2: form 1, BF16 words, eps = 3 * 2^-16;
 * precision 3: form 2, FP16 words of scaled operands, eps = 3 * 2^-22).
 * Step i (E_i -> E_{i+1}, 1 <= i < max deg) is split when for every wanted
 * vector j < n_wanted with deg_j > i:
 *   10 eps rel_j |rho_j|^-(deg_j - i - 1) <= max(tol, rel_j |rho_j|^-deg_j),
 * rel_j = res_j / norm_h, |rho_j| from t_j = (mu_j - c)/e (1 for |t_j| <= 1).
 *   mu, res  HOST, ka doubles.   deg  HOST, ka ints >= 1.
 *   steps    HOST, max(deg) signed chars out: 0 (FP32) or form; steps[0] = 0.
 * Returns CHFSI_INVALID_ARG for ka < 1, form not 1 or 2, e <= 0, tol <= 0,
 * norm_h <= 0, a degree < 1 or a NULL pointer. */
int chfsi_split_schedule(int n_wanted, int ka, const double* mu, const double* res,
                         const int* deg, double c, double e, double tol, double norm_h, int form,
                         signed char* steps);

/* Input features of the degree network for wanted vector j (host only),
 * with t = (mu_j - c)/e, c, e from alpha and beta, |rho| = |t| + sqrt(t^2-1):
 *   f0 = ln(max(res_j, tol_abs) / tol_abs)   f1 = ln(ln|rho|)
 *   f2 = ln(max(f0 / ln|rho|, 1/2))          f3 = ln|t|
 *   f4 = (mu_j - gamma) / (alpha - gamma)    f5 = ln(max(gap_j / e, 1e-12))
 *   f6 = ln(max(res_j, 1e-300) / norm_h)     f7 = min(loop - 1, 4)
 * Writes 8 doubles to f and returns CHFSI_OK, or CHFSI_INVALID_ARG when
 * |t| <= 1 (no analytic rate; such vectors take the guard degree). */
int chfsi_degree_features(double mu, double res, double gap, double alpha, double beta,
                          double gamma, double norm_h, double tol_abs, int loop, double* f);

/* Learned per-vector degrees (degree_mode 2), the network run by the
 * library's HIP kernel: for wanted vector j with features f (above) and
 * prediction y, m_j = max(ceil(m_a * exp(margin - y)), r_j) clamped to
 * [1, deg_max], with m_a = f0 / ln|rho| the analytic continuous degree and
 * r_j the analytic degree (chfsi_degrees).  r_j is used alone when
 * |t_j| <= 1, when a standardised feature lies outside [-6, 6] or when y is
 * not finite.  The blob's margin is applied only when the loop can finish
 * every wanted vector, i.e. every ceil(m_a * exp(-y)) (m_a for the rule's
 * vectors) is <= deg_max; otherwise margin 0 is used.  In the solver's
 * mixed mode a loop that must be capped to FP32's reach also uses margin 0.
 * Guards and the vectors without a rate get the largest wanted degree.
 *   mu, res   HOST, k doubles (ascending mu).  params HOST blob.
 *   deg       HOST, k ints out.  pred, src: HOST k floats / ints out or NULL
 *             (src: 0 rule fallback, 1 network, 2 guard fill).
 *   work      device, >= chfsi_mlp_workspace_bytes(k). */
int chfsi_degrees_learned(int k, const double* mu, const double* res, int n_wanted,
                          double alpha, double beta, double gamma, double norm_h, double tol_abs,
                          int loop, int deg_max, const float* params, void* work,
                          size_t work_bytes, void* stream, int* deg, float* pred, int* src);

/* Sequence-calibrated degrees (degree_mode 3), host only: with speed_j the
 * measured speed of vector j (NaN when unknown) and m_a,j the analytic
 * continuous degree, m_j = max(r_j, ceil(m_a,j * f / speed_j)) clamped to
 * [1, deg_max] (r_j: chfsi_degrees), f = 1.25 when every calibrated
 * ceil(m_a,j / speed_j) and every uncalibrated ceil(m_a,j) is <= deg_max,
 * else 1.  Unknown speeds take r_j; guards and vectors with |t_j| <= 1 the
 * largest wanted degree.  speed may be NULL (all unknown).  src: HOST k
 * ints out or NULL (0 rule, 1 calibrated, 2 guard fill). */
int chfsi_degrees_sequence(int k, const double* mu, const double* res, const double* speed,
                           int n_wanted, double alpha, double beta, double tol_abs, int deg_max,
                           int* deg, int* src);

/* Training and inference kernels of the degree network (device buffers,
 * FP32).  X is n x 8 row-major, T and y hold n floats, params / grad / m /
 * v hold CHFSI_MLP_PARAMS floats.
 *   chfsi_mlp_forward:  y = net(X).
 *   chfsi_mlp_gradient: grad = d/dparams of (1/n) sum (net(X_s) - T_s)^2
 *     (zero for the statistics and the margin), loss (device, 1 float) =
 *     sum of squared errors.  Sums run in a fixed order (deterministic).
 *   chfsi_mlp_adam:     one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 *     bias-corrected, step number t >= 1) on the weights and biases.
 *   chfsi_mlp_train:    `steps` full-batch Adam steps from params (in/out),
 *     moments starting at zero; loss_out HOST (steps floats, mean squared
 *     error before each step) or NULL.
 * work >= chfsi_mlp_workspace_bytes(n). */
size_t chfsi_mlp_workspace_bytes(int n);
int chfsi_mlp_forward(int n, const float* X, const float* params, float* y, void* stream);
int chfsi_mlp_gradient(int n, const float* X, const float* T, const float* params, float* grad,
                       float* loss, void* work, size_t work_bytes, void* stream);
int chfsi_mlp_adam(float* params, const float* grad, float* m, float* v, float lr, int t,
                   void* stream);
int chfsi_mlp_train(int n, const float* X, const float* T, float* params, int steps, float lr,
                    void* work, size_t work_bytes, void* stream, float* loss_out);

/* Filter tile autotuner.  The FP64 Chebyshev-step kernel exists in
 * CHFSI_FILTER_VARIANTS variants: 0 (64 x 64 tiles, the 4M complex split:
 * four real products per complex multiply-add) stages K 8 deep through LDS
 * with four workgroups per CU, 1 stages it 16 deep with two per CU, 2 uses
 * 128 x 128 tiles of 16 waves (one workgroup per CU; windows of N >= 256
 * columns, and not in the grouped launches of chfsi_solve_batch, which take
 * the default instead); 3 and 4 are 0 and 1 with the 3M split (three real products
 * Ar Br, Ai Bi, (Ar + Ai)(Br + Bi) per complex multiply-add; three and two
 * workgroups per CU); 5 and 6 load both operands straight into LDS (no
 * register staging), 5 with the 3M split and three stages in flight, 6
 * with 4M and two.  Variant 5 is the default; another is kept only when it
 * is 2 % faster.  chfsi_autotune_filter times them on each given
 * launch shape (an n x n Hermitian-sized operand times an n x N block, the
 * width N of a filter window; synthetic data in `work`), records the fastest
 * one per device, and every later filter step (single or batched) takes
 * the choice of the nearest recorded shape (log distance in n and N; with
 * none recorded, variant 5).
 *   variant  HOST, count ints out.   tflops  HOST,
 *   CHFSI_FILTER_VARIANTS * count doubles out (complex-equivalent TFLOP/s,
 *   8 n^2 N flops per step for every variant, per shape in variant order;
 *   0.0 where not timed) or NULL.
 *   work     device, >= chfsi_autotune_workspace_bytes(max n, max N).
 * chfsi_autotune_set records a choice directly; chfsi_autotune_reset
 * clears the current device's table. */
#define CHFSI_FILTER_VARIANTS 7
size_t chfsi_autotune_workspace_bytes(int n_max, int N_max);
int chfsi_autotune_filter(int count, const int* n, const int* N, void* work, size_t work_bytes,
                          void* stream, int* variant, double* tflops);
int chfsi_autotune_set(int n, int N, int variant);
int chfsi_autotune_reset(void);

/* General complex GEMM on the library's MFMA kernels:
 * C <- alpha op(A) op(B) + beta C with op in {'N', 'C'} (no-op or conjugate
 * transpose); C is M x N, the inner dimension K.  alpha, beta are complex
 * (HOST, two doubles each).  Uses split-K (and `work`) when M*N is small
 * compared with K, or when K >= 4096 and the last round of workgroups would
 * be far from full.  For K >= 512 the product runs the 3M split (three real
 * products per complex multiply-add): its error stays within a small
 * multiple of eps K max|A| |B| per element, as 4M's does, though the
 * imaginary part's bound is (|Ar| + |Ai|)(|Br| + |Bi|) instead of |A| |B|.
 * C must not overlap A or B. */
int chfsi_zgemm(char opa, char opb, int M, int N, int K,
                const double* alpha, const void* A, int lda, const void* B, int ldb,
                const double* beta, void* C, int ldc,
                void* work, size_t work_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CHFSI_H */
