// Complex FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64).
//
// C = op(A) op(B) is computed with the 4M real split
//   Cr = Ar Br - Ai Bi,   Ci = Ar Bi + Ai Br
// i.e. four real 16x16x4 MFMAs per complex 16x16x4 product, 8 real flops
// per complex multiply-add.  This GEMM is the work of the Chebyshev filter
// (the three-term recurrence of Alg. 2 / eq. 3term in the paper), whose
// epilogue is fused here: the product H*Y_i is never written, the kernel
// writes Y_{i+1} = sa (H Y_i - c Y_i) - sb Y_{i-1} directly over Y_{i-1}.
//
// Tiling: a 256-thread workgroup (4 wave64) owns a 64x64 complex tile of C;
// each wave owns 32x32 (2x2 MFMA tiles, real and imaginary accumulators).
// K advances 8 complex elements per stage through a double-buffered LDS
// tile stored k-major ([k][m] and [k][n]) with a one-element pad so that
// both the coalesced global->LDS transposes and the MFMA operand reads are
// free of bank conflicts.  Operands may be plain (column-major) or
// conjugate-transposed; the loader handles either orientation.
//
// Scheduling: workgroups are dispatched round-robin over the 8 XCDs.  The
// logical tile order is remapped so that consecutive tiles (same row strip
// of A, different column tiles of B) land on the same XCD and share the A
// strip in that XCD's L2.
#include "internal.h"

#include <atomic>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace chfsi {

namespace {

constexpr int BM = 64, BN = 64, BK = 8, NT = 256;
constexpr int GENERAL_3M_MIN_K = 512;   // general products of K >= this use 3M
constexpr int PA = BM + 1, PB = BN + 1;   // LDS pitches in complex elements
constexpr int NXCD = 8;

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ zc cmul(zc a, zc b) {
  return zc{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Global -> registers for one KB x BM stage of op(A) (KB / 4 elements per
// thread).
template <int OPA, int KB>
__device__ __forceinline__ void load_a(const GemmArgs& g, int m0, int k0, int kend, zc r[KB / 4]) {
  const int t = threadIdx.x;
  if (OPA == OP_N) {            // (m, k) = A[m + k lda], m contiguous
    const int m = m0 + (t & 63);
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) {
      const int k = k0 + (t >> 6) + 4 * i;
      r[i] = (m < g.M && k < kend) ? g.A[m + (long)k * g.lda] : zc{0.0, 0.0};
    }
  } else {                      // (m, k) = conj(A[k + m lda]), k contiguous
    const int k = k0 + (t & (KB - 1));
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) {
      const int m = m0 + t / KB + (NT / KB) * i;
      zc v = (m < g.M && k < kend) ? g.A[k + (long)m * g.lda] : zc{0.0, 0.0};
      r[i] = zc{v.x, -v.y};
    }
  }
}

template <int OPA, int KB>
__device__ __forceinline__ void store_a(zc (*As)[PA], const zc r[KB / 4]) {
  const int t = threadIdx.x;
  if (OPA == OP_N) {
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) As[(t >> 6) + 4 * i][t & 63] = r[i];
  } else {
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) As[t & (KB - 1)][t / KB + (NT / KB) * i] = r[i];
  }
}

// Global -> registers for one KB x BN stage of op(B).
template <int OPB, int KB>
__device__ __forceinline__ void load_b(const GemmArgs& g, int n0, int k0, int kend, zc r[KB / 4]) {
  const int t = threadIdx.x;
  if (OPB == OP_N) {            // (k, n) = B[k + n ldb], k contiguous
    const int k = k0 + (t & (KB - 1));
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) {
      const int n = n0 + t / KB + (NT / KB) * i;
      r[i] = (n < g.N && k < kend) ? g.B[k + (long)n * g.ldb] : zc{0.0, 0.0};
    }
  } else {                      // (k, n) = conj(B[n + k ldb]), n contiguous
    const int n = n0 + (t & 63);
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) {
      const int k = k0 + (t >> 6) + 4 * i;
      zc v = (n < g.N && k < kend) ? g.B[n + (long)k * g.ldb] : zc{0.0, 0.0};
      r[i] = zc{v.x, -v.y};
    }
  }
}

template <int OPB, int KB>
__device__ __forceinline__ void store_b(zc (*Bs)[PB], const zc r[KB / 4]) {
  const int t = threadIdx.x;
  if (OPB == OP_N) {
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) Bs[t & (KB - 1)][t / KB + (NT / KB) * i] = r[i];
  } else {
#pragma unroll
    for (int i = 0; i < KB / 4; ++i) Bs[(t >> 6) + 4 * i][t & 63] = r[i];
  }
}

// Lower-triangle tile enumeration: t -> (tm, tn) with tn <= tm.
__device__ __forceinline__ void lower_tile(int t, int& tm, int& tn) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tm = r;
  tn = t - r * (r + 1) / 2;
}

// One 64x64 output tile (tile row tm, tile column tn, K chunk `split`) of
// the launch described by g, with its epilogue; K staged KB deep in LDS;
// CM real products per complex multiply-add (4: the 4M split, 3: 3M).
template <int OPA, int OPB, int EPI, int KB, int CM>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int split, int tm, int tn,
                                          zc (*As)[KB][PA], zc (*Bs)[KB][PB]);

// Lower-triangle tile set without split-K, XCD-aware: XCD x (workgroup w
// runs on XCD w % 8) takes the tile rows tm = x (mod 8) from the bottom row
// up, each row's tiles tn = 0 .. tm in order, so a row's A strip stays in
// one XCD's L2 and the rows with the most tiles (and, for triangular K
// ranges, the longest ones) start first.  Row i of XCD x (tm = top - 8 i)
// holds top + 1 - 8 i tiles, S(i) = i (top + 5) - 4 i^2 precede it.
// Returns false when workgroup b has no tile.
__device__ __forceinline__ bool lower_tile_xcd(const GemmArgs& g, int b, int& tm, int& tn) {
  const int x = b % NXCD, slot = b / NXCD;
  if (x >= g.tiles_m) return false;
  const int top = x + NXCD * ((g.tiles_m - 1 - x) / NXCD);
  const int rows = (top - x) / NXCD + 1;
  auto S = [&](int i) { return (long)i * (top + 5) - 4L * i * i; };
  const double a = top + 5.0;
  int i = (int)((a - sqrt(fmax(a * a - 16.0 * slot, 0.0))) / 8.0);
  while (i > 0 && S(i) > slot) --i;
  while (i + 1 <= rows && S(i + 1) <= slot) ++i;
  if (i >= rows) return false;
  tm = top - NXCD * i;
  tn = slot - (int)S(i);
  return true;
}

// Workgroups of the lower_tile_xcd schedule: 8 x the largest per-XCD count.
int lower_xcd_grid(int tiles_m) {
  long best = 0;
  for (int x = 0; x < NXCD && x < tiles_m; ++x) {
    const long top = x + NXCD * ((tiles_m - 1 - x) / NXCD);
    const long rows = (top - x) / NXCD + 1;
    best = std::max(best, rows * (top + 5) - 4 * rows * rows);
  }
  return (int)(best * NXCD);
}

// Virtual-row scheduling of a rectangular tile set (see zgemm_kernel):
// returns false when workgroup `local` has no tile.
__device__ __forceinline__ bool rect_tile(const GemmArgs& g, int local, int& split, int& tm,
                                          int& tn) {
  const int xcd = local % NXCD, slot = local / NXCD;
  const int vrows = g.splits * g.tiles_m;
  const int rows_x = (vrows - xcd + NXCD - 1) / NXCD;
  const int ri = slot / g.tiles_n;
  tn = slot - ri * g.tiles_n;
  if (ri >= rows_x) return false;
  const int v = xcd + NXCD * (g.rows_desc ? rows_x - 1 - ri : ri);
  split = v / g.tiles_m;
  tm = v - split * g.tiles_m;
  return true;
}

// Resident workgroups per CU: KB = 8 with the 4M split: four (16 waves);
// the kernel fits in 128 registers per lane without spills, with
// accumulators in VGPRs.  The 3M form holds three accumulator sets instead
// of two (32 more registers per lane): three per CU.  KB = 16 (twice the
// LDS per workgroup): two per CU.
constexpr int tile_occupancy(int KB, int CM) { return KB == 8 ? (CM == 4 ? 4 : 3) : 2; }

template <int OPA, int OPB, int EPI, int KB, int CM>
__global__ void __launch_bounds__(NT, tile_occupancy(KB, CM)) zgemm_kernel(GemmArgs g) {
  __shared__ zc As[2][KB][PA];
  __shared__ zc Bs[2][KB][PB];

  // Tile scheduling.  Workgroups are dispatched round-robin over the XCDs
  // (hardware id w runs on XCD w % 8).  For rectangular tile sets XCD x owns
  // the (virtual) tile rows v = x, x + 8, ...: all column tiles of a row stay
  // on one XCD and share the A strip in its L2, and every XCD gets a mix of
  // rows, which balances triangular K ranges.  A virtual row is a (split,
  // tile row) pair.
  int split, tm, tn;
  if (g.lower_only && g.splits == 1) {
    split = 0;
    if (!lower_tile_xcd(g, blockIdx.x, tm, tn)) return;
  } else if (g.lower_only) {
    const int logical = blockIdx.x;
    if (logical >= g.total_tiles * g.splits) return;
    split = logical / g.total_tiles;
    lower_tile(logical - split * g.total_tiles, tm, tn);
  } else {
    if (!rect_tile(g, blockIdx.x, split, tm, tn)) return;
  }
  gemm_tile<OPA, OPB, EPI, KB, CM>(g, split, tm, tn, As, Bs);
}

// Several independent Chebyshev steps (one per problem of a batch) in one
// launch: problem p owns workgroups [slot_begin[p], slot_begin[p + 1]), a
// multiple of the XCD count, scheduled inside its range exactly as a launch
// of its own.
template <int KB, int CM>
__global__ void __launch_bounds__(NT, tile_occupancy(KB, CM))
    zgemm_group_cheb(const GemmArgs* __restrict__ list, const int* __restrict__ slot_begin,
                     int count) {
  __shared__ zc As[2][KB][PA];
  __shared__ zc Bs[2][KB][PB];
  const int b = blockIdx.x;
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (slot_begin[mid] <= b) lo = mid;
    else hi = mid;
  }
  const GemmArgs g = list[lo];
  int split, tm, tn;
  if (!rect_tile(g, b - slot_begin[lo], split, tm, tn)) return;
  gemm_tile<OP_N, OP_N, EPI_CHEB, KB, CM>(g, split, tm, tn, As, Bs);
}

// Wide filter step (tile variant 2): 128 x 128 output tiles, 16 waves in a
// 4 x 4 grid of 32 x 32 sub-tiles, K 8 deep; one workgroup per CU.  Twice
// the reuse of each H element in LDS of the 64 x 64 tile, for wide windows.
constexpr int WBM = 128, WBN = 128, WNT = 1024, WPA = WBM + 1, WPB = WBN + 1;

__global__ void __launch_bounds__(WNT, 1) cheb_wide_kernel(GemmArgs g) {
  __shared__ zc As[2][BK][WPA];
  __shared__ zc Bs[2][BK][WPB];
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
  d4 accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accI[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }
  // one element of each operand per thread and stage: A (m, k) with m
  // contiguous, B (k, n) with k contiguous
  const int am = m0 + (t & (WBM - 1)), ak = t / WBM;
  const int bk = t & (BK - 1), bn = n0 + t / BK;
  const int nk = (g.K + BK - 1) / BK;
  zc ra = zc{0.0, 0.0}, rb = zc{0.0, 0.0};
  auto load = [&](int k0) {
    const int ka = k0 + ak, kb = k0 + bk;
    ra = (am < g.M && ka < g.K) ? g.A[am + (long)ka * g.lda] : zc{0.0, 0.0};
    rb = (bn < g.N && kb < g.K) ? g.B[kb + (long)bn * g.ldb] : zc{0.0, 0.0};
  };
  if (nk > 0) {
    load(0);
    As[0][ak][t & (WBM - 1)] = ra;
    Bs[0][bk][t / BK] = rb;
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) load((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      zc a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[cur][kk * 4 + lk][wm * 32 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[cur][kk * 4 + lk][wn * 32 + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accR[i][j] = mfma(a[i].x, b[j].x, accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accI[i][j] = mfma(a[i].x, b[j].y, accI[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accR[i][j] = mfma(-a[i].y, b[j].y, accR[i][j]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) accI[i][j] = mfma(a[i].y, b[j].x, accI[i][j]);
    }
    if (more) {
      As[cur ^ 1][ak][t & (WBM - 1)] = ra;
      Bs[cur ^ 1][bk][t / BK] = rb;
    }
    __syncthreads();
  }
  // epilogue of the three-term step (FP64 MFMA output: row (l / 16) + 4 r)
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + i * 16 + lk + 4 * r;
        const int col = n0 + wn * 32 + j * 16 + lr;
        if (row >= g.M || col >= g.N) continue;
        const zc yc = g.Ycur[row + (long)col * g.ldyc];
        zc out = zc{g.sa * (accR[i][j][r] - g.shift * yc.x), g.sa * (accI[i][j][r] - g.shift * yc.y)};
        if (g.sb != 0.0) {
          const zc yo = g.Yold[row + (long)col * g.ldyo];
          out.x -= g.sb * yo.x;
          out.y -= g.sb * yo.y;
        }
        g.C[row + (long)col * g.ldc] = out;
      }
}

// Epilogue of a wave's 32 x 32 sub-tile at (r0, c0).  MFMA output layout:
// lane l, register r holds row (l / 16) + 4 r and column l % 16 of the
// 16x16 tile.  The accumulators are combined per the complex split (4M:
// acc0 = Re, acc1 = Im; 3M: Re = acc0 - acc1, Im = acc2 - acc0 - acc1).
template <int EPI, int CM>
__device__ __forceinline__ void tile_store(const GemmArgs& g, int split, int r0, int c0, int lr,
                                           int lk, const d4 (&acc0)[2][2],
                                           const d4 (&acc1)[2][2], const d4 (&acc2)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + i * 16 + lk + 4 * r;
        const int col = c0 + j * 16 + lr;
        if (row >= g.M || col >= g.N) continue;
        const zc acc = CM == 4 ? zc{acc0[i][j][r], acc1[i][j][r]}
                               : zc{acc0[i][j][r] - acc1[i][j][r],
                                    (acc2[i][j][r] - acc0[i][j][r]) - acc1[i][j][r]};
        if (EPI == EPI_STORE) {
          zc out = cmul(g.alpha, acc);
          zc* cp = g.C + row + (long)col * g.ldc;
          if (g.beta.x != 0.0 || g.beta.y != 0.0) {
            const zc cv = *cp;
            const zc bc = cmul(g.beta, cv);
            out.x += bc.x;
            out.y += bc.y;
          }
          *cp = out;
        } else if (EPI == EPI_CHEB) {
          const zc yc = g.Ycur[row + (long)col * g.ldyc];
          zc out = zc{g.sa * (acc.x - g.shift * yc.x), g.sa * (acc.y - g.shift * yc.y)};
          if (g.sb != 0.0) {
            const zc yo = g.Yold[row + (long)col * g.ldyo];
            out.x -= g.sb * yo.x;
            out.y -= g.sb * yo.y;
          }
          g.C[row + (long)col * g.ldc] = out;
        } else {
          g.part[(long)split * g.M * g.N + row + (long)col * g.M] = acc;
        }
      }
}

// K range [kbeg, kend) of tile (tm, tn) in K chunk `split`, after the
// triangular-operand limits.
__device__ __forceinline__ void tile_k_range(const GemmArgs& g, int split, int m0, int n0,
                                             int& kbeg, int& kend) {
  kbeg = split * g.kchunk;
  kend = min(g.K, kbeg + g.kchunk);
  if (g.ktri == KTRI_A_LOWER) kend = min(kend, m0 + BM);
  else if (g.ktri == KTRI_B_UPPER) kend = min(kend, n0 + BN);
  else if (g.ktri == KTRI_A_UPPER) kbeg = max(kbeg, m0);
  else if (g.ktri == KTRI_AB_LOWER) {
    kbeg = max(kbeg, n0);
    kend = min(kend, m0 + BM);
  } else if (g.ktri == KTRI_A_LOWER_B_UPPER) {
    kend = min(kend, min(m0 + BM, n0 + BN));
  }
}

template <int OPA, int OPB, int EPI, int KB, int CM>
__device__ __forceinline__ void gemm_tile(const GemmArgs& g, int split, int tm, int tn,
                                          zc (*As)[KB][PA], zc (*Bs)[KB][PB]) {
  static_assert(CM == 3 || CM == 4, "4M or 3M split");
  const int m0 = tm * BM, n0 = tn * BN;
  int kbeg, kend;
  tile_k_range(g, split, m0, n0, kbeg, kend);

  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int lr = lane & 15, lk = lane >> 4;

  // 4M: acc0 = Re, acc1 = Im.  3M: acc0 = Ar Br, acc1 = Ai Bi,
  // acc2 = (Ar + Ai)(Br + Bi); Re = acc0 - acc1, Im = acc2 - acc0 - acc1.
  d4 acc0[2][2], acc1[2][2], acc2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc0[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acc1[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acc2[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  const int nk = (kend - kbeg + KB - 1) / KB;
  zc ra[KB / 4], rb[KB / 4];
  if (nk > 0) {
    load_a<OPA, KB>(g, m0, kbeg, kend, ra);
    load_b<OPB, KB>(g, n0, kbeg, kend, rb);
    store_a<OPA, KB>(As[0], ra);
    store_b<OPB, KB>(Bs[0], rb);
  }
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) {
      const int k0 = kbeg + (kt + 1) * KB;
      load_a<OPA, KB>(g, m0, k0, kend, ra);
      load_b<OPB, KB>(g, n0, k0, kend, rb);
    }
#pragma unroll
    for (int kk = 0; kk < KB / 4; ++kk) {
      zc a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[cur][kk * 4 + lk][wm * 32 + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[cur][kk * 4 + lk][wn * 32 + j * 16 + lr];
      if constexpr (CM == 4) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc0[i][j] = mfma(a[i].x, b[j].x, acc0[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc1[i][j] = mfma(a[i].x, b[j].y, acc1[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc0[i][j] = mfma(-a[i].y, b[j].y, acc0[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc1[i][j] = mfma(a[i].y, b[j].x, acc1[i][j]);
      } else {
        double as[2], bs[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) as[i] = a[i].x + a[i].y;
#pragma unroll
        for (int j = 0; j < 2; ++j) bs[j] = b[j].x + b[j].y;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc0[i][j] = mfma(a[i].x, b[j].x, acc0[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc1[i][j] = mfma(a[i].y, b[j].y, acc1[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc2[i][j] = mfma(as[i], bs[j], acc2[i][j]);
      }
    }
    if (more) {
      store_a<OPA, KB>(As[cur ^ 1], ra);
      store_b<OPB, KB>(Bs[cur ^ 1], rb);
    }
    __syncthreads();
  }

  tile_store<EPI, CM>(g, split, m0 + wm * 32, n0 + wn * 32, lr, lk, acc0, acc1, acc2);
}

// Direct-to-LDS form of the tile for op(A) = A, op(B) = B (the filter step
// and the plain products): both operands go from global memory straight
// into LDS with global_load_lds_dwordx4 (lane L of an instruction writes
// the 16 bytes at LDS offset 16 L from the wave's pointer), so no registers
// hold staged data and loads run DMA_STAGES(CM) - 1 stages ahead of the
// MFMAs.  Stage layout: the A rows k = 0..7 of 64 complex elements, m
// contiguous, pitch PA elements (one instruction per row: the column
// segment A[m0 .. m0 + 63, k] is 1 KB contiguous); then the B rows n =
// 0..63 of 8 complex elements (128 B, k contiguous as in memory), the
// 16-byte chunk of k stored at position k ^ ((n >> 1) & 7) so that the
// MFMA operand reads of 16 consecutive rows fall on 16 distinct 16-byte
// bank groups (one instruction fills 8 rows).  Out-of-range operands: rows
// m >= M and columns n >= N read the last valid row or column (their
// products only reach outputs that are not stored); A rows k >= K read row
// K - 1, and B elements with k >= kend read a zero page, so the K tail adds
// exact zeros.  With op(B) = B^H (OPB = OP_C: element (k, n) is the
// conjugate of B[n + k ldb]) the rows k of op(B)'s panel are 1 KB contiguous
// segments as well: they are staged like A's (pitch PB, one instruction
// per row, the conjugation applied to the operand registers), and their K
// tail (k >= kend) comes from the zero page.
constexpr int DKB = 8;                               // K per stage
constexpr int DA_BYTES = DKB * PA * 16;              // 8320
constexpr int DB_BYTES = BN * DKB * 16;              // 8192
constexpr int DSTAGE = DA_BYTES + DB_BYTES;          // 16512
constexpr int dma_stages(int CM) { return CM == 3 ? 3 : 2; }
constexpr int dma_stage_bytes(int OPB) {
  return DA_BYTES + (OPB == OP_N ? DB_BYTES : DKB * PB * 16);
}

__device__ __align__(16) double dma_zero_page[2];    // zero-initialised

// One LDS-DMA load: lane L's 16 bytes at gsrc go to LDS byte lds + 16 L
// (lds wave-uniform).  Issued in asm so that the compiler, which does not
// see the LDS write, inserts no wait for it before the LDS reads of the
// other stages; the caller waits with vmcnt before reading this stage (and
// a barrier for the other waves' loads).  No output register.  M0 is a
// register the compiler reserves and does not otherwise use in these
// kernels (no clobber can be declared for it): the block sets it right
// before the load.
__device__ __forceinline__ void lds_dma16(const void* gsrc, unsigned lds) {
  asm volatile(
      "s_mov_b32 m0, %0\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %1, off" ::"s"(lds),
      "v"(gsrc)
      : "memory");
}

template <int EPI, int CM, int OPB = OP_N>
__device__ __forceinline__ void gemm_tile_dma(const GemmArgs& g, int split, int tm, int tn,
                                              char* lds) {
  static_assert(CM == 3 || CM == 4, "4M or 3M split");
  constexpr int NS = dma_stages(CM);
  constexpr int DSTAGE = dma_stage_bytes(OPB);
  const int m0 = tm * BM, n0 = tn * BN;
  int kbeg, kend;
  tile_k_range(g, split, m0, n0, kbeg, kend);
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int lr = lane & 15, lk = lane >> 4;

  d4 acc0[2][2], acc1[2][2], acc2[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc0[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acc1[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acc2[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  // this wave's instructions per stage: A rows k = 4 i + wave (i = 0, 1);
  // B rows n = 8 (4 j + wave) + lane / 8 (j = 0, 1), the chunk that belongs
  // at position lane % 8
  const zc* a_src = g.A + min(m0 + lane, g.M - 1);
  const int bn_row0 = 8 * wave + (lane >> 3), bn_row1 = 8 * (4 + wave) + (lane >> 3);
  const int bc0 = (lane & 7) ^ ((bn_row0 >> 1) & 7), bc1 = (lane & 7) ^ ((bn_row1 >> 1) & 7);
  const zc* b_col0 = g.B + (long)min(n0 + bn_row0, g.N - 1) * g.ldb;
  const zc* b_col1 = g.B + (long)min(n0 + bn_row1, g.N - 1) * g.ldb;
  const zc* zero = (const zc*)dma_zero_page;
  // LDS byte address of the workgroup's ring, uniform
  const unsigned lds_base = (unsigned)(size_t)(__attribute__((address_space(3))) char*)lds;
  const unsigned wave_u = (unsigned)__builtin_amdgcn_readfirstlane(wave);
  // stages that lie wholly inside [kbeg, kend) (all but possibly the last)
  // advance four fixed per-lane pointers by a uniform offset; the last one
  // clamps A's rows and reads B's tail from the zero page
  const zc* pa0 = a_src + (long)(kbeg + wave) * g.lda;
  const zc* pa1 = pa0 + 4 * g.lda;
  const zc* pb0 = b_col0 + kbeg + bc0;
  const zc* pb1 = b_col1 + kbeg + bc1;
  // op(B) = B^H: rows k = 4 j + wave of the k-major panel, lane L taking
  // column n0 + L
  const zc* bh_src = g.B + min(n0 + lane, g.N - 1);
  const zc* ph0 = bh_src + (long)(kbeg + wave) * g.ldb;
  const zc* ph1 = ph0 + 4 * g.ldb;
  auto load = [&](int k0, unsigned st) {
    if (k0 + DKB <= kend) {
      const long ao = (long)(k0 - kbeg) * g.lda;
      lds_dma16(pa0 + ao, st + wave_u * PA * 16);
      lds_dma16(pa1 + ao, st + (4 + wave_u) * PA * 16);
      if constexpr (OPB == OP_N) {
        const int bo = k0 - kbeg;
        lds_dma16(pb0 + bo, st + DA_BYTES + wave_u * 1024);
        lds_dma16(pb1 + bo, st + DA_BYTES + (4 + wave_u) * 1024);
      } else {
        const long bo = (long)(k0 - kbeg) * g.ldb;
        lds_dma16(ph0 + bo, st + DA_BYTES + wave_u * PB * 16);
        lds_dma16(ph1 + bo, st + DA_BYTES + (4 + wave_u) * PB * 16);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int k = min(k0 + 4 * i + wave, g.K - 1);
        lds_dma16(a_src + (long)k * g.lda, st + (4 * i + wave_u) * PA * 16);
      }
      if constexpr (OPB == OP_N) {
        const int k0c = k0 + bc0, k1c = k0 + bc1;
        lds_dma16(k0c < kend ? b_col0 + k0c : zero, st + DA_BYTES + wave_u * 1024);
        lds_dma16(k1c < kend ? b_col1 + k1c : zero, st + DA_BYTES + (4 + wave_u) * 1024);
      } else {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int k = k0 + 4 * j + wave;
          lds_dma16(k < kend ? bh_src + (long)k * g.ldb : zero,
                    st + DA_BYTES + (4 * j + wave_u) * PB * 16);
        }
      }
    }
  };
  auto compute = [&](const char* st) {
    const char* sb = st + DA_BYTES;
#pragma unroll
    for (int kk = 0; kk < DKB / 4; ++kk) {
      const int k = kk * 4 + lk;
      zc a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *(const zc*)(st + (k * PA + wm * 32 + i * 16 + lr) * 16);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if constexpr (OPB == OP_N) {
          const int n = wn * 32 + j * 16 + lr;
          b[j] = *(const zc*)(sb + n * (DKB * 16) + ((k ^ ((n >> 1) & 7)) * 16));
        } else {
          const zc v = *(const zc*)(sb + (k * PB + wn * 32 + j * 16 + lr) * 16);
          b[j] = zc{v.x, -v.y};
        }
      }
      if constexpr (CM == 4) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc0[i][j] = mfma(a[i].x, b[j].x, acc0[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc1[i][j] = mfma(a[i].x, b[j].y, acc1[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc0[i][j] = mfma(-a[i].y, b[j].y, acc0[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc1[i][j] = mfma(a[i].y, b[j].x, acc1[i][j]);
      } else {
        double as[2], bs[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) as[i] = a[i].x + a[i].y;
#pragma unroll
        for (int j = 0; j < 2; ++j) bs[j] = b[j].x + b[j].y;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc0[i][j] = mfma(a[i].x, b[j].x, acc0[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc1[i][j] = mfma(a[i].y, b[j].y, acc1[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc2[i][j] = mfma(as[i], bs[j], acc2[i][j]);
      }
    }
  };

  // NS stages in a ring: stage kt is computed while the loads of stages
  // up to kt + NS - 1 are in flight; each stage ends with this wave's loads
  // of the next stage landed (vmcnt counts the 4 loads per stage in order,
  // and no other vector memory operation is issued in the loop) and a
  // barrier, after which the stage just computed is free
  const int nk = (kend - kbeg + DKB - 1) / DKB;
  if (nk > 0) {
    load(kbeg, lds_base);
    if (NS == 3 && nk > 1) {
      load(kbeg + DKB, lds_base + DSTAGE);
      asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
    } else {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
  }
  __syncthreads();
  int cur = 0;
  for (int kt = 0; kt < nk; ++kt) {
    const bool issue = kt + NS - 1 < nk;
    if (issue) {
      int st = cur + NS - 1;
      if (st >= NS) st -= NS;
      load(kbeg + (kt + NS - 1) * DKB, lds_base + st * DSTAGE);
    }
    compute(lds + cur * DSTAGE);
    __builtin_amdgcn_sched_barrier(0);
    if (NS == 3 && issue) asm volatile("s_waitcnt vmcnt(4)" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    cur = cur + 1 == NS ? 0 : cur + 1;
  }
  tile_store<EPI, CM>(g, split, m0 + wm * 32, n0 + wn * 32, lr, lk, acc0, acc1, acc2);
}

template <int EPI, int CM, int OPB>
__global__ void __launch_bounds__(NT, CM == 3 ? 3 : 4) zgemm_dma_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(1024))) char lds[dma_stages(CM) * dma_stage_bytes(OPB)];
  int split, tm, tn;
  if (!rect_tile(g, blockIdx.x, split, tm, tn)) return;
  gemm_tile_dma<EPI, CM, OPB>(g, split, tm, tn, lds);
}

// Lower-triangle tile sets without split-K (the reduction's Linv T), in
// the per-XCD order of lower_tile_xcd.
template <int EPI, int CM>
__global__ void __launch_bounds__(NT, CM == 3 ? 3 : 4) zgemm_dma_lower_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(1024))) char lds[dma_stages(CM) * DSTAGE];
  int tm, tn;
  if (!lower_tile_xcd(g, blockIdx.x, tm, tn)) return;
  gemm_tile_dma<EPI, CM, OP_N>(g, 0, tm, tn, lds);
}

template <int CM>
__global__ void __launch_bounds__(NT, CM == 3 ? 3 : 4)
    zgemm_group_cheb_dma(const GemmArgs* __restrict__ list, const int* __restrict__ slot_begin,
                         int count) {
  __shared__ __attribute__((aligned(1024))) char lds[dma_stages(CM) * DSTAGE];
  const int b = blockIdx.x;
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (slot_begin[mid] <= b) lo = mid;
    else hi = mid;
  }
  const GemmArgs g = list[lo];
  int split, tm, tn;
  if (!rect_tile(g, b - slot_begin[lo], split, tm, tn)) return;
  gemm_tile_dma<EPI_CHEB, CM>(g, split, tm, tn, lds);
}

// Sum the split-K partials in a fixed order: C = alpha sum_s P_s + beta C.
__global__ void splitk_reduce(int M, int N, int splits, const zc* part, zc alpha, zc beta,
                              zc* C, long ldc, int lower_only) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M * N) return;
  const int row = (int)(idx % M), col = (int)(idx / M);
  if (lower_only && row / BM < col / BN) return;
  zc s = zc{0.0, 0.0};
  for (int p = 0; p < splits; ++p) {
    const zc v = part[(long)p * M * N + idx];
    s.x += v.x;
    s.y += v.y;
  }
  zc out = cmul(alpha, s);
  zc* cp = C + row + (long)col * ldc;
  if (beta.x != 0.0 || beta.y != 0.0) {
    const zc b = cmul(beta, *cp);
    out.x += b.x;
    out.y += b.y;
  }
  *cp = out;
}

// Split-K Chebyshev step: Yout = sa (sum_s P_s - shift Ycur) - sb Yold.
__global__ void cheb_reduce(int M, int N, int splits, const zc* part, const zc* Ycur, long ldyc,
                            const zc* Yold, long ldyo, zc* Yout, long ldyout, double shift,
                            double sa, double sb) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M * N) return;
  const int row = (int)(idx % M), col = (int)(idx / M);
  zc s = zc{0.0, 0.0};
  for (int p = 0; p < splits; ++p) {
    const zc v = part[(long)p * M * N + idx];
    s.x += v.x;
    s.y += v.y;
  }
  const zc yc = Ycur[row + (long)col * ldyc];
  zc out = zc{sa * (s.x - shift * yc.x), sa * (s.y - shift * yc.y)};
  if (sb != 0.0) {
    const zc yo = Yold[row + (long)col * ldyo];
    out.x -= sb * yo.x;
    out.y -= sb * yo.y;
  }
  Yout[row + (long)col * ldyout] = out;
}

// Resident workgroup slots of the device (CUs x 4), cached per device.
int device_slots(int per_cu = 4) {
  static std::atomic<int> cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev] = cus;
  }
  return per_cu * cache[dev];
}

// Split count for a launch of `tiles` output tiles with inner size K, run by
// a kernel with per_cu resident workgroups per CU: the smallest split
// (<= max_splits, chunks >= 1024) whose workgroup count fills the resident
// slots to at least `enough`, else the best one.
int wave_splits(int tiles, int K, int max_splits, double enough, int per_cu) {
  const int slots = device_slots(per_cu);
  int best = 1;
  double best_u = 0.0;
  for (int s = 1; s <= max_splits; ++s) {
    if (s > 1 && K / s < 1024) break;
    const long wg = (long)tiles * s;
    const long waves = (wg + slots - 1) / slots;
    const double u = (double)wg / (double)(waves * slots);
    if (u >= enough) return s;
    if (u > best_u + 1e-9) {
      best_u = u;
      best = s;
    }
  }
  return best;
}

struct Plan {
  int tiles_m, tiles_n, total, splits, kchunk;
};

Plan make_plan(int M, int N, int K, bool lower_only, bool allow_split) {
  Plan p;
  p.tiles_m = (M + BM - 1) / BM;
  p.tiles_n = (N + BN - 1) / BN;
  p.total = lower_only ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  p.splits = 1;
  p.kchunk = ((K + BK - 1) / BK) * BK;
  if (allow_split && p.total < 512 && K >= 1024) {
    int want = (1024 + p.total - 1) / p.total;
    int maxs = K / 256;
    int s = want < maxs ? want : maxs;
    if (s > 1) {
      int chunk = (K + s - 1) / s;
      chunk = ((chunk + BK - 1) / BK) * BK;
      p.kchunk = chunk;
      p.splits = (K + chunk - 1) / chunk;
    }
  } else if (allow_split && !lower_only && K >= 4096) {
    // long products (H Q of Rayleigh-Ritz): split K, as the filter step
    // does, when the last round of resident workgroups would be far from
    // full
    const int s = wave_splits(p.total, K, 4, 0.97, 4);
    if (s > 1) {
      int chunk = (K + s - 1) / s;
      chunk = ((chunk + BK - 1) / BK) * BK;
      p.kchunk = chunk;
      p.splits = (K + chunk - 1) / chunk;
    }
  }
  return p;
}

template <int OPA, int OPB, int EPI, int KB = BK, int CM = 4>
int launch(hipStream_t s, GemmArgs& g) {
  int grid;
  if (g.lower_only && g.splits == 1) {
    grid = lower_xcd_grid(g.tiles_m);
  } else if (g.lower_only) {
    grid = g.total_tiles * g.splits;
  } else {
    const int vrows = g.splits * g.tiles_m;
    grid = ((vrows + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
  }
  // rows whose K range is longest first (triangular A with the long rows at
  // the bottom), so the tail of the launch is made of short tiles
  g.rows_desc = (g.ktri == KTRI_A_LOWER || g.ktri == KTRI_A_LOWER_B_UPPER) ? 1 : 0;
  hipLaunchKernelGGL((zgemm_kernel<OPA, OPB, EPI, KB, CM>), dim3(grid), dim3(NT), 0, s, g);
  return (int)hipGetLastError();
}

template <int EPI, int CM, int OPB = OP_N>
int launch_dma(hipStream_t s, GemmArgs& g);

template <int EPI, int CM>
int launch_dma_lower(hipStream_t s, GemmArgs& g) {
  hipLaunchKernelGGL((zgemm_dma_lower_kernel<EPI, CM>), dim3(lower_xcd_grid(g.tiles_m)), dim3(NT),
                     0, s, g);
  return (int)hipGetLastError();
}

template <int EPI, int CM>
int dispatch_cm(hipStream_t s, Op opa, Op opb, GemmArgs& g) {
  if (opa == OP_N && opb == OP_N) return launch<OP_N, OP_N, EPI, BK, CM>(s, g);
  if (opa == OP_N && opb == OP_C) return launch<OP_N, OP_C, EPI, BK, CM>(s, g);
  if (opa == OP_C && opb == OP_N) return launch<OP_C, OP_N, EPI, BK, CM>(s, g);
  return launch<OP_C, OP_C, EPI, BK, CM>(s, g);
}

// General products: the 3M split for products with a long inner dimension
// (25 % fewer MFMAs; measured 1.2x faster on filter-sized products), on the
// direct-to-LDS tile where op(A) = A (rectangular products with op(B) = B
// or B^H, and unsplit lower-triangle ones).  Lower-triangle products with
// a transposed operand are the Gram and Cholesky-update products (X^H X,
// Q^H Z, A21 A21^H): they keep the 4M split, a small share of the time on
// which the accuracy of CholeskyQR and of the B factor rests (3M's error
// bound on the imaginary part is the larger one).  The reduction's
// products (Linv T, lower triangle, and M Linv^H) take 3M.
template <int EPI>
int dispatch(hipStream_t s, Op opa, Op opb, GemmArgs& g) {
  const bool gram = g.lower_only && (opa != OP_N || opb != OP_N);
  if (!gram && g.K >= GENERAL_3M_MIN_K) {
    if (opa == OP_N && !g.lower_only)
      return opb == OP_N ? launch_dma<EPI, 3, OP_N>(s, g) : launch_dma<EPI, 3, OP_C>(s, g);
    if (opa == OP_N && opb == OP_N && g.splits == 1) return launch_dma_lower<EPI, 3>(s, g);
    return dispatch_cm<EPI, 3>(s, opa, opb, g);
  }
  return dispatch_cm<EPI, 4>(s, opa, opb, g);
}

// Filter tile autotuner: measured (n, N) launch shapes and the faster
// K-stage depth for each, per device.  A launch takes the choice of the
// nearest measured shape (log distance); with no measurement, KB = 8.
struct TuneEntry {
  int n, N, variant;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune[64];

int current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  return dev;
}

// Variant 2 (wide tiles) exists for the unsplit filter step only.
int launch_cheb_wide(hipStream_t s, const GemmArgs& g0) {
  GemmArgs g = g0;
  g.tiles_m = (g.M + WBM - 1) / WBM;
  g.tiles_n = (g.N + WBN - 1) / WBN;
  const int grid = ((g.tiles_m + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
  hipLaunchKernelGGL(cheb_wide_kernel, dim3(grid), dim3(WNT), 0, s, g);
  return (int)hipGetLastError();
}

// Direct-to-LDS tiles (op(A) = A; op(B) = B or B^H): rectangular tile sets.
template <int EPI, int CM, int OPB>
int launch_dma(hipStream_t s, GemmArgs& g) {
  const int vrows = g.splits * g.tiles_m;
  const int grid = ((vrows + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
  g.rows_desc = (g.ktri == KTRI_A_LOWER || g.ktri == KTRI_A_LOWER_B_UPPER) ? 1 : 0;
  hipLaunchKernelGGL((zgemm_dma_kernel<EPI, CM, OPB>), dim3(grid), dim3(NT), 0, s, g);
  return (int)hipGetLastError();
}

// Variants of the filter step: 0 / 1 the 64 x 64 tile with the 4M split,
// K staged 8 / 16 deep through registers; 2 the wide tile (4M); 3 / 4 as
// 0 / 1 with the 3M split; 5 / 6 the direct-to-LDS tile with the 3M / 4M
// split.  A split-K step has no wide form and takes 0 for 2.
template <int EPI>
int launch_cheb_variant(hipStream_t s, GemmArgs& g, int variant) {
  if (variant == 2 && EPI == EPI_CHEB && g.splits == 1) return launch_cheb_wide(s, g);
  if (variant == 1) return launch<OP_N, OP_N, EPI, 16, 4>(s, g);
  if (variant == 3) return launch<OP_N, OP_N, EPI, 8, 3>(s, g);
  if (variant == 4) return launch<OP_N, OP_N, EPI, 16, 3>(s, g);
  if (variant == 5) return launch_dma<EPI, 3>(s, g);
  if (variant == 6) return launch_dma<EPI, 4>(s, g);
  return launch<OP_N, OP_N, EPI, 8, 4>(s, g);
}

// Variant 2 needs a window of at least this many columns.
constexpr int WIDE_MIN_N = 256;


}  // namespace

int filter_variant(int n, int N) {
  const int dev = current_device();
  if (dev < 0) return DEFAULT_FILTER_VARIANT;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const auto& t = g_tune[dev];
  int best = DEFAULT_FILTER_VARIANT;
  double bd = 1e300;
  for (const auto& e : t) {
    const double a = std::log((double)n / e.n), b = std::log((double)N / e.N);
    const double d = a * a + b * b;
    if (d < bd) {
      bd = d;
      best = e.variant;
    }
  }
  if (best == 2 && N < WIDE_MIN_N) best = DEFAULT_FILTER_VARIANT;
  return best;
}

void tune_set(int n, int N, int variant) {
  const int dev = current_device();
  if (dev < 0) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto& t = g_tune[dev];
  for (auto& e : t)
    if (e.n == n && e.N == N) {
      e.variant = variant;
      return;
    }
  t.push_back({n, N, variant});
}

void tune_reset() {
  const int dev = current_device();
  if (dev < 0) return;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[dev].clear();
}

int tune_filter_shape(hipStream_t s, int n, int N, const zc* H, zc* Y0, zc* Y1, int* variant,
                      double tf[FILTER_VARIANTS]) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return (int)hipErrorUnknown;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return (int)hipErrorUnknown;
  }
  Plan p = make_plan(n, N, n, false, false);
  GemmArgs g = {};
  g.M = n; g.N = N; g.K = n;
  g.A = H; g.lda = n; g.B = Y0; g.ldb = n; g.C = Y1; g.ldc = n;
  g.Ycur = Y0; g.ldyc = n; g.Yold = Y1; g.ldyo = n;
  g.shift = 0.25; g.sa = 1e-3; g.sb = 0.5;
  g.tiles_m = p.tiles_m; g.tiles_n = p.tiles_n; g.total_tiles = p.total;
  g.splits = 1; g.kchunk = p.kchunk;
  // rounds alternate the variants (two launches each); the best round of
  // each counts
  const int rounds = 4, reps = 2;
  const bool wide_ok = N >= WIDE_MIN_N;
  float best[FILTER_VARIANTS];
  for (int v = 0; v < FILTER_VARIANTS; ++v) best[v] = 1e30f;
  int err = 0;
  for (int v = 0; v < FILTER_VARIANTS && !err; ++v)
    if (v != 2 || wide_ok) err = launch_cheb_variant<EPI_CHEB>(s, g, v);
  for (int r = 0; r < rounds && !err; ++r) {
    for (int v = 0; v < FILTER_VARIANTS && !err; ++v) {
      if (v == 2 && !wide_ok) continue;
      err = (int)hipEventRecord(e0, s);
      for (int i = 0; i < reps && !err; ++i) err = launch_cheb_variant<EPI_CHEB>(s, g, v);
      if (!err) err = (int)hipEventRecord(e1, s);
      if (!err) err = (int)hipEventSynchronize(e1);
      float ms = 0.f;
      if (!err) err = (int)hipEventElapsedTime(&ms, e0, e1);
      if (!err) best[v] = std::min(best[v], ms);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err) return err;
  // complex-equivalent rate (8 real flops per complex multiply-add, also
  // for the 3M variants, which execute 6)
  for (int v = 0; v < FILTER_VARIANTS; ++v)
    tf[v] = best[v] < 1e29f ? 8.0 * (double)n * n * N * reps / (1e-3 * best[v]) / 1e12 : 0.0;
  // another variant than the default only when clearly (2 %) faster
  constexpr int d = DEFAULT_FILTER_VARIANT;
  int pick = d;
  for (int v = 0; v < FILTER_VARIANTS; ++v)
    if (v != d && tf[v] > 1.02 * tf[d] && tf[v] > tf[pick]) pick = v;
  *variant = pick;
  tune_set(n, N, *variant);
  return 0;
}

size_t zgemm_work_elems(int M, int N, int K) {
  Plan p = make_plan(M, N, K, false, true);
  return p.splits > 1 ? (size_t)p.splits * M * N : 0;
}

int zgemm(hipStream_t s, Op opa, Op opb, int M, int N, int K, zc alpha, const zc* A, long lda,
          const zc* B, long ldb, zc beta, zc* C, long ldc, bool lower_only, zc* work,
          size_t work_elems, int ktri) {
  if (M <= 0 || N <= 0) return 0;
  if (lower_only && M != N) return (int)hipErrorInvalidValue;
  Plan p = make_plan(M, N, K, lower_only, work != nullptr);
  if (p.splits > 1 && (size_t)p.splits * M * N > work_elems) {
    p = make_plan(M, N, K, lower_only, false);
  }
  GemmArgs g = {};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta;
  g.splits = p.splits; g.kchunk = p.kchunk; g.part = work;
  g.tiles_m = p.tiles_m; g.tiles_n = p.tiles_n; g.lower_only = lower_only ? 1 : 0;
  g.total_tiles = p.total;
  g.ktri = ktri;
  if (K <= 0) {
    // C = beta C: run a single k-empty pass through the store epilogue
    g.splits = 1; g.kchunk = BK; g.K = 0;
    return dispatch<EPI_STORE>(s, opa, opb, g);
  }
  if (p.splits == 1) return dispatch<EPI_STORE>(s, opa, opb, g);
  int err = dispatch<EPI_PARTIAL>(s, opa, opb, g);
  if (err) return err;
  const long total = (long)M * N;
  const int threads = 256;
  hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)((total + threads - 1) / threads)),
                     dim3(threads), 0, s, M, N, p.splits, (const zc*)work, alpha, beta, C, ldc,
                     g.lower_only);
  return (int)hipGetLastError();
}

GemmArgs cheb_group_args(int n, int N, const zc* H, long ldh, const zc* Ycur, long ldyc,
                         const zc* Yold, long ldyo, zc* Yout, long ldyout, double shift, double sa,
                         double sb, int* slots) {
  Plan p = make_plan(n, N, n, false, false);
  GemmArgs g = {};
  g.M = n; g.N = N; g.K = n;
  g.A = H; g.lda = ldh; g.B = Ycur; g.ldb = ldyc; g.C = Yout; g.ldc = ldyout;
  g.Ycur = Ycur; g.ldyc = ldyc; g.Yold = Yold; g.ldyo = ldyo;
  g.shift = shift; g.sa = sa; g.sb = sb;
  g.tiles_m = p.tiles_m; g.tiles_n = p.tiles_n; g.total_tiles = p.total;
  g.splits = 1;
  g.kchunk = p.kchunk;
  *slots = ((p.tiles_m + NXCD - 1) / NXCD) * p.tiles_n * NXCD;
  return g;
}

int cheb_step_group(hipStream_t s, const GemmArgs* list, const int* slot_begin, int count,
                    int total_slots, int variant) {
  if (count <= 0 || total_slots <= 0) return 0;
  // (the wide variant has no grouped form: the default instead)
  if (variant == 2) variant = DEFAULT_FILTER_VARIANT;
  if (variant == 1)
    hipLaunchKernelGGL((zgemm_group_cheb<16, 4>), dim3(total_slots), dim3(NT), 0, s, list,
                       slot_begin, count);
  else if (variant == 3)
    hipLaunchKernelGGL((zgemm_group_cheb<8, 3>), dim3(total_slots), dim3(NT), 0, s, list,
                       slot_begin, count);
  else if (variant == 4)
    hipLaunchKernelGGL((zgemm_group_cheb<16, 3>), dim3(total_slots), dim3(NT), 0, s, list,
                       slot_begin, count);
  else if (variant == 5)
    hipLaunchKernelGGL((zgemm_group_cheb_dma<3>), dim3(total_slots), dim3(NT), 0, s, list,
                       slot_begin, count);
  else if (variant == 6)
    hipLaunchKernelGGL((zgemm_group_cheb_dma<4>), dim3(total_slots), dim3(NT), 0, s, list,
                       slot_begin, count);
  else
    hipLaunchKernelGGL((zgemm_group_cheb<8, 4>), dim3(total_slots), dim3(NT), 0, s, list,
                       slot_begin, count);
  return (int)hipGetLastError();
}

int cheb_step(hipStream_t s, int n, int N, const zc* H, long ldh, const zc* Ycur, long ldyc,
              const zc* Yold, long ldyo, zc* Yout, long ldyout, double shift, double sa,
              double sb, zc* part, size_t part_elems) {
  if (N <= 0) return 0;
  Plan p = make_plan(n, N, n, false, false);
  GemmArgs g = {};
  g.M = n; g.N = N; g.K = n;
  g.A = H; g.lda = ldh; g.B = Ycur; g.ldb = ldyc; g.C = Yout; g.ldc = ldyout;
  g.Ycur = Ycur; g.ldyc = ldyc; g.Yold = Yold; g.ldyo = ldyo;
  g.shift = shift; g.sa = sa; g.sb = sb;
  g.tiles_m = p.tiles_m; g.tiles_n = p.tiles_n; g.total_tiles = p.total;
  const int variant = filter_variant(n, N);
  int splits = 1;
  if (part != nullptr) {
    const int max_s = (int)std::min<size_t>(CHEB_MAX_SPLITS, part_elems / ((size_t)n * N));
    // a filter step is long (up to 0.2 s at n = 30 000): split K until the
    // last round of four workgroups per CU is nearly full.  At n = 30 000
    // and 1800 columns (13 601 tiles) one launch of the 4M tile leaves 5 %
    // of the slot time idle in its last round and two splits 1.6 %
    // (measured 1.3 % faster); the 3M tiles, three per CU, would fill 98 %
    // of their last round unsplit, yet run 1.8 % faster with the two splits
    // as well (85.8 against 84.3 TFLOP/s): counting four slots per CU for
    // every variant matched the measurements best.
    if (max_s > 1) splits = wave_splits(p.total, n, max_s, 0.97, 4);
  }
  if (splits == 1) {
    g.splits = 1;
    g.kchunk = p.kchunk;
    return launch_cheb_variant<EPI_CHEB>(s, g, variant);
  }
  int chunk = (n + splits - 1) / splits;
  chunk = ((chunk + BK - 1) / BK) * BK;
  g.kchunk = chunk;
  g.splits = (n + chunk - 1) / chunk;
  g.part = part;
  int err = launch_cheb_variant<EPI_PARTIAL_CHEB>(s, g, variant);
  if (err) return err;
  const long total = (long)n * N;
  hipLaunchKernelGGL(cheb_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, n, N,
                     g.splits, (const zc*)part, Ycur, ldyc, Yold, ldyo, Yout, ldyout, shift, sa,
                     sb);
  return (int)hipGetLastError();
}

}  // namespace chfsi
