// BF16-split form of the defect step of the mixed-precision Chebyshev
// filter, on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.
//
// The defect recurrence (the FP32 form is described in cfilter32.hip)
//   E_{i+1} = 2 sigma_{i+1} (Ht E_i + R diag(p_i(mu_t)) / e) - sigma_{i+1} sigma_i E_{i-1}
// keeps E in FP32 between steps.  Here the product H E_i is formed from
// two-term BF16 splits of both operands: x = x_hi + x_lo with
// x_hi = bf16(x) and x_lo = bf16(x - x_hi), both rounded to nearest even,
// and a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi (three BF16 products into one
// FP32 accumulator).  The dropped terms (a_lo b_lo and the parts of a and b
// beyond the two BF16 words) are at most about 3 * 2^-16 |a| |b|, so the
// step's error is that fraction of |H| |E_i|: like the FP32 step it scales
// with the residuals, 2^8 times coarser.  A step of the filter may use this
// form when its error, damped by the steps after it (eq. resl), stays
// far below what the filter aims at (the solver's schedule decides per
// step).  BF16 keeps the exponent range of FP32, so the splits need no
// per-column scaling: every defect column here is many orders of magnitude
// above the smallest normal FP32 number.
//
// Operand layout ("split panel"): a complex matrix is stored as rows r of a
// reduction index k padded to Kp (a multiple of 32, zero filled); row r
// holds Kp / 8 groups of 64 bytes, group g = the four planes re_hi, im_hi,
// re_lo, im_lo of k = 8g .. 8g + 7, 8 BF16 each.  H is stored by its rows
// (r = m, k = column of H); E_i by its columns (r = column, k = row).  One
// 16-byte LDS read then gives an MFMA lane its 8 consecutive k of a plane.
//
// FP16 form (v_mfma_f32_16x16x32_f16): the same two-word split with FP16
// words, x_hi = fp16(x), x_lo = fp16(x - x_hi), 11 significant bits each,
// so the dropped terms are at most about 3 * 2^-22 |a| |b| -- close to the
// rounding of the FP32 step itself, at the BF16 step's cost.  FP16 has a
// narrow exponent range, so the operands are scaled by powers of two first:
// H by one factor, each column of E_i by its own, both chosen from the
// largest magnitude so that it lands in [2^14, 2^15); the epilogue undoes
// the scaling exactly.  Words that fall into FP16's subnormal range (hi
// words of entries 2^28, lo words of entries 2^17 below the largest one)
// keep an absolute error of at most 2^-25 of the scaled unit, 2^-39 of the
// largest magnitude, which adds at most n 2^-39 max|H| max|E_i[:, j]| to an
// element of column j of the product.
#include "internal.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>

namespace chfsi {

namespace {

typedef float2 cf;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 hf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int SBK = 32;                        // K per LDS stage
constexpr int SPLIT_WIDE_MIN_N = 257;          // windows that take the 128 x 128 tile
constexpr int GROUP_B = 64;                    // bytes per (row, 8 k) group
constexpr int ROWB = (SBK / 8) * GROUP_B;      // LDS bytes per tile row and stage
constexpr int NXCD = 8;

__device__ __forceinline__ unsigned bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float bf16_val(unsigned h) { return __uint_as_float(h << 16); }

// hi and lo BF16 words of x
__device__ __forceinline__ void split1(float x, unsigned& hi, unsigned& lo) {
  hi = bf16_rne(x);
  lo = bf16_rne(x - bf16_val(hi));
}

// hi and lo FP16 words of x (round to nearest even; x - hi is exact in FP32)
__device__ __forceinline__ void split1h(float x, unsigned& hi, unsigned& lo) {
  const _Float16 h = (_Float16)x;
  const _Float16 l = (_Float16)(x - (float)h);
  hi = __builtin_bit_cast(unsigned short, h);
  lo = __builtin_bit_cast(unsigned short, l);
}

// the four planes of 8 complex values -> 4 x 16 bytes (FP16 words when H16,
// after scaling by sc)
template <bool H16 = false>
__device__ __forceinline__ void split8(const cf* v, uint4* planes, float sc = 1.f) {
  unsigned rh[8], ih[8], rl[8], il[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if constexpr (H16) {
      split1h(v[i].x * sc, rh[i], rl[i]);
      split1h(v[i].y * sc, ih[i], il[i]);
    } else {
      split1(v[i].x, rh[i], rl[i]);
      split1(v[i].y, ih[i], il[i]);
    }
  }
  auto pack = [](const unsigned* w) {
    return uint4{w[0] | (w[1] << 16), w[2] | (w[3] << 16), w[4] | (w[5] << 16),
                 w[6] | (w[7] << 16)};
  };
  planes[0] = pack(rh);
  planes[1] = pack(ih);
  planes[2] = pack(rl);
  planes[3] = pack(il);
}


// operand words and matrix instruction of the two forms
template <bool H16>
struct Words;
template <>
struct Words<false> {
  typedef bf8 V;
  static __device__ __forceinline__ V cast(uint4 v) { return __builtin_bit_cast(bf8, v); }
  static __device__ __forceinline__ f4 mma(const V& a, const V& b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Words<true> {
  typedef hf8 V;
  static __device__ __forceinline__ V cast(uint4 v) { return __builtin_bit_cast(hf8, v); }
  static __device__ __forceinline__ f4 mma(const V& a, const V& b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// sign flip of 8 BF16 or FP16 words (bit 15 of each half)
__device__ __forceinline__ uint4 neg_bf16(uint4 v) {
  const unsigned s = 0x80008000u;
  return uint4{v.x ^ s, v.y ^ s, v.z ^ s, v.w ^ s};
}

struct SplitArgs {
  int M, N, Kp;
  const char* As; long a_row;   // split panel of H (rows m), bytes per row
  const char* Bs; long b_row;   // split panel of E_i (rows = columns of the window)
  const cf* Ecur; long lde;     // E_i in FP32
  const cf* Eold;               // E_{i-1}
  cf* Eout;                     // E_{i+1} (may alias Eold)
  const cf* R; long ldr;        // residual block (FP32)
  const float* cr;              // per-column coefficient of R
  float shift, sa, sb;
  char* Bnext;                  // split panel of E_{i+1} (same geometry as Bs) or null
  float inv_a;                  // FP16 form: 1 / (scale of H)
  const float* inv_b;           // FP16 form: 1 / (scale of each window column)
  int tiles_m, tiles_n;
  int splits, kstages;          // split-K: K stages per split (splits = 1: none)
  cf* part;                     // split-K partials: part[s * M * N + i + j * M]
};

// One defect step on tiles of BM x BN complex outputs: WGM x WGN waves, each
// owning TI x TJ sub-tiles of 16 x 16 (BM = 16 WGM TI, BN = 16 WGN TJ), K
// staged 32 deep through two LDS stages of (BM + BN) rows x 256 B; tile rows
// interleaved over the 8 XCDs.  The operand rows go from global memory
// straight to LDS (global_load_lds_dwordx4: one instruction of a wave fills
// 1 KB, 4 tile rows, lane L taking 16 B of row L / 16), so no registers hold
// staged data and the next stage's loads run under the current stage's
// MFMAs.  The 16-byte chunks of LDS row r sit at position chunk ^ (r & 15):
// the fragment reads of 16 consecutive rows then touch 16 distinct chunk
// positions, all 64 banks once.  Instances: 64 x 64 with 4 waves of 32 x 32
// (64 KB of LDS, two workgroups per CU) and 128 x 128 with 8 waves of 32 x
// 64 (128 KB, one per CU: half the operand traffic per output and a third
// fewer LDS reads per MFMA).
template <int WGM, int WGN, int TI, int TJ>
struct SplitTile {
  static constexpr int BM = 16 * WGM * TI, BN = 16 * WGN * TJ;
  static constexpr int NTH = 64 * WGM * WGN;
  static constexpr int LDS_STAGE = (BM + BN) * ROWB;
  static constexpr int BLOCKS = (BM + BN) / 4;       // 1 KB blocks per stage
  static constexpr int PER_WAVE = BLOCKS / (NTH / 64);
  static_assert(BLOCKS % (NTH / 64) == 0, "whole blocks per wave");
};

template <int WGM, int WGN, int TI, int TJ, bool H16>
__device__ __forceinline__ void split_tile_body(const SplitArgs& g, char* lds0, char* lds1,
                                                int bid) {
  using W = Words<H16>;
  typedef typename W::V V;
  using T = SplitTile<WGM, WGN, TI, TJ>;
  constexpr int BM = T::BM, NW = T::NTH / 64, PW = T::PER_WAVE;
  // virtual tile rows (split, tile row) interleaved over the XCDs
  const int xcd = bid % NXCD, slot = bid / NXCD;
  const int vrows = g.splits * g.tiles_m;
  const int rows_x = (vrows - xcd + NXCD - 1) / NXCD;
  const int ri = slot / g.tiles_n;
  const int tn = slot - ri * g.tiles_n;
  if (ri >= rows_x) return;
  const int v = xcd + NXCD * ri;
  const int split = v / g.tiles_m, tm = v - split * g.tiles_m;
  const int m0 = tm * BM, n0 = tn * T::BN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int lr = lane & 15, lg = lane >> 4;

  f4 accR[TI][TJ], accI[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      accR[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  // this lane's source in each of the wave's 1 KB blocks: tile row
  // 4 b + lane / 16 (A rows first, then B rows), the chunk that belongs at
  // position lane % 16; rows beyond M or N read a valid row instead (their
  // products only reach outputs that are not stored)
  const char* src[PW];
#pragma unroll
  for (int i = 0; i < PW; ++i) {
    const int b = i * NW + wave;
    const int row = 4 * b + (lane >> 4);
    const int chunk = (lane & 15) ^ (row & 15);
    if (row < BM)
      src[i] = g.As + (long)min(m0 + row, g.M - 1) * g.a_row + chunk * 16;
    else
      src[i] = g.Bs + (long)min(n0 + row - BM, g.N - 1) * g.b_row + chunk * 16;
  }
  auto load = [&](int k0, char* buf) {
#pragma unroll
    for (int i = 0; i < PW; ++i)
      __builtin_amdgcn_global_load_lds(
          (const void*)(src[i] + (long)k0 * 8),
          (__attribute__((address_space(3))) void*)(buf + (i * NW + wave) * 1024), 16, 0, 0);
  };
  auto compute = [&](const char* la) {
    const char* lb = la + BM * ROWB;
    uint4 a[TI][4], b[TJ][4];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const int r = wm * 16 * TI + i * 16 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        a[i][q] = *(const uint4*)(la + r * ROWB + (((lg * 4 + q) ^ (r & 15)) * 16));
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int r = wn * 16 * TJ + j * 16 + lr;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        b[j][q] = *(const uint4*)(lb + r * ROWB + (((lg * 4 + q) ^ (r & 15)) * 16));
    }
    // planes: 0 re_hi, 1 im_hi, 2 re_lo, 3 im_lo
    // real part: Ar Br - Ai Bi (the A imaginary planes negated)
    // imaginary part: Ar Bi + Ai Br
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const V arh = W::cast(a[i][0]), arl = W::cast(a[i][2]);
      const V aih = W::cast(a[i][1]), ail = W::cast(a[i][3]);
      const V nih = W::cast(neg_bf16(a[i][1])), nil = W::cast(neg_bf16(a[i][3]));
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const V brh = W::cast(b[j][0]), brl = W::cast(b[j][2]);
        const V bih = W::cast(b[j][1]), bil = W::cast(b[j][3]);
        accR[i][j] = W::mma(arh, brh, accR[i][j]);
        accI[i][j] = W::mma(arh, bih, accI[i][j]);
        accR[i][j] = W::mma(nih, bih, accR[i][j]);
        accI[i][j] = W::mma(aih, brh, accI[i][j]);
        accR[i][j] = W::mma(arh, brl, accR[i][j]);
        accI[i][j] = W::mma(arh, bil, accI[i][j]);
        accR[i][j] = W::mma(nih, bil, accR[i][j]);
        accI[i][j] = W::mma(aih, brl, accI[i][j]);
        accR[i][j] = W::mma(arl, brh, accR[i][j]);
        accI[i][j] = W::mma(arl, bih, accI[i][j]);
        accR[i][j] = W::mma(nil, bih, accR[i][j]);
        accI[i][j] = W::mma(ail, brh, accI[i][j]);
      }
    }
  };
  // two LDS stages used alternately (the loop is unrolled by two so that
  // each stage's buffer is fixed); every stage ends with this wave's loads
  // landed and a barrier, so the other buffer is free for the next loads
  const int kt0 = split * g.kstages;
  const int nk = min(g.Kp / SBK, kt0 + g.kstages) - kt0;
  if (nk > 0) load(kt0 * SBK, lds0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    if (kt + 1 < nk) load((kt0 + kt + 1) * SBK, lds1);
    compute(lds0);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (kt + 1 >= nk) break;
    if (kt + 2 < nk) load((kt0 + kt + 2) * SBK, lds0);
    compute(lds1);
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
  }
  // MFMA output: lane l, register r holds row 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int rbase = m0 + wm * 16 * TI + i * 16 + 4 * lg;
      const int col = n0 + wn * 16 * TJ + j * 16 + lr;
      if (col >= g.N) continue;
      float unscale = 1.f;   // FP16 form: undo the operand scaling (powers of two)
      if constexpr (H16) unscale = g.inv_a * g.inv_b[col];
      if (g.splits > 1) {    // split-K: unscaled partial sums, epilogue in the reduction
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rbase + r;
          if (row < g.M)
            g.part[(long)split * g.M * g.N + row + (long)col * g.M] =
                cf{accR[i][j][r] * unscale, accI[i][j][r] * unscale};
        }
        continue;
      }
      cf out[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rbase + r;
        out[r] = cf{0.f, 0.f};
        if (row >= g.M) continue;
        const cf ec = g.Ecur[row + (long)col * g.lde];
        const cf rr = g.R[row + (long)col * g.ldr];
        const float crj = g.cr[col];
        float pr = accR[i][j][r], pi = accI[i][j][r];
        if constexpr (H16) {
          pr *= unscale;
          pi *= unscale;
        }
        cf o = cf{g.sa * (pr - g.shift * ec.x) + crj * rr.x,
                  g.sa * (pi - g.shift * ec.y) + crj * rr.y};
        if (g.sb != 0.f) {
          const cf eo = g.Eold[row + (long)col * g.lde];
          o.x -= g.sb * eo.x;
          o.y -= g.sb * eo.y;
        }
        g.Eout[row + (long)col * g.lde] = o;
        out[r] = o;
      }
      // the split of E_{i+1} for a following BF16 step: 4 consecutive k of
      // column col, zeros beyond M (inside the padding); the FP16 form
      // needs the column's scale first and splits in a pass of its own
      if (!H16 && g.Bnext && rbase < g.Kp) {
        unsigned rh[4], ih[4], rl[4], il[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          split1(out[r].x, rh[r], rl[r]);
          split1(out[r].y, ih[r], il[r]);
        }
        char* p = g.Bnext + col * g.b_row + (rbase >> 3) * GROUP_B + (rbase & 7) * 2;
        *(uint2*)(p + 0) = uint2{rh[0] | (rh[1] << 16), rh[2] | (rh[3] << 16)};
        *(uint2*)(p + 16) = uint2{ih[0] | (ih[1] << 16), ih[2] | (ih[3] << 16)};
        *(uint2*)(p + 32) = uint2{rl[0] | (rl[1] << 16), rl[2] | (rl[3] << 16)};
        *(uint2*)(p + 48) = uint2{il[0] | (il[1] << 16), il[2] | (il[3] << 16)};
      }
    }
}

using TileSmall = SplitTile<2, 2, 2, 2>;   // 64 x 64, 256 threads
using TileWide = SplitTile<4, 2, 2, 4>;    // 128 x 128, 512 threads

__global__ void __launch_bounds__(TileSmall::NTH, 2) defect_gemm_split(SplitArgs g) {
  __shared__ __attribute__((aligned(1024))) char lds0[TileSmall::LDS_STAGE];
  __shared__ __attribute__((aligned(1024))) char lds1[TileSmall::LDS_STAGE];
  split_tile_body<2, 2, 2, 2, false>(g, lds0, lds1, blockIdx.x);
}

__global__ void __launch_bounds__(TileWide::NTH, 1) defect_gemm_split_wide(SplitArgs g) {
  __shared__ __attribute__((aligned(1024))) char lds0[TileWide::LDS_STAGE];
  __shared__ __attribute__((aligned(1024))) char lds1[TileWide::LDS_STAGE];
  split_tile_body<4, 2, 2, 4, false>(g, lds0, lds1, blockIdx.x);
}

__global__ void __launch_bounds__(TileSmall::NTH, 2) defect_gemm_h16(SplitArgs g) {
  __shared__ __attribute__((aligned(1024))) char lds0[TileSmall::LDS_STAGE];
  __shared__ __attribute__((aligned(1024))) char lds1[TileSmall::LDS_STAGE];
  split_tile_body<2, 2, 2, 2, true>(g, lds0, lds1, blockIdx.x);
}

__global__ void __launch_bounds__(TileWide::NTH, 1) defect_gemm_h16_wide(SplitArgs g) {
  __shared__ __attribute__((aligned(1024))) char lds0[TileWide::LDS_STAGE];
  __shared__ __attribute__((aligned(1024))) char lds1[TileWide::LDS_STAGE];
  split_tile_body<4, 2, 2, 4, true>(g, lds0, lds1, blockIdx.x);
}

// Grouped launches (batches of independent problems): problem p of the
// list owns the workgroups [slot_begin[p], slot_begin[p+1]), a multiple of
// 8, so that the XCD interleaving inside each range is that of a launch of
// its own; a binary search over slot_begin maps a workgroup to its problem.
__device__ __forceinline__ int group_of(const int* slot_begin, int count, int b) {
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (slot_begin[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

template <bool H16>
__global__ void __launch_bounds__(TileSmall::NTH, 2) defect_group_small(const SplitArgs* list,
                                                                      const int* slot_begin,
                                                                      int count) {
  __shared__ __attribute__((aligned(1024))) char lds0[TileSmall::LDS_STAGE];
  __shared__ __attribute__((aligned(1024))) char lds1[TileSmall::LDS_STAGE];
  const int p = group_of(slot_begin, count, blockIdx.x);
  split_tile_body<2, 2, 2, 2, H16>(list[p], lds0, lds1, blockIdx.x - slot_begin[p]);
}

template <bool H16>
__global__ void __launch_bounds__(TileWide::NTH, 1) defect_group_wide(const SplitArgs* list,
                                                                    const int* slot_begin,
                                                                    int count) {
  __shared__ __attribute__((aligned(1024))) char lds0[TileWide::LDS_STAGE];
  __shared__ __attribute__((aligned(1024))) char lds1[TileWide::LDS_STAGE];
  const int p = group_of(slot_begin, count, blockIdx.x);
  split_tile_body<4, 2, 2, 4, H16>(list[p], lds0, lds1, blockIdx.x - slot_begin[p]);
}

// Power-of-two scale that brings the largest magnitude m into [2^14, 2^15)
// (1 for m = 0; capped at 2^100 so that its inverse stays a normal number).
__device__ __forceinline__ int h16_scale_exp(float m) {
  if (!(m > 0.f) || !isfinite(m)) return 0;
  return min(14 - ilogbf(m), 100);
}

// FP16 split panel of FP32 columns, each scaled by its own power of two:
// one workgroup (256 threads) per column; inv[j] receives 1 / scale.
__device__ __forceinline__ void split_col_h16_body(int K, int Kp, const cf* E, long lde, char* S,
                                                   long srow, float* inv, int j, float* red) {
  const int t = threadIdx.x;
  const cf* col = E + (long)j * lde;
  float m = 0.f;
  for (int r = t; r < K; r += 256) {
    const cf v = col[r];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  red[t] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmaxf(red[t], red[t + w]);
    __syncthreads();
  }
  const int ex = h16_scale_exp(red[0]);
  const float sc = ldexpf(1.f, ex);
  const int groups = Kp / 8;
  for (int grp = t; grp < groups; grp += 256) {
    cf v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = grp * 8 + i;
      v[i] = k < K ? col[k] : cf{0.f, 0.f};
    }
    uint4 pl[4];
    split8<true>(v, pl, sc);
    uint4* dst = (uint4*)(S + j * srow + (long)grp * GROUP_B);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = pl[q];
  }
  if (t == 0) inv[j] = ldexpf(1.f, -ex);
}

__global__ void __launch_bounds__(256) split_cols_h16(int K, int Kp, const cf* E, long lde,
                                                      char* S, long srow, float* inv) {
  __shared__ float red[256];
  split_col_h16_body(K, Kp, E, lde, S, srow, inv, blockIdx.x, red);
}

// Per-column split panels of several problems' windows in one launch: one
// workgroup per column, problem p owning the columns [col_begin[p],
// col_begin[p+1]).  FP16 words of scaled values (with inv) or BF16 words.
struct ColSplitArgs {
  int K, Kp;
  const cf* E; long lde;
  char* S; long srow;
  float* inv;
};

template <bool H16>
__global__ void __launch_bounds__(256) split_cols_group(const ColSplitArgs* list,
                                                        const int* col_begin, int count) {
  __shared__ float red[256];
  const int p = group_of(col_begin, count, blockIdx.x);
  const ColSplitArgs& a = list[p];
  const int j = blockIdx.x - col_begin[p];
  if constexpr (H16) {
    split_col_h16_body(a.K, a.Kp, a.E, a.lde, a.S, a.srow, a.inv, j, red);
  } else {
    const cf* col = a.E + (long)j * a.lde;
    for (int grp = threadIdx.x; grp < a.Kp / 8; grp += 256) {
      cf v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = grp * 8 + i;
        v[i] = k < a.K ? col[k] : cf{0.f, 0.f};
      }
      uint4 pl[4];
      split8(v, pl);
      uint4* dst = (uint4*)(a.S + j * a.srow + (long)grp * GROUP_B);
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[q] = pl[q];
    }
  }
}

// Largest |re|, |im| of count complex64 values: one partial per workgroup.
__global__ void __launch_bounds__(256) absmax_part(long count, const cf* X, float* part) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  float m = 0.f;
  for (long i = (long)blockIdx.x * 256 + t; i < count; i += (long)gridDim.x * 256) {
    const cf v = X[i];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  red[t] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmaxf(red[t], red[t + w]);
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = red[0];
}

// Split panel of FP32 columns: row j of S = column j of E (K values, zero
// padded to Kp).  One thread per (column, group of 8).
__global__ void split_cols(int K, int Kp, int cols, const cf* E, long lde, char* S, long srow) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int groups = Kp / 8;
  if (idx >= (long)groups * cols) return;
  const int j = (int)(idx / groups), grp = (int)(idx % groups);
  cf v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = grp * 8 + i;
    v[i] = k < K ? E[k + (long)j * lde] : cf{0.f, 0.f};
  }
  uint4 pl[4];
  split8(v, pl);
  uint4* dst = (uint4*)(S + j * srow + (long)grp * GROUP_B);
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[q] = pl[q];
}

// Split panel of the rows of an FP64 matrix: row m of S = H[m, :] (values
// rounded to FP32 first, as in the FP32 step), through a 32 x 64 LDS tile.
constexpr int TM = 32, TK = 64;
template <bool H16>
__global__ void split_rows(int n, int Kp, const zc* H, long ldh, char* S, long srow, float sc) {
  __shared__ cf tile[TK][TM + 1];
  const int m0 = blockIdx.x * TM, k0 = blockIdx.y * TK;
  const int t = threadIdx.x;
  // load: m fastest (a column of H is contiguous)
  for (int e = t; e < TM * TK; e += blockDim.x) {
    const int mm = e % TM, kk = e / TM;
    const int m = m0 + mm, k = k0 + kk;
    cf v = cf{0.f, 0.f};
    if (m < n && k < n) {
      const zc h = H[m + (long)k * ldh];
      v = cf{(float)h.x, (float)h.y};
    }
    tile[kk][mm] = v;
  }
  __syncthreads();
  // store: a thread per (row m, group of 8 k)
  for (int e = t; e < TM * (TK / 8); e += blockDim.x) {
    const int grp = e % (TK / 8), mm = e / (TK / 8);
    const int m = m0 + mm;
    const int kg = k0 + grp * 8;
    if (m >= n || kg >= Kp) continue;
    cf v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = tile[grp * 8 + i][mm];
    uint4 pl[4];
    split8<H16>(v, pl, sc);
    uint4* dst = (uint4*)(S + m * srow + (long)(kg / 8) * GROUP_B);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = pl[q];
  }
}

// Compute units of the current device (cached per device).
int split_device_cus() {
  static std::atomic<int> cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}

}  // namespace

int split_kp(int K) { return ((K + SBK - 1) / SBK) * SBK; }

size_t split_panel_bytes(int rows, int K) { return (size_t)rows * (size_t)split_kp(K) * 8; }

int matrix_to_split(hipStream_t s, int n, const zc* H, long ldh, void* Hs) {
  const int kp = split_kp(n);
  dim3 grid((unsigned)((n + TM - 1) / TM), (unsigned)((kp + TK - 1) / TK));
  hipLaunchKernelGGL(split_rows<false>, grid, dim3(256), 0, s, n, kp, H, ldh, (char*)Hs,
                     (long)kp * 8, 1.f);
  return (int)hipGetLastError();
}

int matrix_to_split_h16(hipStream_t s, int n, const zc* H, long ldh, const void* H32,
                        void* Hs, float* part, float* inv_out) {
  constexpr int PARTS = 1024;
  const long count = (long)n * n;
  const int blocks = (int)std::min<long>(PARTS, (count + 255) / 256);
  hipLaunchKernelGGL(absmax_part, dim3(blocks), dim3(256), 0, s, count, (const cf*)H32, part);
  int e = (int)hipGetLastError();
  if (e) return e;
  float hp[PARTS];
  e = (int)hipMemcpyAsync(hp, part, sizeof(float) * blocks, hipMemcpyDeviceToHost, s);
  if (e) return e;
  e = (int)hipStreamSynchronize(s);
  if (e) return e;
  float m = 0.f;
  for (int i = 0; i < blocks; ++i) m = std::max(m, hp[i]);
  int ex = 0;
  if (m > 0.f && std::isfinite(m)) ex = std::min(14 - std::ilogb(m), 100);
  const int kp = split_kp(n);
  dim3 grid((unsigned)((n + TM - 1) / TM), (unsigned)((kp + TK - 1) / TK));
  hipLaunchKernelGGL(split_rows<true>, grid, dim3(256), 0, s, n, kp, H, ldh, (char*)Hs,
                     (long)kp * 8, std::ldexp(1.f, ex));
  *inv_out = std::ldexp(1.f, -ex);
  return (int)hipGetLastError();
}

int cols_to_split_h16(hipStream_t s, int K, int cols, const void* E, long lde, void* S,
                      float* inv) {
  if (cols <= 0) return 0;
  const int kp = split_kp(K);
  hipLaunchKernelGGL(split_cols_h16, dim3((unsigned)cols), dim3(256), 0, s, K, kp, (const cf*)E,
                     lde, (char*)S, (long)kp * 8, inv);
  return (int)hipGetLastError();
}

int cols_to_split(hipStream_t s, int K, int cols, const void* E, long lde, void* S) {
  if (cols <= 0) return 0;
  const int kp = split_kp(K);
  const long total = (long)(kp / 8) * cols;
  hipLaunchKernelGGL(split_cols, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, K, kp,
                     cols, (const cf*)E, lde, (char*)S, (long)kp * 8);
  return (int)hipGetLastError();
}

int defect_step_split(hipStream_t s, int n, int N, const void* Hs, const void* Es,
                      const void* Ecur, const void* Eold, void* Eout, const void* R32,
                      const float* cr, float shift, float sa, float sb, void* Es_next) {
  if (N <= 0) return 0;
  SplitArgs g = {};
  g.M = n; g.N = N; g.Kp = split_kp(n);
  g.As = (const char*)Hs; g.a_row = (long)g.Kp * 8;
  g.Bs = (const char*)Es; g.b_row = (long)g.Kp * 8;
  g.Ecur = (const cf*)Ecur; g.Eold = (const cf*)Eold; g.Eout = (cf*)Eout; g.lde = n;
  g.R = (const cf*)R32; g.ldr = n; g.cr = cr;
  g.shift = shift; g.sa = sa; g.sb = sb;
  g.Bnext = (char*)Es_next;
  g.splits = 1;
  g.kstages = g.Kp / SBK;
  if (N >= SPLIT_WIDE_MIN_N) {
    g.tiles_m = (n + TileWide::BM - 1) / TileWide::BM;
    g.tiles_n = (N + TileWide::BN - 1) / TileWide::BN;
    const int grid = ((g.tiles_m + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
    hipLaunchKernelGGL(defect_gemm_split_wide, dim3(grid), dim3(TileWide::NTH), 0, s, g);
    return (int)hipGetLastError();
  }
  g.tiles_m = (n + TileSmall::BM - 1) / TileSmall::BM;
  g.tiles_n = (N + TileSmall::BN - 1) / TileSmall::BN;
  const int grid = ((g.tiles_m + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
  hipLaunchKernelGGL(defect_gemm_split, dim3(grid), dim3(TileSmall::NTH), 0, s, g);
  return (int)hipGetLastError();
}

int split_wide_min_cols() { return SPLIT_WIDE_MIN_N; }

size_t split_group_arg_bytes() { return sizeof(SplitArgs); }
size_t colsplit_group_arg_bytes() { return sizeof(ColSplitArgs); }

int split_group_fill(bool h16, bool wide, int n, int N, const void* Hs, float inv_h,
                     const void* Es, const float* inv_e, const void* Ecur, const void* Eold,
                     void* Eout, const void* R32, const float* cr, float shift, float sa,
                     float sb, void* Es_next, void* out) {
  SplitArgs g = {};
  g.M = n; g.N = N; g.Kp = split_kp(n);
  g.As = (const char*)Hs; g.a_row = (long)g.Kp * 8;
  g.Bs = (const char*)Es; g.b_row = (long)g.Kp * 8;
  g.Ecur = (const cf*)Ecur; g.Eold = (const cf*)Eold; g.Eout = (cf*)Eout; g.lde = n;
  g.R = (const cf*)R32; g.ldr = n; g.cr = cr;
  g.shift = shift; g.sa = sa; g.sb = sb;
  g.Bnext = h16 ? nullptr : (char*)Es_next;
  g.inv_a = inv_h; g.inv_b = inv_e;
  g.splits = 1;
  g.kstages = g.Kp / SBK;
  const int bm = wide ? TileWide::BM : TileSmall::BM, bn = wide ? TileWide::BN : TileSmall::BN;
  g.tiles_m = (n + bm - 1) / bm;
  g.tiles_n = (N + bn - 1) / bn;
  std::memcpy(out, &g, sizeof(g));
  return ((g.tiles_m + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
}

int split_group_launch(hipStream_t s, bool h16, bool wide, const void* dargs, const int* dslots,
                       int count, int total) {
  if (count <= 0 || total <= 0) return 0;
  const SplitArgs* l = (const SplitArgs*)dargs;
  if (wide) {
    if (h16)
      hipLaunchKernelGGL(defect_group_wide<true>, dim3(total), dim3(TileWide::NTH), 0, s, l,
                         dslots, count);
    else
      hipLaunchKernelGGL(defect_group_wide<false>, dim3(total), dim3(TileWide::NTH), 0, s, l,
                         dslots, count);
  } else {
    if (h16)
      hipLaunchKernelGGL(defect_group_small<true>, dim3(total), dim3(TileSmall::NTH), 0, s, l,
                         dslots, count);
    else
      hipLaunchKernelGGL(defect_group_small<false>, dim3(total), dim3(TileSmall::NTH), 0, s, l,
                         dslots, count);
  }
  return (int)hipGetLastError();
}

int colsplit_group_fill(int K, const void* E, long lde, void* S, float* inv, void* out) {
  ColSplitArgs a = {};
  a.K = K; a.Kp = split_kp(K);
  a.E = (const cf*)E; a.lde = lde;
  a.S = (char*)S; a.srow = (long)a.Kp * 8;
  a.inv = inv;
  std::memcpy(out, &a, sizeof(a));
  return 0;
}

int colsplit_group_launch(hipStream_t s, bool h16, const void* dargs, const int* dcols, int count,
                          int total_cols) {
  if (count <= 0 || total_cols <= 0) return 0;
  const ColSplitArgs* l = (const ColSplitArgs*)dargs;
  if (h16)
    hipLaunchKernelGGL(split_cols_group<true>, dim3(total_cols), dim3(256), 0, s, l, dcols, count);
  else
    hipLaunchKernelGGL(split_cols_group<false>, dim3(total_cols), dim3(256), 0, s, l, dcols, count);
  return (int)hipGetLastError();
}

int defect_step_h16(hipStream_t s, int n, int N, const void* Hs, float inv_h, const void* Es,
                    const float* inv_e, const void* Ecur, const void* Eold, void* Eout,
                    const void* R32, const float* cr, float shift, float sa, float sb,
                    void* part, size_t part_elems) {
  if (N <= 0) return 0;
  SplitArgs g = {};
  g.M = n; g.N = N; g.Kp = split_kp(n);
  g.As = (const char*)Hs; g.a_row = (long)g.Kp * 8;
  g.Bs = (const char*)Es; g.b_row = (long)g.Kp * 8;
  g.Ecur = (const cf*)Ecur; g.Eold = (const cf*)Eold; g.Eout = (cf*)Eout; g.lde = n;
  g.R = (const cf*)R32; g.ldr = n; g.cr = cr;
  g.shift = shift; g.sa = sa; g.sb = sb;
  g.Bnext = nullptr;
  g.inv_a = inv_h; g.inv_b = inv_e;
  g.splits = 1;
  g.kstages = g.Kp / SBK;
  if (N >= SPLIT_WIDE_MIN_N) {
    g.tiles_m = (n + TileWide::BM - 1) / TileWide::BM;
    g.tiles_n = (N + TileWide::BN - 1) / TileWide::BN;
    const int grid = ((g.tiles_m + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
    hipLaunchKernelGGL(defect_gemm_h16_wide, dim3(grid), dim3(TileWide::NTH), 0, s, g);
    return (int)hipGetLastError();
  }
  g.tiles_m = (n + TileSmall::BM - 1) / TileSmall::BM;
  g.tiles_n = (N + TileSmall::BN - 1) / TileSmall::BN;
  // split-K that fills the resident slots (two workgroups per CU) evenly
  const int stages = g.Kp / SBK;
  const int slots = 2 * split_device_cus();
  const long tiles = (long)g.tiles_m * g.tiles_n;
  const int max_s = (int)std::min<size_t>(8, part ? part_elems / ((size_t)n * N) : 1);
  double best_u = 0.0;
  int sp_best = 1;
  for (int sp = 1; sp <= max_s; ++sp) {
    if (sp > 1 && n / sp < 512) break;
    const long wg = tiles * sp;
    const double u = (double)wg / (double)(((wg + slots - 1) / slots) * slots);
    if (u > best_u + 1e-9) { best_u = u; sp_best = sp; }
    if (u >= 0.9) break;
  }
  g.kstages = (stages + sp_best - 1) / sp_best;
  g.splits = (stages + g.kstages - 1) / g.kstages;
  g.part = (cf*)part;
  const int grid = ((g.splits * g.tiles_m + NXCD - 1) / NXCD) * g.tiles_n * NXCD;
  hipLaunchKernelGGL(defect_gemm_h16, dim3(grid), dim3(TileSmall::NTH), 0, s, g);
  int e = (int)hipGetLastError();
  if (e || g.splits == 1) return e;
  return defect_reduce_launch(s, n, N, g.splits, part, Ecur, Eold, Eout, n, R32, n, cr, shift,
                              sa, sb);
}

}  // namespace chfsi
