// 16-bit passes over A (A stored in BF16 or FP16): v_mfma_f32_16x16x32_bf16 /
// _f16 with FP32 accumulation, for the sketch / power products T = A X and
// the orbit products T = A^T Y of Alg. 3 / Alg. 4, and for the projection
// A Q2 of eq. (M) with Q2 split into a 16-bit high and low part. The format
// is a template parameter (kFmtBF16 / kFmtF16); both MFMAs take the same
// operand layout.
//
// Power-of-two scaling (see H16Scale): the cast kernels scale the skinny
// operand, the epilogues and the reductions undo it on the FP64 output, and
// the sums of squares of A weight column j by 4^-e_j, so a run on
// A_stored = A diag(2^e_j) computes exactly what a run on A would.
//
// The 16x16x32 MFMA takes from each lane 8 16-bit values that are
// consecutive in the contraction index. Layouts are chosen so that every
// operand fragment is one 16-byte LDS read or global load:
//   * skinny operands are stored TRANSPOSED in HBM (LP rows of length K),
//     written that way by the library's own cast kernels;
//   * NN (T = A X): a tile of 64 RT rows x KB contraction indices of A and
//     the matching LP x KB block of the skinny operand are staged in LDS
//     (row runs of 2 KB bytes per load); lane l then reads row l % 16 of a
//     16-row tile and 8 consecutive contraction indices starting at
//     8 * (l / 16) of each step of 32 as one 16-byte LDS read, and the same
//     indices of a skinny column as another;
//   * TN (T = A^T Y): the contraction runs over rows of A, so a tile of
//     KST rows x (64 RT) columns of A is staged in LDS row-major (coalesced
//     16-byte loads and writes) and each lane gathers its 8 rows with
//     16-bit LDS reads. Inside every block of 32 contraction indices the
//     k-slot of lane group g, element t is row 4 t + g: the four lane groups
//     then read four consecutive LDS rows, which fall on disjoint banks for
//     a row stride of 64 RT + 8 elements. Y is stored with the same
//     permutation (position 8 g + t of each 32-block holds row 4 t + g), so
//     its fragment is again one 16-byte read.
// Partial sums per contraction split are summed afterwards in a fixed order.
//
// This header holds the kernel templates and their launch templates; each
// format is instantiated in a translation unit of its own (gemm_bf16.hip,
// gemm_f16.hip) so that the two compile in parallel.
#pragma once
#include "half16.hpp"

namespace sor {

__device__ inline int xcd_remap_b(int b, int nb) {
  return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

// Contiguous logical ranges per XCD for any workgroup count (see xcd_remap_any
// of the FP32 / FP64 passes).
__device__ inline int xcd_remap_any(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

union Frag {
  uint4 u;
  u32x4_t w;
  bf16x8 v;
  f16x8 f;
  uint16_t h[8];
};

// 8 consecutive 16-bit values p[0..7] as one 16-byte word, with zeros where
// ok_t is false: the path for unaligned rows and ragged ends. It builds whole
// 32-bit words, so that the vector path beside it keeps its loaded registers
// as they are (values assembled from 16-bit halves would make the compiler
// unpack, and so wait for, every vector load at once).
__device__ inline u32x4_t load8_slow(const uint16_t* p, int nvalid) {
  uint32_t w[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const uint32_t lo = 2 * t < nvalid ? p[2 * t] : 0u;
    const uint32_t hi = 2 * t + 1 < nvalid ? p[2 * t + 1] : 0u;
    w[t] = lo | (hi << 16);
  }
  return u32x4_t{w[0], w[1], w[2], w[3]};
}

__device__ inline u32x4_t load16_nt(const uint16_t* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
}

template <int FMT> __device__ inline f32x4 mfma16(const Frag& a, const Frag& b, f32x4 c) {
  if constexpr (FMT == kFmtBF16) return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0);
  else return __builtin_amdgcn_mfma_f32_16x16x32_f16(a.f, b.f, c, 0, 0, 0);
}

// The 8 column exponents of columns c .. c + 7 (0 beyond c1 or without cexp).
__device__ inline void load_exp8(const int* __restrict__ cexp, int64_t c, int64_t c1, int (&ev)[8]) {
#pragma unroll
  for (int t = 0; t < 8; ++t) ev[t] = (cexp && c + t < c1) ? cexp[c + t] : 0;
}

// Exponent that undoes the operand scaling on output row `orow`.
template <bool TRANS>
__device__ inline int out_shift(const H16Scale* sc, const int* cexp, int64_t orow) {
  if constexpr (TRANS) return -sc->tn_base - (cexp ? cexp[orow] : 0);
  else return -sc->nn_base;
}

// Epilogue: with a single contraction split the tiles go straight to the
// FP64 output T (row stride ldo; CT 16 columns, or CT 8 with `fold`, where
// the products with the high and low parts of the skinny operand, held by the
// same lane, are added in FP64), with the operand scaling undone for FP16
// (BF16 operands are never scaled); otherwise to the FP32 partials P (this
// split's and column block's, row stride ldp). Both pointers are already
// offset to the workgroup's column block.
template <int FMT, bool TRANS, int RT, int CT>
__device__ inline void store_tiles(const f32x4 (&acc)[RT][CT], int64_t base, int w, int g, int li,
                                   int64_t OUT, float* P, int64_t ldp, double* Tout, int64_t ldo, int fold,
                                   const H16Scale* sc, const int* cexp) {
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t orow = base + (int64_t)(w * RT + rt) * kTile + 4 * g + r;
      if (orow >= OUT) continue;
      if (Tout) {
        int sh = 0;
        if constexpr (FMT == kFmtF16) sh = out_shift<TRANS>(sc, cexp, orow);
        if (fold) {
#pragma unroll
          for (int ct = 0; ct < CT / 2; ++ct) {
            const double v = (double)acc[rt][ct][r] + (double)acc[rt][ct + CT / 2][r];
            Tout[orow * ldo + ct * kTile + li] = FMT == kFmtF16 ? ldexp(v, sh) : v;
          }
        } else {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const double v = (double)acc[rt][ct][r];
            Tout[orow * ldo + ct * kTile + li] = FMT == kFmtF16 ? ldexp(v, sh) : v;
          }
        }
      } else {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) P[orow * ldp + ct * kTile + li] = acc[rt][ct][r];
      }
    }
}

// Column blocks (ncb > 1): the skinny operand is cut into blocks of CT 16
// operand rows (its transposed layout holds block cb at rows cb CT 16 ..;
// with `fold` each block holds its high part followed by its low part), the
// workgroups of one (split, tile) take neighbouring logical indices (one XCD,
// A from HBM about once), and block cb writes output columns cb CT 16 .. (cb
// CT 8 .. with `fold`) of outputs and partial sums ncb blocks wide.
struct H16Block {
  int s, tile, cb, u;
};
__device__ inline H16Block h16_block(int tiles, int nsplit, int ncb) {
  const int nb = tiles * nsplit * ncb;
  const int v = ncb > 1 ? xcd_remap_any((int)blockIdx.x, nb) : xcd_remap_b((int)blockIdx.x, nb);
  H16Block b;
  b.cb = v % ncb;
  b.u = v / ncb;
  b.s = b.u / tiles;
  b.tile = b.u % tiles;
  return b;
}


// ---------------------------------------------------------------------------
// NN: P_s[r][c] = sum_{k in split s} A[r][k] X[k][c]; X given as XT (LP x ldx).
// A workgroup owns 64 RT rows and walks its contraction range in blocks of KB
// indices. Per block the tile of A (64 RT rows x KB) and the skinny block
// (LP x KB of XT) are loaded by the whole workgroup into registers one block
// ahead, then stored to LDS between two barriers: every wave instruction of
// the A loads reads KB * 2 bytes of consecutive columns from each of 512 /
// KB rows (256 B or more; HBM serves reads in such runs far better than in
// the 64 B pieces of the MFMA operand layout). Each wave then reads its MFMA
// operands from LDS with 16-byte reads: A fragments of its 16 RT rows (row
// l % 16, contraction 8 (l / 16) .. + 7 of each step of 32) and B fragments
// of the skinny block. LDS rows are padded by 8 values so the 16 rows of a
// fragment read start 4 banks apart. KB is the largest of 256, 128, 64 whose
// tiles fit 76 KB of LDS (two workgroups per CU). NRM: also the FP64 sum of
// squares of the A elements read (FP16: column j weighted by 4^-e_j), one
// value per workgroup in normp. kchunk must be a multiple of KB.
constexpr int nn_lds_bytes(int RT, int LP, int KB) { return (64 * RT + LP) * (KB + 8) * 2; }
constexpr int nn_kb(int RT, int LP) {
  return nn_lds_bytes(RT, LP, 256) <= 76 * 1024 ? 256 : (nn_lds_bytes(RT, LP, 128) <= 76 * 1024 ? 128 : 64);
}

template <int FMT, int RT, int CT, bool NRM>
__global__ void __launch_bounds__(256, 2)
k_h16_nn(const uint16_t* __restrict__ A, int64_t lda, int64_t OUT, int64_t K,
         const uint16_t* __restrict__ XT, int64_t ldx, int64_t kchunk, int tiles, int nsplit, int ncb,
         int vec_ok, float* __restrict__ P, double* __restrict__ normp, double* __restrict__ Tout,
         int fold, const H16Scale* __restrict__ sc, const int* __restrict__ cexp) {
  constexpr int LP = CT * kTile;
  constexpr int BR = 64 * RT;                 // rows of A per workgroup
  constexpr int KB = nn_kb(RT, LP);           // contraction indices per block
  constexpr int KS = KB + 8;                  // LDS row stride (A tile and skinny block)
  constexpr int CPR = KB / 8;                 // 16-byte chunks per row of a block
  constexpr int ACH = BR * CPR / 256;         // A chunks per thread per block
  constexpr int XTOT = LP * CPR;              // skinny chunks per block
  constexpr int XCH = (XTOT + 255) / 256;     // ... per thread
  constexpr int NJ = KB / 32;                 // MFMA steps per block
  static_assert(ACH * 256 == BR * CPR && 256 % CPR == 0, "A tile must split evenly over the workgroup");
  __shared__ __attribute__((aligned(16))) uint16_t As[BR * KS];
  __shared__ __attribute__((aligned(16))) uint16_t Xs[LP * KS];
  __shared__ double red[4];
  const H16Block bk = h16_block(tiles, nsplit, ncb);
  const int s = bk.s, tile = bk.tile;
  const bool nrm_on = NRM && bk.cb == 0;  // uniform over the workgroup
  XT += (int64_t)bk.cb * LP * ldx;
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int g = l / kTile, li = l % kTile;
  const int64_t k0 = (int64_t)s * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  const int64_t base = (int64_t)tile * BR;

  f32x4 acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0, 0, 0, 0};
  double nrm = 0.0;

  // chunk q of a block: row q / CPR, contraction 8 (q % CPR) .. + 7. As 256
  // is a multiple of CPR, a thread's chunks all cover the same 8 columns, so
  // FP16 column exponents are loaded once per block, with the block.
  u32x4_t ar[ACH], xr[XCH];
  int evn[8];
  auto load_block = [&](int64_t kb) {
    if constexpr (NRM && FMT == kFmtF16) load_exp8(cexp, kb + 8 * (threadIdx.x % CPR), k1, evn);
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int64_t row = base + q / CPR, kk = kb + 8 * (q % CPR);
      const bool in = row < OUT && kk < k1;
      if (vec_ok)  // rows 16-byte aligned and K % 8 == 0: whole chunks or none
        ar[i] = in ? load16_nt(A + row * lda + kk) : u32x4_t{0, 0, 0, 0};
      else
        ar[i] = in ? load8_slow(A + row * lda + kk, (int)min<int64_t>(8, k1 - kk)) : u32x4_t{0, 0, 0, 0};
    }
    // XT is zero-padded to ldx >= round_up(K, 128) + 128: whole blocks are in bounds
#pragma unroll
    for (int i = 0; i < XCH; ++i) {
      const int q = threadIdx.x + 256 * i;
      if (q < XTOT) xr[i] = *reinterpret_cast<const u32x4_t*>(XT + (int64_t)(q / CPR) * ldx + kb + 8 * (q % CPR));
    }
  };

  if (k0 < k1) load_block(k0);
  for (int64_t kb = k0; kb < k1; kb += KB) {
    __syncthreads();  // the previous block's operands have been read
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
      const int q = threadIdx.x + 256 * i;
      *reinterpret_cast<u32x4_t*>(As + (q / CPR) * KS + 8 * (q % CPR)) = ar[i];
    }
#pragma unroll
    for (int i = 0; i < XCH; ++i) {
      const int q = threadIdx.x + 256 * i;
      if (q < XTOT) *reinterpret_cast<u32x4_t*>(Xs + (q / CPR) * KS + 8 * (q % CPR)) = xr[i];
    }
    [[maybe_unused]] int ev[8];
    if constexpr (NRM && FMT == kFmtF16)
#pragma unroll
      for (int t = 0; t < 8; ++t) ev[t] = evn[t];
    __syncthreads();
    if (kb + KB < k1) load_block(kb + KB);
    // the sum of squares of this thread's chunks, read back from LDS while
    // the next block's loads are in flight
    if (nrm_on) {
#pragma unroll
      for (int i = 0; i < ACH; ++i) {
        const int q = threadIdx.x + 256 * i;
        Frag f;
        f.w = *reinterpret_cast<const u32x4_t*>(As + (q / CPR) * KS + 8 * (q % CPR));
        if constexpr (FMT == kFmtBF16) {
          float qs = 0.f;  // 8 squares of BF16 values (exact in FP32): a short FP32 sum, then FP64
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const float x = bf16_to_f32(f.h[t]);
            qs += x * x;
          }
          nrm += (double)qs;
        } else {
          // squares of FP16 values are exact in FP64, and so is the weight
          // 4^-e_j: with or without column exponents the same sum results
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const double x = (double)h16_to_f32<FMT>(f.h[t]);
            nrm += ldexp(x * x, -2 * ev[t]);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      Frag af[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
        af[rt].w = *reinterpret_cast<const u32x4_t*>(As + ((w * RT + rt) * kTile + li) * KS + 32 * j + 8 * g);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        Frag bx;
        bx.w = *reinterpret_cast<const u32x4_t*>(Xs + (ct * kTile + li) * KS + 32 * j + 8 * g);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma16<FMT>(af[rt], bx, acc[rt][ct]);
      }
    }
  }

  const int64_t ldp = (int64_t)ncb * LP, ldo = fold ? ldp / 2 : ldp;
  store_tiles<FMT, false, RT, CT>(acc, base, w, g, li, OUT, P + (int64_t)s * OUT * ldp + (int64_t)bk.cb * LP, ldp,
                                  Tout ? Tout + (int64_t)bk.cb * (fold ? LP / 2 : LP) : nullptr, ldo, fold, sc, cexp);
  if (nrm_on) {
    nrm = wave_sum(nrm);
    __syncthreads();
    if (l == 0) red[w] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) normp[bk.u] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ---------------------------------------------------------------------------
// TN: P_s[n][c] = sum_{i in split s} A[i][n] Y[i][c]; Y given as the permuted
// transpose YT (LP x ldy): YT[c][32 J + 8 g + t] = Y[32 J + 4 t + g][c].
// (The sum of squares of A is taken in the first NN pass only.)
template <int FMT, int RT, int CT, int KST>
__global__ void __launch_bounds__(256, 2)
k_h16_tn(const uint16_t* __restrict__ A, int64_t lda, int64_t OUT, int64_t K,
         const uint16_t* __restrict__ YT, int64_t ldy, int64_t kchunk, int tiles, int nsplit, int ncb,
         int vec_ok, float* __restrict__ P, double* __restrict__ Tout,
         const H16Scale* __restrict__ sc, const int* __restrict__ cexp) {
  constexpr int LP = CT * kTile;
  constexpr int BN = 64 * RT;                 // columns of A per workgroup
  constexpr int AS = BN + 8;                  // LDS row stride of the A tile
  constexpr int YS = KST + 8;                 // LDS row stride of the Y tile
  constexpr int ACH = KST * BN / 8 / 256;     // 16-byte A chunks per thread per step
  constexpr int YTOT = LP * KST / 8;          // 16-byte Y chunks per step
  constexpr int YCH = (YTOT + 255) / 256;     // ... per thread
  constexpr int NJ = KST / 32;                // MFMA contraction chunks per step
  __shared__ __attribute__((aligned(16))) uint16_t As[KST * AS];
  __shared__ __attribute__((aligned(16))) uint16_t Ys[LP * YS];

  const H16Block bk = h16_block(tiles, nsplit, ncb);
  const int s = bk.s, tile = bk.tile;
  YT += (int64_t)bk.cb * LP * ldy;
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int g = l / kTile, li = l % kTile;
  const int64_t k0 = (int64_t)s * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  const int64_t base = (int64_t)tile * BN;

  f32x4 acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0, 0, 0, 0};

  // A chunk q: tile row r = q / (BN / 8), columns 8 * (q % (BN / 8)) .. + 7.
  // vec_ok (rows 16-byte aligned, OUT % 8 == 0): whole chunks or none.
  auto load_a = [&](u32x4_t (&ar)[ACH], int64_t kb) {
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int r = q / (BN / 8), cc = 8 * (q % (BN / 8));
      const int64_t row = kb + r, col = base + cc;
      const bool in = row < k1 && col < OUT;
      if (vec_ok)
        ar[i] = in ? load16_nt(A + row * lda + col) : u32x4_t{0, 0, 0, 0};
      else
        ar[i] = in ? load8_slow(A + row * lda + col, (int)min<int64_t>(8, OUT - col)) : u32x4_t{0, 0, 0, 0};
    }
  };
  auto load_y = [&](u32x4_t (&yr)[YCH], int64_t kb) {
#pragma unroll
    for (int i = 0; i < YCH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int c = q / (KST / 8), o = 8 * (q % (KST / 8));
      if (q < YTOT) yr[i] = *reinterpret_cast<const u32x4_t*>(YT + c * ldy + kb + o);  // YT zero-padded to ldy
    }
  };

  u32x4_t ar[ACH], yr[YCH];
  if (k0 < k1) { load_a(ar, k0); load_y(yr, k0); }
  for (int64_t kb = k0; kb < k1; kb += KST) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int r = q / (BN / 8), cc = 8 * (q % (BN / 8));
      *reinterpret_cast<u32x4_t*>(As + r * AS + cc) = ar[i];
    }
#pragma unroll
    for (int i = 0; i < YCH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int c = q / (KST / 8), o = 8 * (q % (KST / 8));
      if (q < YTOT) *reinterpret_cast<u32x4_t*>(Ys + c * YS + o) = yr[i];
    }
    __syncthreads();
    if (kb + KST < k1) { load_a(ar, kb + KST); load_y(yr, kb + KST); }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      Frag af[RT];
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const int col = (w * RT + rt) * kTile + li;
#pragma unroll
        for (int t = 0; t < 8; ++t) af[rt].h[t] = As[(32 * j + 4 * t + g) * AS + col];
      }
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        Frag b;
        b.u = *reinterpret_cast<const uint4*>(Ys + (ct * kTile + li) * YS + 32 * j + 8 * g);
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma16<FMT>(af[rt], b, acc[rt][ct]);
      }
    }
  }

  const int64_t ldp = (int64_t)ncb * LP;
  store_tiles<FMT, true, RT, CT>(acc, base, w, g, li, OUT, P + (int64_t)s * OUT * ldp + (int64_t)bk.cb * LP, ldp,
                                 Tout ? Tout + (int64_t)bk.cb * LP : nullptr, ldp, 0, sc, cexp);
}

// ------------------------------------------------------------ launch templates

// Rows (NN) or columns (TN) of A per workgroup = 64 rt, rt in {1, 2, 4}.
// With nsplit == 1 the result goes straight to Tout (FP64). normp (NN only):
// the sums of squares of A, one per workgroup.
// LP: total operand width (ncb column blocks of LP / ncb).
template <int FMT, int RT>
inline hipError_t launch_h16_rt(bool trans, const uint16_t* A, int64_t lda, int64_t OUT, int64_t K,
                                const uint16_t* XT, int64_t ldx, int LP, int64_t kchunk, int nsplit, int ncb,
                                float* P, double* normp, double* Tout, int fold, const H16Scale* sc,
                                const int* cexp, hipStream_t st) {
  const int tiles = (int)ceil_div(OUT, 64 * RT);
  if (tiles == 0 || nsplit == 0) return hipSuccess;
  if (trans && normp) return hipErrorInvalidValue;
  if (ncb < 1 || LP % (ncb * kTile) || (fold && (LP / ncb) % (2 * kTile))) return hipErrorInvalidValue;
  const int CTB = LP / ncb / kTile;
  // whole 16-byte chunks: aligned rows, and no chunk straddling the end of a
  // row (NN: K % 8 == 0; TN: OUT % 8 == 0)
  const int vec_ok = ((lda * 2) % 16 == 0) && (((uintptr_t)A) % 16 == 0) && ((trans ? OUT : K) % 8 == 0);
  double* To = nsplit == 1 ? Tout : nullptr;
  constexpr int KST = RT >= 4 ? 64 : 128;
  dim3 grid((unsigned)(tiles * nsplit * ncb)), block(256);
#define SORSVD_BF(C)                                                                               \
  case C:                                                                                          \
    if (trans)                                                                                     \
      hipLaunchKernelGGL((k_h16_tn<FMT, RT, C, KST>), grid, block, 0, st, A, lda, OUT, K, XT, ldx, \
                         kchunk, tiles, nsplit, ncb, vec_ok, P, To, sc, cexp);                     \
    else if (kchunk % nn_kb(RT, C * kTile) != 0)                                                   \
      return hipErrorInvalidValue;                                                                 \
    else if (normp)                                                                                \
      hipLaunchKernelGGL((k_h16_nn<FMT, RT, C, true>), grid, block, 0, st, A, lda, OUT, K, XT,     \
                         ldx, kchunk, tiles, nsplit, ncb, vec_ok, P, normp, To, fold, sc, cexp);   \
    else                                                                                           \
      hipLaunchKernelGGL((k_h16_nn<FMT, RT, C, false>), grid, block, 0, st, A, lda, OUT, K, XT,    \
                         ldx, kchunk, tiles, nsplit, ncb, vec_ok, P, normp, To, fold, sc, cexp);   \
    break;
  switch (CTB) {
    SORSVD_BF(1) SORSVD_BF(2) SORSVD_BF(3) SORSVD_BF(4) SORSVD_BF(5) SORSVD_BF(6)
    SORSVD_BF(7) SORSVD_BF(8) SORSVD_BF(10) SORSVD_BF(12) SORSVD_BF(14) SORSVD_BF(16)
    default: return hipErrorInvalidValue;
  }
#undef SORSVD_BF
  return hipGetLastError();
}

template <int FMT>
inline hipError_t launch_h16_fmt(bool trans, const uint16_t* A, int64_t lda, int64_t OUT, int64_t K,
                                 const uint16_t* XT, int64_t ldx, int LP, int64_t kchunk, int nsplit, int ncb,
                                 float* P, double* normp, double* Tout, int fold, int rt, const H16Scale* sc,
                                 const int* cexp, hipStream_t st) {
  switch (rt) {
    case 1: return launch_h16_rt<FMT, 1>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, ncb, P, normp, Tout, fold, sc, cexp, st);
    case 2: return launch_h16_rt<FMT, 2>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, ncb, P, normp, Tout, fold, sc, cexp, st);
    case 4: return launch_h16_rt<FMT, 4>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, ncb, P, normp, Tout, fold, sc, cexp, st);
    default: return hipErrorInvalidValue;
  }
}

// Workgroups of a 16-bit pass kernel that the current device holds at once
// (resident workgroups per CU times the CUs); 0 when no device answers.
template <int FMT, int RT>
inline int h16_blocks_per_cu(bool trans, int CT) {
  constexpr int KST = RT >= 4 ? 64 : 128;
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SORSVD_BF(C)                                                                                          \
  case C:                                                                                                     \
    e = trans ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                 \
                    &nb, reinterpret_cast<const void*>(&k_h16_tn<FMT, RT, C, KST>), 256, 0)                  \
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                 \
                    &nb, reinterpret_cast<const void*>(&k_h16_nn<FMT, RT, C, false>), 256, 0);               \
    break;
  switch (CT) {
    SORSVD_BF(1) SORSVD_BF(2) SORSVD_BF(3) SORSVD_BF(4) SORSVD_BF(5) SORSVD_BF(6)
    SORSVD_BF(7) SORSVD_BF(8) SORSVD_BF(10) SORSVD_BF(12) SORSVD_BF(14) SORSVD_BF(16)
    default: break;
  }
#undef SORSVD_BF
  return e == hipSuccess ? nb : 0;
}

template <int FMT>
inline int h16_blocks(bool trans, int rt, int CT) {
  return rt == 1 ? h16_blocks_per_cu<FMT, 1>(trans, CT)
                 : (rt == 2 ? h16_blocks_per_cu<FMT, 2>(trans, CT) : h16_blocks_per_cu<FMT, 4>(trans, CT));
}

}  // namespace sor
