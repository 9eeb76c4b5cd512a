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
//   * NN (T = A X): lane l takes row l % 16 of A and 8 consecutive
//     contraction indices starting at 8 * (l / 16) per step of 32 (a 16-byte
//     load straight from HBM into registers), and the matching 16 bytes of
//     the transposed skinny operand from L2; no LDS, no barriers;
//   * TN (T = A^T Y): the contraction runs over rows of A, so a tile of
//     128 rows x (64 RT) columns of A is staged in LDS row-major (coalesced
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
// FP64 output T (OUT x LP, or OUT x LP/2 with `fold`, where the products with
// the high and low parts of the skinny operand, held by the same lane, are
// added in FP64), with the operand scaling undone for FP16 (BF16 operands are
// never scaled); otherwise to the FP32 partials P[s].
template <int FMT, bool TRANS, int RT, int CT>
__device__ inline void store_tiles(const f32x4 (&acc)[RT][CT], int64_t base, int w, int g, int li,
                                   int64_t OUT, int s, float* P, double* Tout, int fold,
                                   const H16Scale* sc, const int* cexp) {
  constexpr int LP = CT * kTile;
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
            Tout[orow * (LP / 2) + ct * kTile + li] = FMT == kFmtF16 ? ldexp(v, sh) : v;
          }
        } else {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) {
            const double v = (double)acc[rt][ct][r];
            Tout[orow * LP + ct * kTile + li] = FMT == kFmtF16 ? ldexp(v, sh) : v;
          }
        }
      } else {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          P[((int64_t)s * OUT + orow) * LP + ct * kTile + li] = acc[rt][ct][r];
      }
    }
}


// ---------------------------------------------------------------------------
// NN: P_s[r][c] = sum_{k in split s} A[r][k] X[k][c]; X given as XT (LP x ldx).
// Each wave owns 16 RW rows and streams them in steps of 32 contraction
// indices: per step a lane loads one 16-byte A fragment per row tile (row
// l % 16, indices 8 (l / 16) .. + 7, the MFMA operand layout) straight into
// registers, and a ring of D steps keeps D - 1 steps of A loads in flight
// behind the MFMAs. The skinny operand is shared by the four waves through
// LDS: blocks of KB contraction indices of XT (LP x KB) are loaded by the
// whole workgroup one block ahead and stored to the other of two LDS buffers
// (one barrier per block); each wave then reads its 16-byte B fragments from
// LDS (rows padded by 8 values, so the 16 rows of a read start 4 banks apart).
// Loading them per wave from L2 instead doubles the vector-memory traffic at
// l = 64 and triples it for the refinement pass. NRM: also the FP64 sum of
// squares of the A elements read (FP16: column j weighted by 4^-e_j), one
// value per workgroup in normp. kchunk must be a multiple of KB.
template <int CT> constexpr int nn_kb() { return CT >= 10 ? 64 : 128; }

template <int FMT, int RW, int CT, bool NRM>
__global__ void __launch_bounds__(256, 2)
k_h16_nn(const uint16_t* __restrict__ A, int64_t lda, int64_t OUT, int64_t K,
         const uint16_t* __restrict__ XT, int64_t ldx, int64_t kchunk, int tiles, int nsplit,
         int vec_ok, float* __restrict__ P, double* __restrict__ normp, double* __restrict__ Tout,
         int fold, const H16Scale* __restrict__ sc, const int* __restrict__ cexp) {
  constexpr int KS32 = 32;
  constexpr int LP = CT * kTile;
  constexpr int KB = nn_kb<CT>();        // contraction indices per skinny block
  constexpr int D = KB / KS32;           // A ring depth = steps per block
  constexpr int XS = KB + 8;             // LDS row stride of a skinny block
  constexpr int XCH = LP * KB / 8 / 256; // 16-byte skinny chunks per thread per block
  static_assert(XCH * 256 * 8 == LP * KB, "skinny block must split evenly over the workgroup");
  __shared__ __attribute__((aligned(16))) uint16_t Xs[2][LP * XS];
  __shared__ double red[4];
  const int nb = tiles * nsplit;
  const int v = xcd_remap_b((int)blockIdx.x, nb);
  const int s = v / tiles, tile = v % tiles;
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int g = l / kTile, li = l % kTile;
  const int64_t k0 = (int64_t)s * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  const int64_t base = (int64_t)tile * (64 * RW);

  f32x4 acc[RW][CT];
#pragma unroll
  for (int rt = 0; rt < RW; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = f32x4{0, 0, 0, 0};
  double nrm = 0.0;

  auto load_a = [&](Frag (&a)[RW], int64_t kb) {
    const int64_t kk = kb + 8 * g;
#pragma unroll
    for (int rt = 0; rt < RW; ++rt) {
      const int64_t row = base + (int64_t)(w * RW + rt) * kTile + li;
      const bool in = row < OUT && kk < k1;
      if (vec_ok)  // rows 16-byte aligned and K % 8 == 0: whole chunks or none
        a[rt].w = in ? load16_nt(A + row * lda + kk) : u32x4_t{0, 0, 0, 0};
      else
        a[rt].w = in ? load8_slow(A + row * lda + kk, (int)min<int64_t>(8, k1 - kk)) : u32x4_t{0, 0, 0, 0};
    }
  };
  // chunk q of a block: skinny row c = q / (KB / 8), values 8 (q % (KB / 8)) .. + 7
  // (XT is zero-padded to ldx >= round_up(K, 128) + 128, so whole blocks are in bounds)
  u32x4_t xr[XCH];
  auto load_x = [&](int64_t kb) {
#pragma unroll
    for (int i = 0; i < XCH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int c = q / (KB / 8), o = 8 * (q % (KB / 8));
      xr[i] = *reinterpret_cast<const u32x4_t*>(XT + (int64_t)c * ldx + kb + o);
    }
  };
  auto store_x = [&](int b) {
#pragma unroll
    for (int i = 0; i < XCH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int c = q / (KB / 8), o = 8 * (q % (KB / 8));
      *reinterpret_cast<u32x4_t*>(&Xs[b][c * XS + o]) = xr[i];
    }
  };

  Frag ab[D][RW];
  if (k0 < k1) {
    load_x(k0);
    store_x(0);
#pragma unroll
    for (int d = 0; d < D - 1; ++d) load_a(ab[d], k0 + (int64_t)d * KS32);
    if (k0 + KB < k1) load_x(k0 + KB);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t kb = k0; kb < k1; kb += KB) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int64_t knext = kb + (int64_t)(j + D - 1) * KS32;
      if (knext < k1) load_a(ab[(j + D - 1) % D], knext);
      if (kb + (int64_t)j * KS32 < k1) {
        if constexpr (NRM) {
          if constexpr (FMT == kFmtBF16) {
#pragma unroll
            for (int rt = 0; rt < RW; ++rt) {
              float q = 0.f;  // 8 squares of BF16 values (exact in FP32): a short FP32 sum, then FP64
#pragma unroll
              for (int t = 0; t < 8; ++t) {
                const float x = bf16_to_f32(ab[j][rt].h[t]);
                q += x * x;
              }
              nrm += (double)q;
            }
          } else {
            // squares of FP16 values are exact in FP64, and so is the weight
            // 4^-e_j: with or without column exponents the same sum results
            int ev[8];
            load_exp8(cexp, kb + (int64_t)j * KS32 + 8 * g, k1, ev);
#pragma unroll
            for (int rt = 0; rt < RW; ++rt)
#pragma unroll
              for (int t = 0; t < 8; ++t) {
                const double x = (double)h16_to_f32<FMT>(ab[j][rt].h[t]);
                nrm += ldexp(x * x, -2 * ev[t]);
              }
          }
        }
        Frag bx[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          bx[ct].w = *reinterpret_cast<const u32x4_t*>(&Xs[buf][(ct * kTile + li) * XS + KS32 * j + 8 * g]);
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int rt = 0; rt < RW; ++rt) acc[rt][ct] = mfma16<FMT>(ab[j][rt], bx[ct], acc[rt][ct]);
      }
    }
    // the other buffer was last read in the previous block, which every wave
    // finished before the barrier that ended it
    if (kb + KB < k1) store_x(buf ^ 1);
    __syncthreads();
    buf ^= 1;
    if (kb + 2 * KB < k1) load_x(kb + 2 * KB);
  }

  store_tiles<FMT, false, RW, CT>(acc, base, w, g, li, OUT, s, P, Tout, fold, sc, cexp);
  if constexpr (NRM) {
    nrm = wave_sum(nrm);
    if (l == 0) red[w] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) normp[v] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ---------------------------------------------------------------------------
// TN: P_s[n][c] = sum_{i in split s} A[i][n] Y[i][c]; Y given as the permuted
// transpose YT (LP x ldy): YT[c][32 J + 8 g + t] = Y[32 J + 4 t + g][c].
// (The sum of squares of A is taken in the first NN pass only.)
template <int FMT, int RT, int CT, int KST>
__global__ void __launch_bounds__(256, 2)
k_h16_tn(const uint16_t* __restrict__ A, int64_t lda, int64_t OUT, int64_t K,
         const uint16_t* __restrict__ YT, int64_t ldy, int64_t kchunk, int tiles, int nsplit,
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

  const int nb = tiles * nsplit;
  const int v = xcd_remap_b((int)blockIdx.x, nb);
  const int s = v / tiles, tile = v % tiles;
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

  store_tiles<FMT, true, RT, CT>(acc, base, w, g, li, OUT, s, P, Tout, 0, sc, cexp);
}

// ------------------------------------------------------------ launch templates

// Rows (NN) or columns (TN) of A per workgroup = 64 rt, rt in {1, 2, 4}.
// With nsplit == 1 the result goes straight to Tout (FP64). normp (NN only):
// the sums of squares of A, one per workgroup.
template <int FMT, int RT>
inline hipError_t launch_h16_rt(bool trans, const uint16_t* A, int64_t lda, int64_t OUT, int64_t K,
                                const uint16_t* XT, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                                float* P, double* normp, double* Tout, int fold, const H16Scale* sc,
                                const int* cexp, hipStream_t st) {
  const int tiles = (int)ceil_div(OUT, 64 * RT);
  if (tiles == 0 || nsplit == 0) return hipSuccess;
  if (trans && normp) return hipErrorInvalidValue;
  // whole 16-byte chunks: aligned rows, and no chunk straddling the end of a
  // row (NN: K % 8 == 0; TN: OUT % 8 == 0)
  const int vec_ok = ((lda * 2) % 16 == 0) && (((uintptr_t)A) % 16 == 0) && ((trans ? OUT : K) % 8 == 0);
  double* To = nsplit == 1 ? Tout : nullptr;
  constexpr int KST = RT >= 4 ? 64 : 128;
  dim3 grid((unsigned)(tiles * nsplit)), block(256);
#define SORSVD_BF(C)                                                                               \
  case C:                                                                                          \
    if (trans)                                                                                     \
      hipLaunchKernelGGL((k_h16_tn<FMT, RT, C, KST>), grid, block, 0, st, A, lda, OUT, K, XT, ldx, \
                         kchunk, tiles, nsplit, vec_ok, P, To, sc, cexp);                          \
    else if (kchunk % nn_kb<C>() != 0)                                                             \
      return hipErrorInvalidValue;                                                                 \
    else if (normp)                                                                                \
      hipLaunchKernelGGL((k_h16_nn<FMT, RT, C, true>), grid, block, 0, st, A, lda, OUT, K, XT,     \
                         ldx, kchunk, tiles, nsplit, vec_ok, P, normp, To, fold, sc, cexp);        \
    else                                                                                           \
      hipLaunchKernelGGL((k_h16_nn<FMT, RT, C, false>), grid, block, 0, st, A, lda, OUT, K, XT,    \
                         ldx, kchunk, tiles, nsplit, vec_ok, P, normp, To, fold, sc, cexp);        \
    break;
  switch (LP / kTile) {
    SORSVD_BF(1) SORSVD_BF(2) SORSVD_BF(3) SORSVD_BF(4) SORSVD_BF(5) SORSVD_BF(6)
    SORSVD_BF(7) SORSVD_BF(8) SORSVD_BF(10) SORSVD_BF(12) SORSVD_BF(14) SORSVD_BF(16)
    default: return hipErrorInvalidValue;
  }
#undef SORSVD_BF
  return hipGetLastError();
}

template <int FMT>
inline hipError_t launch_h16_fmt(bool trans, const uint16_t* A, int64_t lda, int64_t OUT, int64_t K,
                                 const uint16_t* XT, int64_t ldx, int LP, int64_t kchunk, int nsplit, float* P,
                                 double* normp, double* Tout, int fold, int rt, const H16Scale* sc,
                                 const int* cexp, hipStream_t st) {
  switch (rt) {
    case 1: return launch_h16_rt<FMT, 1>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, P, normp, Tout, fold, sc, cexp, st);
    case 2: return launch_h16_rt<FMT, 2>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, P, normp, Tout, fold, sc, cexp, st);
    case 4: return launch_h16_rt<FMT, 4>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, P, normp, Tout, fold, sc, cexp, st);
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
