// BF16 passes over A (A stored in BF16): BF16 MFMA (v_mfma_f32_16x16x32_bf16)
// with FP32 accumulation, for the sketch / power products T = A X and the
// orbit products T = A^T Y of Alg. 3 / Alg. 4, and for the projection A Q2
// of eq. (M) with Q2 split into a BF16 high and low part.
//
// The 16x16x32 BF16 MFMA takes from each lane 8 BF16 values that are
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
#include <map>
#include <mutex>
#include <tuple>

#include "common.hpp"

namespace sor {

__device__ inline f32x4 mfma_bf16(const bf16x8& a, const bf16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline int xcd_remap_b(int b, int nb) {
  return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

union Frag {
  uint4 u;
  bf16x8 v;
  uint16_t h[8];
};

__device__ inline double sumsq_bf16(const Frag& f) {
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const double x = (double)bf16_to_f32(f.h[t]);
    s += x * x;
  }
  return s;
}

// Epilogue: with a single contraction split the tiles go straight to the
// FP64 output T (OUT x LP, or OUT x LP/2 with `fold`, where the products with
// the high and low parts of the skinny operand, held by the same lane, are
// added in FP64); otherwise to the FP32 partials P[s].
template <int RT, int CT>
__device__ inline void store_tiles(const f32x4 (&acc)[RT][CT], int64_t base, int w, int g, int li,
                                   int64_t OUT, int s, float* P, double* Tout, int fold) {
  constexpr int LP = CT * kTile;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t orow = base + (int64_t)(w * RT + rt) * kTile + 4 * g + r;
      if (orow >= OUT) continue;
      if (Tout) {
        if (fold) {
#pragma unroll
          for (int ct = 0; ct < CT / 2; ++ct)
            Tout[orow * (LP / 2) + ct * kTile + li] =
                (double)acc[rt][ct][r] + (double)acc[rt][ct + CT / 2][r];
        } else {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) Tout[orow * LP + ct * kTile + li] = (double)acc[rt][ct][r];
        }
      } else {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
          P[((int64_t)s * OUT + orow) * LP + ct * kTile + li] = acc[rt][ct][r];
      }
    }
}

constexpr int kKS = 128;        // contraction indices per step
constexpr int kXS = kKS + 8;    // LDS row stride of transposed skinny tiles (16-byte aligned rows)

// ---------------------------------------------------------------------------
// NN: P_s[r][c] = sum_{k in split s} A[r][k] X[k][c]; X given as XT (LP x ldx).
// No LDS and no barriers: each wave owns 16 RW rows and streams them in
// steps of 32 contraction indices. Per step a lane loads one 16-byte A
// fragment per row tile (row l % 16, indices 8 (l / 16) .. + 7) and one
// 16-byte skinny fragment per column tile (column l % 16, same indices; an
// L2 hit), exactly the MFMA operand layouts. A ring of D steps of fragments
// keeps D - 1 steps of loads in flight behind the MFMAs.
template <int RW, int CT, int D>
__global__ void __launch_bounds__(256, 2)
k_bf16_nn(const bf16_t* __restrict__ A, int64_t lda, int64_t OUT, int64_t K,
          const bf16_t* __restrict__ XT, int64_t ldx, int64_t kchunk, int tiles, int nsplit,
          int vec_ok, float* __restrict__ P, double* __restrict__ normp, double* __restrict__ Tout,
          int fold) {
  constexpr int KS32 = 32;
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

  auto load = [&](Frag (&a)[RW], Frag (&x)[CT], int64_t kb) {
    const int64_t kk = kb + 8 * g;
#pragma unroll
    for (int rt = 0; rt < RW; ++rt) {
      const int64_t row = base + (int64_t)(w * RW + rt) * kTile + li;
      if (row < OUT && kk + 8 <= k1 && vec_ok) {
        a[rt].u = load_stream16(A + row * lda + kk);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t)
          a[rt].h[t] = (row < OUT && kk + t < k1) ? A[row * lda + kk + t] : (bf16_t)0;
      }
    }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)  // XT is zero-padded to ldx >= round_up(K, 128)
      x[ct].u = *reinterpret_cast<const uint4*>(XT + (int64_t)(ct * kTile + li) * ldx + kk);
  };

  Frag ab[D][RW], xb[D][CT];
#pragma unroll
  for (int d = 0; d < D - 1; ++d) load(ab[d], xb[d], k0 + (int64_t)d * KS32);
  for (int64_t kb = k0; kb < k1; kb += (int64_t)D * KS32) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t knext = kb + (int64_t)(d + D - 1) * KS32;
      if (knext < k1) load(ab[(d + D - 1) % D], xb[(d + D - 1) % D], knext);
      if (kb + (int64_t)d * KS32 < k1) {
        if (normp) {
#pragma unroll
          for (int rt = 0; rt < RW; ++rt) {
            float q = 0.f;  // 8 squares of BF16 values: a short FP32 sum, then FP64
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const float x = bf16_to_f32(ab[d][rt].h[t]);
              q += x * x;
            }
            nrm += (double)q;
          }
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int rt = 0; rt < RW; ++rt) acc[rt][ct] = mfma_bf16(ab[d][rt].v, xb[d][ct].v, acc[rt][ct]);
      }
    }
  }

  store_tiles<RW, CT>(acc, base, w, g, li, OUT, s, P, Tout, fold);
  if (normp) {
    nrm = wave_sum(nrm);
    if (l == 0) red[w] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) normp[v] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ---------------------------------------------------------------------------
// TN: P_s[n][c] = sum_{i in split s} A[i][n] Y[i][c]; Y given as the permuted
// transpose YT (LP x ldy): YT[c][32 J + 8 g + t] = Y[32 J + 4 t + g][c].
template <int RT, int CT, int KST>
__global__ void __launch_bounds__(256, 2)
k_bf16_tn(const bf16_t* __restrict__ A, int64_t lda, int64_t OUT, int64_t K,
          const bf16_t* __restrict__ YT, int64_t ldy, int64_t kchunk, int tiles, int nsplit,
          int vec_ok, float* __restrict__ P, double* __restrict__ normp, double* __restrict__ Tout) {
  constexpr int LP = CT * kTile;
  constexpr int BN = 64 * RT;                 // columns of A per workgroup
  constexpr int AS = BN + 8;                  // LDS row stride of the A tile
  constexpr int YS = KST + 8;                 // LDS row stride of the Y tile
  constexpr int ACH = KST * BN / 8 / 256;     // 16-byte A chunks per thread per step
  constexpr int YTOT = LP * KST / 8;          // 16-byte Y chunks per step
  constexpr int YCH = (YTOT + 255) / 256;     // ... per thread
  constexpr int NJ = KST / 32;                // MFMA contraction chunks per step
  __shared__ __attribute__((aligned(16))) bf16_t As[KST * AS];
  __shared__ __attribute__((aligned(16))) bf16_t Ys[LP * YS];
  __shared__ double red[4];

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
  double nrm = 0.0;

  // A chunk q: tile row r = q / (BN / 8), columns 8 * (q % (BN / 8)) .. + 7
  auto load_a = [&](uint4 (&ar)[ACH], int64_t kb) {
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int r = q / (BN / 8), cc = 8 * (q % (BN / 8));
      const int64_t row = kb + r, col = base + cc;
      Frag f;
      if (row < k1 && col + 8 <= OUT && vec_ok) {
        f.u = load_stream16(A + row * lda + col);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t)
          f.h[t] = (row < k1 && col + t < OUT) ? A[row * lda + col + t] : (bf16_t)0;
      }
      ar[i] = f.u;
    }
  };
  auto load_y = [&](uint4 (&yr)[YCH], int64_t kb) {
#pragma unroll
    for (int i = 0; i < YCH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int c = q / (KST / 8), o = 8 * (q % (KST / 8));
      if (q < YTOT) yr[i] = *reinterpret_cast<const uint4*>(YT + c * ldy + kb + o);  // YT zero-padded to ldy
    }
  };

  uint4 ar[ACH], yr[YCH];
  if (k0 < k1) { load_a(ar, k0); load_y(yr, k0); }
  for (int64_t kb = k0; kb < k1; kb += KST) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ACH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int r = q / (BN / 8), cc = 8 * (q % (BN / 8));
      *reinterpret_cast<uint4*>(As + r * AS + cc) = ar[i];
      if (normp) {
        Frag f;
        f.u = ar[i];
        nrm += sumsq_bf16(f);
      }
    }
#pragma unroll
    for (int i = 0; i < YCH; ++i) {
      const int q = threadIdx.x + 256 * i;
      const int c = q / (KST / 8), o = 8 * (q % (KST / 8));
      if (q < YTOT) *reinterpret_cast<uint4*>(Ys + c * YS + o) = yr[i];
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
        for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = mfma_bf16(af[rt].v, b.v, acc[rt][ct]);
      }
    }
  }

  store_tiles<RT, CT>(acc, base, w, g, li, OUT, s, P, Tout, 0);
  if (normp) {
    nrm = wave_sum(nrm);
    if (l == 0) red[w] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) normp[v] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// ---------------------------------------------------------------------------
// Skinny operand of a BF16 pass: Q (rows x LP, FP64, row-major) -> the
// transposed BF16 layout QT (LP x ldt), optionally with the contraction
// permutation of the TN kernel, optionally followed by the low part
// QT[LP + c][.] = bf16(Q - hi) (the refinement split). Rows rows..ldt-1 are
// written as zeros. Tiles of 64 rows go through LDS so that both the reads
// of Q and the writes of QT are coalesced.
__global__ void __launch_bounds__(256)
k_cast_bf16_t(const double* __restrict__ Q, int64_t rows, int LP, int64_t ldt, int permute,
              int with_lo, bf16_t* __restrict__ QT) {
  __shared__ double tile[64][129];
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  for (int i = threadIdx.x; i < 64 * LP; i += 256) {
    const int rr = i / LP, c = i % LP;
    const int64_t r = r0 + rr;
    tile[rr][c] = (r < rows) ? Q[r * LP + c] : 0.0;
  }
  __syncthreads();
  const int parts = with_lo ? 2 : 1;
  for (int i = threadIdx.x; i < 64 * LP * parts; i += 256) {
    const int rr = i % 64, cp = i / 64;
    const int c = cp % LP, part = cp / LP;
    const int64_t r = r0 + rr;
    if (r >= ldt) continue;
    const double q = tile[rr][c];
    const bf16_t hi = f64_to_bf16(q);
    const bf16_t val = part == 0 ? hi : f64_to_bf16(q - (double)bf16_to_f32(hi));
    int64_t pos = r;
    if (permute) {  // row 32 J + 4 t + g -> position 32 J + 8 g + t
      const int64_t J = r / 32, within = r % 32;
      pos = 32 * J + 8 * (within % 4) + within / 4;
    }
    QT[((int64_t)part * LP + c) * ldt + pos] = val;
  }
}

// out[r][c] = sum_s (P[s][r][c] + P[s][r][c + LPh]) for c < ncols: the
// refinement pass adds the products with the high and low parts of Q2.
__global__ void __launch_bounds__(256)
k_reduce_fold(const float* __restrict__ P, int64_t OUT, int LP2, int nsplit, double* __restrict__ out,
              int64_t ldo, int ncols) {
  const int LPh = LP2 / 2;
  const int64_t total = OUT * LPh;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int64_t r = idx / LPh;
  const int c = (int)(idx % LPh);
  double acc = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    const float* p = P + ((int64_t)s * OUT + r) * LP2;
    acc += (double)p[c] + (double)p[c + LPh];
  }
  if (c < ncols) out[r * ldo + c] = acc;
}

// ------------------------------------------------------------------ launchers

// Rows (NN) or columns (TN) of A per workgroup = 64 rt, rt in {1, 2, 4}.
// With nsplit == 1 the result goes straight to Tout (FP64).
template <int RT>
static hipError_t launch_bf16_rt(bool trans, const bf16_t* A, int64_t lda, int64_t OUT, int64_t K,
                                 const bf16_t* XT, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                                 float* P, double* normp, double* Tout, int fold, hipStream_t st) {
  const int tiles = (int)ceil_div(OUT, 64 * RT);
  if (tiles == 0 || nsplit == 0) return hipSuccess;
  const int vec_ok = ((lda * 2) % 16 == 0) && (((uintptr_t)A) % 16 == 0);
  double* To = nsplit == 1 ? Tout : nullptr;
  constexpr int KST = RT >= 4 ? 64 : 128;
  dim3 grid((unsigned)(tiles * nsplit)), block(256);
#define SORSVD_BF(C, D)                                                                            \
  case C:                                                                                          \
    if (trans)                                                                                     \
      hipLaunchKernelGGL((k_bf16_tn<RT, C, KST>), grid, block, 0, st, A, lda, OUT, K, XT, ldx,    \
                         kchunk, tiles, nsplit, vec_ok, P, normp, To);                             \
    else                                                                                           \
      hipLaunchKernelGGL((k_bf16_nn<RT, C, D>), grid, block, 0, st, A, lda, OUT, K, XT, ldx,      \
                         kchunk, tiles, nsplit, vec_ok, P, normp, To, fold);                       \
    break;
  switch (LP / kTile) {
    SORSVD_BF(1, 4) SORSVD_BF(2, 4) SORSVD_BF(3, 4) SORSVD_BF(4, 4) SORSVD_BF(5, 3) SORSVD_BF(6, 3)
    SORSVD_BF(7, 3) SORSVD_BF(8, 3) SORSVD_BF(10, 2) SORSVD_BF(12, 2) SORSVD_BF(14, 2) SORSVD_BF(16, 2)
    default: return hipErrorInvalidValue;
  }
#undef SORSVD_BF
  return hipGetLastError();
}

hipError_t launch_bf16_pass(bool trans, const bf16_t* A, int64_t lda, int64_t OUT, int64_t K,
                            const bf16_t* XT, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                            float* P, double* normp, double* Tout, int fold, int rt, hipStream_t st) {
  switch (rt) {
    case 1: return launch_bf16_rt<1>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, P, normp, Tout, fold, st);
    case 2: return launch_bf16_rt<2>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, P, normp, Tout, fold, st);
    case 4: return launch_bf16_rt<4>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, P, normp, Tout, fold, st);
    default: return hipErrorInvalidValue;
  }
}

// Workgroups of a BF16 pass kernel that the current device holds at once
// (resident workgroups per CU times the CUs); 0 when no device answers.
template <int RT>
static int bf16_blocks_per_cu(bool trans, int CT) {
  constexpr int KST = RT >= 4 ? 64 : 128;
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SORSVD_BF(C, D)                                                                                       \
  case C:                                                                                                     \
    e = trans ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                 \
                    &nb, reinterpret_cast<const void*>(&k_bf16_tn<RT, C, KST>), 256, 0)                      \
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(                                                 \
                    &nb, reinterpret_cast<const void*>(&k_bf16_nn<RT, C, D>), 256, 0);                       \
    break;
  switch (CT) {
    SORSVD_BF(1, 4) SORSVD_BF(2, 4) SORSVD_BF(3, 4) SORSVD_BF(4, 4) SORSVD_BF(5, 3) SORSVD_BF(6, 3)
    SORSVD_BF(7, 3) SORSVD_BF(8, 3) SORSVD_BF(10, 2) SORSVD_BF(12, 2) SORSVD_BF(14, 2) SORSVD_BF(16, 2)
    default: break;
  }
#undef SORSVD_BF
  return e == hipSuccess ? nb : 0;
}

int bf16_slots(bool trans, int rt, int LP) {
  static std::mutex mu;
  static std::map<std::tuple<int, bool, int, int>, int> cache;
  if (LP % kTile || LP < kTile || (rt != 1 && rt != 2 && rt != 4)) return 0;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  std::lock_guard<std::mutex> g(mu);
  const auto key = std::make_tuple(dev, trans, rt, LP);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  const int CT = LP / kTile;
  const int nb = rt == 1 ? bf16_blocks_per_cu<1>(trans, CT)
                         : (rt == 2 ? bf16_blocks_per_cu<2>(trans, CT) : bf16_blocks_per_cu<4>(trans, CT));
  (void)hipGetLastError();
  const int slots = cus > 0 && nb > 0 ? cus * nb : 0;
  cache[key] = slots;
  return slots;
}

// contraction step of the bf16 kernels for a given rt (splits are multiples of it)
int bf16_step(bool trans, int rt) { return (trans && rt >= 4) ? 64 : 128; }

hipError_t launch_cast_bf16_t(const double* Q, int64_t rows, int LP, int64_t ldt, int permute,
                              int with_lo, bf16_t* QT, hipStream_t st) {
  const int64_t blocks = ceil_div(ldt, 64);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_bf16_t, dim3((unsigned)blocks), dim3(256), 0, st, Q, rows, LP, ldt,
                     permute, with_lo, QT);
  return hipGetLastError();
}

hipError_t launch_reduce_fold(const float* P, int64_t OUT, int LP2, int nsplit, double* out,
                              int64_t ldo, int ncols, hipStream_t st) {
  const int64_t total = OUT * (LP2 / 2);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_fold, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, P, OUT,
                     LP2, nsplit, out, ldo, ncols);
  return hipGetLastError();
}

}  // namespace sor
