// Tile body of the streaming skinny products over A (shared by the
// single-problem kernels and the persistent batched kernels).
//
//   NN:  out = A[:, k0:k1] X[k0:k1, :]      TN:  out = A[k0:k1, :]^T Y[k0:k1, :]
//
// A is row-major (lda); the skinny operand is K x LP row-major (LP = 16 CT,
// padding columns zero). One workgroup of 4 waves owns 64 RT output rows
// (rows of A for NN, columns of A for TN) and all LP output columns, so every
// element of A is read from HBM once per pass. Each wave keeps RT x CT
// accumulator tiles (16 x 16). A fragments go straight from HBM to registers
// (lane l takes output row l % 16 and a run of VK consecutive contraction
// indices starting at VK * (l / 16)); the skinny operand is staged in LDS and
// read as the MFMA B operand. Both operands use the same lane -> contraction
// map, so any permutation of the contraction inside a step is harmless.
// Loads for later steps are issued before the MFMAs of the current one.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace sor {

template <typename T> struct Traits;

template <> struct Traits<double> {
  using acc_t = double;
  using accv = f64x4;
  static constexpr int VK = 8;
  __device__ static inline accv mfma(double a, double b, accv c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // lane l, register r of the 16x16 result tile holds row out_row(l, r), column l % 16
  __device__ static inline int out_row(int l, int r) { return 4 * r + l / 16; }
};

template <> struct Traits<float> {
  using acc_t = float;
  using accv = f32x4;
  static constexpr int VK = 8;
  __device__ static inline accv mfma(float a, float b, accv c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int l, int r) { return 4 * (l / 16) + r; }
};

template <typename T, int N> struct VecLoad;
template <> struct VecLoad<double, 8> {
  __device__ static inline void run(const double* p, double (&a)[8]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 v = load_stream16(p + 2 * i);
      a[2 * i] = __hiloint2double((int)v.y, (int)v.x);
      a[2 * i + 1] = __hiloint2double((int)v.w, (int)v.z);
    }
  }
};
template <> struct VecLoad<float, 8> {
  __device__ static inline void run(const float* p, float (&a)[8]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint4 v = load_stream16(p + 4 * i);
      a[4 * i] = __uint_as_float(v.x); a[4 * i + 1] = __uint_as_float(v.y);
      a[4 * i + 2] = __uint_as_float(v.z); a[4 * i + 3] = __uint_as_float(v.w);
    }
  }
};

__device__ inline int xcd_remap(int b, int nb) {
  return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

// Workgroup b of nb, dispatched to XCD b % 8, takes logical index v from a
// contiguous range per XCD (any nb): XCD x receives nb / 8 workgroups, plus
// one when x < nb % 8, and numbers them in dispatch order. Logical neighbours
// therefore run on the same XCD at about the same time and share its L2.
__device__ inline int xcd_remap_any(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}


// LDS of the staged skinny operand: two buffers (the next step's rows are
// stored while the current ones feed the MFMAs) of KS rows, row stride LP + 2.
// With that stride the four 16-lane groups of a B-operand read, whose rows lie
// VK apart, start 16 banks apart, so each 32-lane half of the wave hits 32
// distinct banks.
template <typename T, int CT>
constexpr int xs_elems() { return 2 * 4 * Traits<T>::VK * (CT * kTile + 2); }

// Output: if Tout != null, out[r][c] -> Tout[r * ldo + c] in FP64 (c < LP);
// else -> P[r * ldp + c] in the accumulator type (a partial sum). Tout may
// alias A (the in-place T <- T R^{-1}): the workgroup writes only its own
// output rows, after it has read all of its input rows. If nrm != null the
// FP64 sum of squares of the A elements this workgroup read is stored there.
// Xs: LDS of xs_elems<T, CT>() elements; red: LDS of 4 doubles.
// PD: A fragments are loaded PD steps ahead (1 or 2). tri (FP64 NN only): X is
// upper triangular (X[k][c0 + c] = 0 for k > c0 + c, as R^{-1}, where X is
// the column block starting at column c0 of the whole operand), so the MFMAs
// of a step whose contraction indices all lie below a 16-column output tile
// are skipped (their products are exact zeros). tri = 2 (FP64 A^T A, X = A):
// only the upper triangle of the product is wanted (the Cholesky factor reads
// no other), so the MFMAs of the 16 x 16 output tiles wholly below the
// diagonal are skipped and those tiles are left zero. ldp: row stride of the
// partial sums P (the width of the whole output when X is one column block).
// Epi (optional): called as epi(orow, c, value) for every output row orow <
// OUT and column c of the tile instead of storing it (Tout and P unused).
struct NoEpi {
  __device__ void operator()(int64_t, int, double) const {}
};

template <typename T, bool TRANS, int RT, int CT, int PD = (sizeof(T) == 4 ? 2 : 1), typename Epi = NoEpi>
__device__ __attribute__((always_inline)) inline void skinny_tile(const T* A, int64_t lda, int64_t OUT, int64_t k0, int64_t k1,
                                   const T* __restrict__ X, int64_t ldx, int64_t base, int vec_ok,
                                   typename Traits<T>::acc_t* P, double* Tout, int64_t ldo,
                                   double* nrm_out, T* Xs, double* red, int tri = 0,
                                   int64_t ldp = CT * kTile, int64_t c0 = 0, Epi* epi = nullptr) {
  using Tr = Traits<T>;
  using accv = typename Tr::accv;
  constexpr int LP = CT * kTile;
  constexpr int VK = Tr::VK;
  constexpr int KS = 4 * VK;          // contraction indices per step
  constexpr int LPS = LP + 2;         // LDS row stride (see xs_elems)
  constexpr int XPT = KS * LP / 256;  // skinny-operand elements staged per thread per step
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int g = l / kTile, li = l % kTile;

  accv acc[RT][CT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = accv{0, 0, 0, 0};
  double nrm = 0.0;

  auto load_a = [&](T (&a)[RT][VK], int64_t kb) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int64_t orow = base + (int64_t)(w * RT + rt) * kTile + li;
      const int64_t kk0 = kb + VK * g;
      if (!TRANS) {
        if (orow < OUT && kk0 + VK <= k1 && vec_ok) {
          VecLoad<T, VK>::run(A + orow * lda + kk0, a[rt]);
        } else {
#pragma unroll
          for (int j = 0; j < VK; ++j)
            a[rt][j] = (orow < OUT && kk0 + j < k1) ? A[orow * lda + kk0 + j] : T(0);
        }
      } else {
#pragma unroll
        for (int j = 0; j < VK; ++j)
          a[rt][j] = (orow < OUT && kk0 + j < k1) ? A[(kk0 + j) * lda + orow] : T(0);
      }
    }
  };
  // Skinny rows of a step: thread t stages row t / 8 of it, columns
  // (t % 8) XPT .. + XPT - 1, so one base address serves all of a thread's
  // loads and LDS stores (per-element addresses cost ~60 registers). Rows
  // past k1 (last step only) are read clamped and stored as zeros.
  static_assert(KS * 8 == 256 && XPT * 8 == LP, "one row of the step per 8 threads");
  const int xrow = threadIdx.x / 8, xcol = (threadIdx.x % 8) * XPT;
  auto load_x = [&](T (&xr)[XPT], int64_t kb) {
    const int64_t kk = kb + xrow;
    const T* src = X + (kk < k1 ? kk : k1 - 1) * ldx + xcol;
#pragma unroll
    for (int i = 0; i < XPT; ++i) xr[i] = src[i];
  };
  auto store_x = [&](const T (&xr)[XPT], T* buf, int64_t kb) {
    const bool in = kb + xrow < k1;
    T* dst = buf + xrow * LPS + xcol;
#pragma unroll
    for (int i = 0; i < XPT; ++i) dst[i] = in ? xr[i] : T(0);
  };

  // A fragments PD steps ahead (FP32 by default two, to cover the HBM latency
  // under load with the MFMA time of one step; FP64 one, for the registers)
  static_assert(PD == 1 || PD == 2, "prefetch depth");
  T a[RT][VK];
  T an[RT][VK];
  T xr[XPT];
  T* xb = Xs;                  // rows of the current step
  T* xn = Xs + KS * LPS;       // rows of the next step
  __syncthreads();             // LDS may still be read by the previous tile of a persistent loop
  if (k0 < k1) {
    load_a(a, k0);
    load_x(xr, k0);
    store_x(xr, xb, k0);
    if (PD == 2 && k0 + KS < k1) load_a(an, k0 + KS);
  }
  __syncthreads();
  for (int64_t kb = k0; kb < k1; kb += KS) {
    T an2[RT][VK];
    const bool more = kb + KS < k1;
    if (PD == 2) {
      // the X rows of the next step first: waiting for them below does not
      // wait for the A fragments two steps ahead
      if (more) load_x(xr, kb + KS);
      if (kb + 2 * KS < k1) load_a(an2, kb + 2 * KS);
    } else if (more) {
      load_a(an, kb + KS);
      load_x(xr, kb + KS);
    }
    if (nrm_out) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int j = 0; j < VK; ++j) nrm += (double)a[rt][j] * (double)a[rt][j];
    }
    // B fragments of contraction index j + 1 are read from LDS while the
    // MFMAs of index j run (the scheduling barriers keep the reads ahead of
    // the MFMAs instead of next to their uses, where the LDS latency would
    // stall the matrix pipe between every few MFMAs)
    T bq[2][CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) bq[0][ct] = xb[(VK * g) * LPS + ct * kTile + li];
#pragma unroll
    for (int j = 0; j < VK; ++j) {
      if (j + 1 < VK) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) bq[(j + 1) & 1][ct] = xb[(VK * g + j + 1) * LPS + ct * kTile + li];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        if constexpr (sizeof(T) == 8 && !TRANS)
          if (tri && kb - c0 >= (int64_t)(ct + 1) * kTile) continue;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
          // (tri = 2, A^T A: the 16 x 16 output tiles wholly below the
          // diagonal are not formed; only the upper triangle is read)
          if constexpr (sizeof(T) == 8 && TRANS)
            if (tri == 2 && c0 + (int64_t)(ct + 1) * kTile <= base + (int64_t)(w * RT + rt) * kTile) continue;
          acc[rt][ct] = Tr::mfma(a[rt][j], bq[j & 1][ct], acc[rt][ct]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (more) {
      // the other buffer was last read in the previous step, which every wave
      // finished before the barrier that ended it
      store_x(xr, xn, kb + KS);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int j = 0; j < VK; ++j) {
          a[rt][j] = an[rt][j];
          if (PD == 2) an[rt][j] = an2[rt][j];
        }
    }
    __syncthreads();  // the next step's rows are in LDS; the current ones may be overwritten
    T* t = xb;
    xb = xn;
    xn = t;
  }

#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = base + (int64_t)(w * RT + rt) * kTile + Tr::out_row(l, r);
        if (orow < OUT) {
          if constexpr (!std::is_same<Epi, NoEpi>::value) (*epi)(orow, ct * kTile + li, (double)acc[rt][ct][r]);
          else if (Tout) Tout[orow * ldo + ct * kTile + li] = (double)acc[rt][ct][r];
          else P[orow * ldp + ct * kTile + li] = acc[rt][ct][r];
        }
      }
    }
  }
  if (nrm_out) {
    nrm = wave_sum(nrm);
    __syncthreads();
    if (l == 0) red[w] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) *nrm_out = (red[0] + red[1]) + (red[2] + red[3]);
  }
  __syncthreads();  // LDS is reused by the next tile of a persistent loop
}

}  // namespace sor
