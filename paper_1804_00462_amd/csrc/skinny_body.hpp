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
// Loads for the next step are issued before the MFMAs of the current one.
#pragma once
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


// Output: if Tout != null, out[r][c] -> Tout[r * ldo + c] in FP64 (c < LP);
// else -> P[r * LP + c] in the accumulator type (a partial sum). Tout may
// alias A (the in-place T <- T R^{-1}): the workgroup writes only its own
// output rows, after it has read all of its input rows. If nrm != null the
// FP64 sum of squares of the A elements this workgroup read is stored there.
// Xs: LDS of at least 4 VK (16 CT + 1) elements; red: LDS of 4 doubles.
template <typename T, bool TRANS, int RT, int CT>
__device__ inline void skinny_tile(const T* A, int64_t lda, int64_t OUT, int64_t k0, int64_t k1,
                                   const T* __restrict__ X, int64_t ldx, int64_t base, int vec_ok,
                                   typename Traits<T>::acc_t* P, double* Tout, int64_t ldo,
                                   double* nrm_out, T* Xs, double* red) {
  using Tr = Traits<T>;
  using accv = typename Tr::accv;
  constexpr int LP = CT * kTile;
  constexpr int VK = Tr::VK;
  constexpr int KS = 4 * VK;          // contraction indices per step
  constexpr int LPS = LP + 1;         // LDS row stride (odd: spreads the 4 lane groups over banks)
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
  auto load_x = [&](T (&xr)[XPT], int64_t kb) {
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int idx = threadIdx.x + 256 * i;
      const int r = idx / LP, c = idx % LP;
      const int64_t kk = kb + r;
      xr[i] = (kk < k1) ? X[kk * ldx + c] : T(0);
    }
  };

  T a[RT][VK];
  T xr[XPT];
  if (k0 < k1) { load_a(a, k0); load_x(xr, k0); }
  for (int64_t kb = k0; kb < k1; kb += KS) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < XPT; ++i) {
      const int idx = threadIdx.x + 256 * i;
      Xs[(idx / LP) * LPS + idx % LP] = xr[i];
    }
    __syncthreads();
    T an[RT][VK];
    const bool more = kb + KS < k1;
    if (more) { load_a(an, kb + KS); load_x(xr, kb + KS); }
    if (nrm_out) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int j = 0; j < VK; ++j) nrm += (double)a[rt][j] * (double)a[rt][j];
    }
#pragma unroll
    for (int j = 0; j < VK; ++j) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const T b = Xs[(VK * g + j) * LPS + ct * kTile + li];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) acc[rt][ct] = Tr::mfma(a[rt][j], b, acc[rt][ct]);
      }
    }
    if (more) {
#pragma unroll
      for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int j = 0; j < VK; ++j) a[rt][j] = an[rt][j];
    }
  }

#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t orow = base + (int64_t)(w * RT + rt) * kTile + Tr::out_row(l, r);
        if (orow < OUT) {
          if (Tout) Tout[orow * ldo + ct * kTile + li] = (double)acc[rt][ct][r];
          else P[orow * LP + ct * kTile + li] = acc[rt][ct][r];
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
