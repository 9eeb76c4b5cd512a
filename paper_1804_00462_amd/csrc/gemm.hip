// Streaming skinny products over A: the passes of SOR-SVD.
//
//   NN:  P_s = A[:, K_s] X[K_s, :]      (T1 = A Omega, eq. T1; T1 = A T2 and
//                                         the A Q2 half of eq. M in Alg. 4)
//   TN:  P_s = A[K_s, :]^T Y[K_s, :]    (T2 = A^T T1, eq. AT1; Alg. 4's T2 update)
//
// A is row-major (lda); the skinny operand is K x LP row-major (LP = the
// sketch width rounded up to the 16-wide MFMA tile, padding columns zero).
// The contraction is split into `nsplit` chunks; each workgroup owns 64*RT
// output rows (rows of A for NN, columns of A for TN) and ALL LP output
// columns, so every element of A is read from HBM exactly once per pass.
// Partials P_s are summed afterwards in a fixed order (deterministic, no
// atomics).
//
// Per workgroup: 4 waves; each wave keeps RT x CT accumulator tiles (16x16).
// A fragments go straight from HBM to registers (lane l takes output row
// l % 16 and a run of VK consecutive contraction indices starting at
// VK * (l / 16)); the skinny operand is staged in LDS and read as the MFMA B
// operand. Both operands use the same lane -> contraction-index map, so any
// permutation of the contraction inside a step is harmless. Loads for the next
// step are issued before the MFMAs of the current one.
//
// P may alias A (the in-place T <- T R^{-1} of the QR step): a workgroup
// writes only its own output rows, after it has read all of its input rows.
//
// Workgroups are renumbered so that each of the 8 XCDs receives a contiguous
// run of (split, tile) pairs: workgroups on one XCD mostly share one split,
// i.e. one slab of the skinny operand, which then stays in that XCD's L2.
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
    const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) { double2 v = q[i]; a[2 * i] = v.x; a[2 * i + 1] = v.y; }
  }
};
template <> struct VecLoad<float, 8> {
  __device__ static inline void run(const float* p, float (&a)[8]) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      float4 v = q[i];
      a[4 * i] = v.x; a[4 * i + 1] = v.y; a[4 * i + 2] = v.z; a[4 * i + 3] = v.w;
    }
  }
};

__device__ inline int xcd_remap(int b, int nb) {
  return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

template <typename T, bool TRANS, int RT, int CT>
__global__ void __launch_bounds__(256, 2)
k_skinny(const T* A, int64_t lda, int64_t OUT, int64_t K,
         const T* __restrict__ X, int64_t ldx, int64_t kchunk, int tiles, int nsplit,
         int vec_ok, typename Traits<T>::acc_t* P, double* __restrict__ normp,
         const int* __restrict__ skipflag) {
  if (skipflag && *skipflag) return;  // product not needed (see the Cholesky QR step)
  using Tr = Traits<T>;
  using accv = typename Tr::accv;
  constexpr int LP = CT * kTile;
  constexpr int VK = Tr::VK;
  constexpr int KS = 4 * VK;          // contraction indices per step
  constexpr int LPS = LP + 1;         // LDS row stride (odd: spreads the 4 lane groups over banks)
  constexpr int XPT = KS * LP / 256;  // skinny-operand elements staged per thread per step
  __shared__ T Xs[KS * LPS];
  __shared__ double red[4];

  const int nb = tiles * nsplit;
  const int v = xcd_remap((int)blockIdx.x, nb);
  const int s = v / tiles, tile = v % tiles;
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int g = l / kTile, li = l % kTile;
  const int64_t k0 = (int64_t)s * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  const int64_t base = (int64_t)tile * (64 * RT);

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
    if (normp) {
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
        if (orow < OUT) P[((int64_t)s * OUT + orow) * LP + ct * kTile + li] = acc[rt][ct][r];
      }
    }
  }
  if (normp) {
    nrm = wave_sum(nrm);
    if (l == 0) red[w] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) normp[v] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// out[r][c] = sum_{s = 0..nsplit-1} P[s][r][c] in FP64, for c < ncols, in a
// fixed order: lane t of an 8-lane group sums s = t, t + 8, ... in turn, then
// the 8 lane sums are combined by a fixed DPP tree.
template <typename Acc>
__global__ void __launch_bounds__(256)
k_reduce(const Acc* __restrict__ P, int64_t OUT, int LP, int nsplit, double* __restrict__ out,
         int64_t ldo, int ncols) {
  const int64_t total = OUT * LP;
  const int64_t idx = (int64_t)blockIdx.x * 32 + threadIdx.x / 8;
  const int ln = threadIdx.x % 8;
  double acc = 0.0;
  if (idx < total)
    for (int s = ln; s < nsplit; s += 8) acc += (double)P[(int64_t)s * total + idx];
  acc = sum8(acc);
  if (idx < total && ln == 0) {
    const int64_t r = idx / LP;
    const int c = (int)(idx % LP);
    if (c < ncols) out[r * ldo + c] = acc;
  }
}

// dst[r][c] = src[r][c] for c < cols, 0 for cols <= c < LP (row-major, element type T).
template <typename T>
__global__ void __launch_bounds__(256)
k_pack(const double* __restrict__ src, int64_t rows, int cols, int64_t lds, T* __restrict__ dst, int LP) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * LP) return;
  const int64_t r = idx / LP;
  const int c = (int)(idx % LP);
  dst[idx] = c < cols ? (T)src[r * lds + c] : T(0);
}

// Skinny operand of the next pass in A's compute type (row-major rows x LP).
__global__ void __launch_bounds__(256)
k_cast_f32(const double* __restrict__ Q, int64_t n_elem, float* __restrict__ Xc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx < n_elem) Xc[idx] = (float)Q[idx];
}

// Clear the strict lower triangle of an l x l row-major matrix.
__global__ void __launch_bounds__(256) k_zero_lower(double* __restrict__ R, int l) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx < l * l && idx % l < idx / l) R[idx] = 0.0;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_zero_lower(double* R, int l, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_lower, dim3((unsigned)ceil_div((int64_t)l * l, 256)), dim3(256), 0, st, R, l);
  return hipGetLastError();
}

template <typename T, bool TRANS, int RT>
static hipError_t launch_ct(int CT, const T* A, int64_t lda, int64_t OUT, int64_t K, const T* X,
                            int64_t ldx, int64_t kchunk, int tiles, int nsplit, int vec_ok,
                            typename Traits<T>::acc_t* P, double* normp, const int* skipflag,
                            hipStream_t st) {
  dim3 grid((unsigned)(tiles * nsplit)), block(256);
#define SORSVD_CASE(C)                                                                           \
  case C:                                                                                        \
    hipLaunchKernelGGL((k_skinny<T, TRANS, RT, C>), grid, block, 0, st, A, lda, OUT, K, X, ldx, \
                       kchunk, tiles, nsplit, vec_ok, P, normp, skipflag);                       \
    break;
  switch (CT) {
    SORSVD_CASE(1) SORSVD_CASE(2) SORSVD_CASE(3) SORSVD_CASE(4)
    SORSVD_CASE(5) SORSVD_CASE(6) SORSVD_CASE(7) SORSVD_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef SORSVD_CASE
  return hipGetLastError();
}

// Output rows per workgroup (64 * RT): FP32 always uses RT = 2; FP64 uses
// RT = 2 only when one workgroup then covers all output rows (the l x l Gram
// and projection products), so the tall operand is read once.
template <typename T> constexpr bool has_rt1() { return true; }
template <> constexpr bool has_rt1<float>() { return false; }

int skinny_rt(int a_type, int64_t OUT) { return (a_type == 1 || OUT <= 128) ? 2 : 1; }

template <typename T, int RT>
static hipError_t launch_rt(bool trans, const T* A, int64_t lda, int64_t OUT, int64_t K, const T* X,
                            int64_t ldx, int LP, int64_t kchunk, int nsplit,
                            typename Traits<T>::acc_t* P, double* normp, const int* skipflag,
                            hipStream_t st) {
  const int tiles = (int)ceil_div(OUT, 64 * RT);
  if (tiles == 0 || nsplit == 0) return hipSuccess;
  const int vec_ok = ((lda * (int64_t)sizeof(T)) % 16 == 0) && (((uintptr_t)A) % 16 == 0);
  if (trans)
    return launch_ct<T, true, RT>(LP / kTile, A, lda, OUT, K, X, ldx, kchunk, tiles, nsplit, vec_ok, P, normp, skipflag, st);
  return launch_ct<T, false, RT>(LP / kTile, A, lda, OUT, K, X, ldx, kchunk, tiles, nsplit, vec_ok, P, normp, skipflag, st);
}

template <typename T>
hipError_t launch_skinny(bool trans, const T* A, int64_t lda, int64_t OUT, int64_t K, const T* X,
                         int64_t ldx, int LP, int64_t kchunk, int nsplit,
                         typename Traits<T>::acc_t* P, double* normp, const int* skipflag,
                         hipStream_t st) {
  if constexpr (has_rt1<T>()) {
    if (OUT > 128)
      return launch_rt<T, 1>(trans, A, lda, OUT, K, X, ldx, LP, kchunk, nsplit, P, normp, skipflag, st);
  }
  return launch_rt<T, 2>(trans, A, lda, OUT, K, X, ldx, LP, kchunk, nsplit, P, normp, skipflag, st);
}

hipError_t launch_skinny_f64(bool trans, const double* A, int64_t lda, int64_t OUT, int64_t K,
                             const double* X, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                             double* P, double* normp, const int* skipflag, hipStream_t st) {
  return launch_skinny<double>(trans, A, lda, OUT, K, X, ldx, LP, kchunk, nsplit, P, normp, skipflag, st);
}

hipError_t launch_skinny_f32(bool trans, const float* A, int64_t lda, int64_t OUT, int64_t K,
                             const float* X, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                             float* P, double* normp, const int* skipflag, hipStream_t st) {
  return launch_skinny<float>(trans, A, lda, OUT, K, X, ldx, LP, kchunk, nsplit, P, normp, skipflag, st);
}

int skinny_rows_per_block(int a_type, int64_t OUT) { return 64 * skinny_rt(a_type, OUT); }
int skinny_step(int a_type) { return a_type == 0 ? 32 : (a_type == 1 ? 32 : 128); }

hipError_t launch_reduce_f64(const double* P, int64_t OUT, int LP, int nsplit, double* out,
                             int64_t ldo, int ncols, hipStream_t st) {
  const int64_t total = OUT * LP;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL((k_reduce<double>), dim3((unsigned)ceil_div(total, 32)), dim3(256), 0, st,
                     P, OUT, LP, nsplit, out, ldo, ncols);
  return hipGetLastError();
}

hipError_t launch_reduce_f32(const float* P, int64_t OUT, int LP, int nsplit, double* out,
                             int64_t ldo, int ncols, hipStream_t st) {
  const int64_t total = OUT * LP;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL((k_reduce<float>), dim3((unsigned)ceil_div(total, 32)), dim3(256), 0, st,
                     P, OUT, LP, nsplit, out, ldo, ncols);
  return hipGetLastError();
}

hipError_t launch_pack_f64(const double* src, int64_t rows, int cols, int64_t lds, double* dst,
                           int LP, hipStream_t st) {
  if (rows * LP == 0) return hipSuccess;
  hipLaunchKernelGGL((k_pack<double>), dim3((unsigned)ceil_div(rows * LP, 256)), dim3(256), 0, st,
                     src, rows, cols, lds, dst, LP);
  return hipGetLastError();
}

hipError_t launch_pack_f32(const double* src, int64_t rows, int cols, int64_t lds, float* dst,
                           int LP, hipStream_t st) {
  if (rows * LP == 0) return hipSuccess;
  hipLaunchKernelGGL((k_pack<float>), dim3((unsigned)ceil_div(rows * LP, 256)), dim3(256), 0, st,
                     src, rows, cols, lds, dst, LP);
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double* Q, int64_t n_elem, float* Xc, hipStream_t st) {
  if (n_elem == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cast_f32, dim3((unsigned)ceil_div(n_elem, 256)), dim3(256), 0, st, Q, n_elem, Xc);
  return hipGetLastError();
}

}  // namespace sor
