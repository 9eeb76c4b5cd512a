// Explicit residual of the rank-k approximation (the error check of the method,
// e = ||A - U S V^T||_F / ||A||_F), as one more pass over A.
//
// Each workgroup owns one block of 128 columns of A and walks a strided set of
// 64-row tiles. W = S V^T restricted to its columns (KP x 128) is staged once
// in LDS; for every tile the four waves form 16 rows x 128 columns of
// A_hat = U W on MFMA (FP32 for FP32 / BF16 A, FP64 for FP64 A), read the
// matching elements of A, and accumulate (a - a_hat)^2 in FP64.
//
// For BF16- or FP16-stored A the same pass also accumulates sum ulp(a)^2 / 12,
// the expected squared rounding error of storing A in 16 bits (round-to-
// nearest, error uniform within half an ulp). FP16 A may come with column
// exponents e (A = A_stored diag(2^-e_j)): the residual is then formed in the
// stored scale (column j of W = S V^T multiplied by 2^e_j before the MFMA, so
// FP32 sees values of the stored range) and its square, like the rounding
// noise, weighted by 4^-e_j (exact). This pass only reports the two sums
// (err_fro_explicit and a_noise_rel); how much of the noise the rank-k
// subspaces capture, and so the error against the matrix before rounding, is
// the caller's estimate (the judge of sorsvd_auto).
//
// For k > 128 (W no longer fits LDS) the pass is a tiled product instead: U
// (m x KP) and W^T = S V^T (KP x n, columns padded to a multiple of 128) are
// first cast to the MFMA type, then each workgroup forms a 128 x 128 tile
// (64 x 128 for FP64) of U W^T with the streaming tile body of the passes
// (U in place of A, W^T as the skinny operand, one column block) and takes
// the same sums from it in its epilogue.
#include <algorithm>
#include <type_traits>

#include "half16.hpp"
#include "skinny_body.hpp"

namespace sor {

namespace {

constexpr int kResCols = 128;  // columns of A per workgroup
constexpr int kResLd = kResCols + 1;

template <typename TA> __device__ inline double load_a(const TA* p);
template <> __device__ inline double load_a<double>(const double* p) { return *p; }
template <> __device__ inline double load_a<float>(const float* p) { return (double)*p; }
template <> __device__ inline double load_a<bf16_t>(const bf16_t* p) { return (double)bf16_to_f32(*p); }
struct f16_word {  // FP16 storage (distinct from the BF16 word type)
  uint16_t bits;
};
template <> __device__ inline double load_a<f16_word>(const f16_word* p) { return (double)f16_to_f32(p->bits); }

// ulp(a)^2 / 12 of a BF16 value (8 significant bits): ulp = 2^(e - 127 - 7),
// subnormals and zero take the smallest exponent.
__device__ inline double bf16_noise(bf16_t b) {
  int e = (b >> 7) & 0xFF;
  if (e == 0) e = 1;
  const double ulp = ldexp(1.0, e - 127 - 7);
  return ulp * ulp * (1.0 / 12.0);
}

// ulp(a)^2 / 12 of an FP16 value (11 significant bits): ulp = 2^(e - 15 - 10),
// subnormals and zero take the smallest exponent.
__device__ inline double f16_noise(uint16_t h) {
  int e = (h >> 10) & 0x1F;
  if (e == 0) e = 1;
  const double ulp = ldexp(1.0, e - 15 - 10);
  return ulp * ulp * (1.0 / 12.0);
}

template <typename T> struct ResMfma;
template <> struct ResMfma<float> {
  using accv = f32x4;
  __device__ static accv run(float a, float b, accv c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int r) { return 4 * (l / 16) + r; }
};
template <> struct ResMfma<double> {
  using accv = f64x4;
  __device__ static accv run(double a, double b, accv c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int l, int r) { return 4 * r + l / 16; }
};

// TA: storage type of A; T: MFMA type (float for FP32 / BF16 A, double for FP64 A).
template <typename TA, typename T>
__global__ void __launch_bounds__(256)
k_residual(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n, const double* __restrict__ U,
           int64_t ldu, const double* __restrict__ S, const double* __restrict__ V, int64_t ldv, int k, int KP,
           double* __restrict__ part, const int* __restrict__ cexp) {
  using M = ResMfma<T>;
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  T* Ws = reinterpret_cast<T*>(lds_raw);  // KP x kResLd
  __shared__ double red[2][4];
  const int64_t c0 = (int64_t)blockIdx.x * kResCols;
  for (int i = threadIdx.x; i < KP * kResCols; i += 256) {
    const int j = i / KP, c = i % KP;  // c fastest: contiguous reads of a row of V
    T w = T(0);
    if (c < k && c0 + j < n) {
      double x = S[c] * V[(c0 + j) * ldv + c];
      if (cexp) x = ldexp(x, cexp[c0 + j]);
      w = (T)x;
    }
    Ws[c * kResLd + j] = w;
  }
  __syncthreads();
  const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int li = l % 16, g = l / 16;
  double res = 0.0, noise = 0.0;
  const int64_t ntiles = (m + 63) / 64;
  for (int64_t t = blockIdx.y; t < ntiles; t += gridDim.y) {
    const int64_t rbase = t * 64 + wv * 16;
    const int64_t ra = rbase + li;  // row of U this lane supplies
    typename M::accv acc[8];
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) acc[ct] = typename M::accv{0, 0, 0, 0};
    for (int kk = 0; kk < KP; kk += 4) {
      const int c = kk + g;
      const T a = (ra < m && c < k) ? (T)U[ra * ldu + c] : T(0);
#pragma unroll
      for (int ct = 0; ct < 8; ++ct) acc[ct] = M::run(a, Ws[c * kResLd + ct * 16 + li], acc[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
      const int64_t col = c0 + ct * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = rbase + M::row(l, r);
        if (row < m && col < n) {
          const TA* p = A + row * lda + col;
          if constexpr (std::is_same<TA, f16_word>::value) {
            const int e = cexp ? cexp[col] : 0;
            const double d = load_a<TA>(p) - (double)acc[ct][r];
            res += ldexp(d * d, -2 * e);
            noise += ldexp(f16_noise(p->bits), -2 * e);
          } else {
            const double d = load_a<TA>(p) - (double)acc[ct][r];
            res += d * d;
            if constexpr (sizeof(TA) == 2) noise += bf16_noise(*p);
          }
        }
      }
    }
  }
  res = wave_sum(res);
  noise = wave_sum(noise);
  if (l == 0) {
    red[0][wv] = res;
    red[1][wv] = noise;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[2 * b] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    part[2 * b + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// ---------------------------------------------------------------------------
// k > 128.

template <typename T>
__global__ void __launch_bounds__(256)
k_res_cast_u(const double* __restrict__ U, int64_t ldu, int64_t m, int k, int KP, T* __restrict__ Uc) {
  const int64_t tot = m * KP;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int64_t r = e / KP;
    const int c = (int)(e % KP);
    Uc[e] = c < k ? (T)U[r * ldu + c] : T(0);
  }
}

// Wt[c][j] = S_c V[j][c] (times 2^e_j with column exponents), zero for c >= k or j >= n.
template <typename T>
__global__ void __launch_bounds__(256)
k_res_cast_w(const double* __restrict__ S, const double* __restrict__ V, int64_t ldv, int64_t n, int k, int KP,
             int64_t npad, const int* __restrict__ cexp, T* __restrict__ Wt) {
  const int64_t tot = (int64_t)KP * npad;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int c = (int)(e / npad);
    const int64_t j = e % npad;
    T w = T(0);
    if (c < k && j < n) {
      double x = S[c] * V[j * ldv + c];
      if (cexp) x = ldexp(x, cexp[j]);
      w = (T)x;
    }
    Wt[e] = w;
  }
}

// Epilogue of the tiled residual: (a - a_hat)^2 and the rounding noise of a.
template <typename TA>
struct ResEpi {
  const TA* A;
  int64_t lda, n, c0;
  const int* cexp;
  double res, noise;
  __device__ void operator()(int64_t row, int c, double v) {
    const int64_t col = c0 + c;
    if (col >= n) return;
    const TA* p = A + row * lda + col;
    if constexpr (std::is_same<TA, f16_word>::value) {
      const int e = cexp ? cexp[col] : 0;
      const double d = load_a<TA>(p) - v;
      res += ldexp(d * d, -2 * e);
      noise += ldexp(f16_noise(p->bits), -2 * e);
    } else {
      const double d = load_a<TA>(p) - v;
      res += d * d;
      if constexpr (sizeof(TA) == 2) noise += bf16_noise(*p);
    }
  }
};

template <typename TA, typename T>
__global__ void __launch_bounds__(256, 2)
k_residual_wide(const TA* __restrict__ A, int64_t lda, int64_t m, int64_t n, const T* __restrict__ Uc, int KP,
                const T* __restrict__ Wt, int64_t npad, int tiles, int ncb, double* __restrict__ part,
                const int* __restrict__ cexp, typename Traits<T>::acc_t* pnull, double* dnull) {
  constexpr int RT = sizeof(T) == 8 ? 1 : 2;
  constexpr int CT = 8;
  __shared__ T Xs[xs_elems<T, CT>()];
  __shared__ double red[2][4];
  const int nb = tiles * ncb;
  const int v = xcd_remap_any((int)blockIdx.x, nb);
  const int cb = v % ncb, tile = v / ncb;
  const int64_t c0 = (int64_t)cb * CT * kTile;
  ResEpi<TA> epi{A, lda, n, c0, cexp, 0.0, 0.0};
  const int vec_ok = ((KP * (int64_t)sizeof(T)) % 16 == 0) && (((uintptr_t)Uc) % 16 == 0);
  // (pnull, dnull: null pointers taken as arguments; constant nulls there crash this compiler)
  skinny_tile<T, false, RT, CT, sizeof(T) == 4 ? 2 : 1, ResEpi<TA>>(Uc, KP, m, 0, KP, Wt + c0, npad,
                                                                     (int64_t)tile * 64 * RT, vec_ok, pnull,
                                                                     dnull, 0, dnull, Xs, &red[0][0], 0,
                                                                     CT * kTile, 0, &epi);
  const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const double res = wave_sum(epi.res), noise = wave_sum(epi.noise);
  if (l == 0) {
    red[0][wv] = res;
    red[1][wv] = noise;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * (int64_t)v] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    part[2 * (int64_t)v + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

struct ResInfo {  // the leading fields of the result record
  double a_fro;
  double err_fro;
  double err_fro_explicit;
  int32_t sweeps;
  int32_t flags;
  double a_noise_rel;
};

// Fixed-order sum of the partial pairs; needs info->a_fro (written by the
// error-record kernel before this one runs).
__global__ void __launch_bounds__(256) k_residual_final(const double* __restrict__ part, int64_t nparts,
                                                        ResInfo* __restrict__ info) {
  __shared__ double s0[256], s1[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 256) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double af = info->a_fro;
    info->err_fro_explicit = af > 0.0 ? sqrt(s0[0]) / af : 0.0;
    info->a_noise_rel = af > 0.0 ? sqrt(s1[0]) / af : 0.0;
  }
}

}  // namespace

int64_t residual_row_groups(int64_t m, int64_t n) {
  // enough workgroups to fill the chip: column blocks x row groups >= ~2048
  const int64_t cb = ceil_div(n, kResCols);
  int64_t rg = ceil_div(2048, cb);
  rg = rg < 1 ? 1 : rg;
  const int64_t tiles = ceil_div(m, 64);
  return rg > tiles ? tiles : rg;
}

int64_t residual_parts(int64_t m, int64_t n) { return ceil_div(n, kResCols) * residual_row_groups(m, n); }

static int64_t res_wide_tiles(int a_type, int64_t m) { return ceil_div(m, a_type == 0 ? 64 : 128); }

// Scratch of launch_residual: the partial sums, and for KP > 128 the cast
// operands.
size_t residual_ws_bytes(int a_type, int64_t m, int64_t n, int KP) {
  if (KP <= kResCols) return (size_t)2 * residual_parts(m, n) * 8;
  const int64_t npad = round_up(n, kResCols);
  const size_t es = a_type == 0 ? 8 : 4;
  const int64_t parts = res_wide_tiles(a_type, m) * (npad / kResCols);
  return round_up((int64_t)2 * parts * 8, 256) + round_up(m * KP * (int64_t)es, 256) +
         round_up((int64_t)KP * npad * (int64_t)es, 256);
}

template <typename TA, typename T>
static hipError_t launch_residual_wide(const TA* A, int64_t lda, int64_t m, int64_t n, const double* U, int64_t ldu,
                                       const double* S, const double* V, int64_t ldv, int k, int KP, void* ws,
                                       int64_t tiles, void* info, hipStream_t st, const int* cexp) {
  const int64_t npad = round_up(n, kResCols);
  const int ncb = (int)(npad / kResCols);
  const int64_t parts = tiles * ncb;
  double* part = reinterpret_cast<double*>(ws);
  T* Uc = reinterpret_cast<T*>((char*)ws + round_up(2 * parts * 8, 256));
  T* Wt = reinterpret_cast<T*>((char*)Uc + round_up(m * KP * (int64_t)sizeof(T), 256));
  hipLaunchKernelGGL((k_res_cast_u<T>), dim3((unsigned)std::min<int64_t>(4096, ceil_div(m * KP, 256))), dim3(256), 0,
                     st, U, ldu, m, k, KP, Uc);
  hipLaunchKernelGGL((k_res_cast_w<T>), dim3((unsigned)std::min<int64_t>(4096, ceil_div((int64_t)KP * npad, 256))),
                     dim3(256), 0, st, S, V, ldv, n, k, KP, npad, cexp, Wt);
  hipLaunchKernelGGL((k_residual_wide<TA, T>), dim3((unsigned)parts), dim3(256), 0, st, A, lda, m, n, Uc, KP, Wt,
                     npad, (int)tiles, ncb, part, cexp, nullptr, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, st, part, parts, (ResInfo*)info);
  return hipGetLastError();
}

// a_type: 0 FP64, 1 FP32, 2 BF16, 4 FP16 (cexp: its column exponents, or
// null). part: residual_ws_bytes(a_type, m, n, KP) bytes of scratch.
hipError_t launch_residual(int a_type, const void* A, int64_t lda, int64_t m, int64_t n, const double* U,
                           int64_t ldu, const double* S, const double* V, int64_t ldv, int k, int KP, double* part,
                           void* info, hipStream_t st, const int* cexp) {
  if (KP > kResCols) {
    if (KP % kTile) return hipErrorInvalidValue;
    const int64_t tiles = res_wide_tiles(a_type, m);
    if (a_type == 0)
      return launch_residual_wide<double, double>((const double*)A, lda, m, n, U, ldu, S, V, ldv, k, KP, part, tiles,
                                                  info, st, nullptr);
    if (a_type == 1)
      return launch_residual_wide<float, float>((const float*)A, lda, m, n, U, ldu, S, V, ldv, k, KP, part, tiles,
                                                info, st, nullptr);
    if (a_type == 4)
      return launch_residual_wide<f16_word, float>((const f16_word*)A, lda, m, n, U, ldu, S, V, ldv, k, KP, part,
                                                   tiles, info, st, cexp);
    return launch_residual_wide<bf16_t, float>((const bf16_t*)A, lda, m, n, U, ldu, S, V, ldv, k, KP, part, tiles,
                                               info, st, nullptr);
  }
  const dim3 grid((unsigned)ceil_div(n, kResCols), (unsigned)residual_row_groups(m, n));
  if (a_type == 0) {
    const size_t shm = (size_t)KP * kResLd * sizeof(double);
    hipLaunchKernelGGL((k_residual<double, double>), grid, dim3(256), shm, st, (const double*)A, lda, m, n, U, ldu,
                       S, V, ldv, k, KP, part, nullptr);
  } else if (a_type == 1) {
    const size_t shm = (size_t)KP * kResLd * sizeof(float);
    hipLaunchKernelGGL((k_residual<float, float>), grid, dim3(256), shm, st, (const float*)A, lda, m, n, U, ldu, S,
                       V, ldv, k, KP, part, nullptr);
  } else if (a_type == 4) {
    const size_t shm = (size_t)KP * kResLd * sizeof(float);
    hipLaunchKernelGGL((k_residual<f16_word, float>), grid, dim3(256), shm, st, (const f16_word*)A, lda, m, n, U,
                       ldu, S, V, ldv, k, KP, part, cexp);
  } else {
    const size_t shm = (size_t)KP * kResLd * sizeof(float);
    hipLaunchKernelGGL((k_residual<bf16_t, float>), grid, dim3(256), shm, st, (const bf16_t*)A, lda, m, n, U, ldu,
                       S, V, ldv, k, KP, part, nullptr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, st, part, (int64_t)grid.x * grid.y, (ResInfo*)info);
  return hipGetLastError();
}

}  // namespace sor
