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
// noise, weighted by 4^-e_j (exact). Against the matrix before rounding, the
// approximation error is then estimated as sqrt(e_stored^2 - that sum / ||A||^2):
// the rounding error is spread over all n singular directions, so only a
// fraction (k / n)^2 of it is captured by the rank-k approximation.
#include <type_traits>

#include "half16.hpp"

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

// a_type: 0 FP64, 1 FP32, 2 BF16, 4 FP16 (cexp: its column exponents, or
// null). part: 2 residual_parts(m, n) doubles.
hipError_t launch_residual(int a_type, const void* A, int64_t lda, int64_t m, int64_t n, const double* U,
                           int64_t ldu, const double* S, const double* V, int64_t ldv, int k, int KP, double* part,
                           void* info, hipStream_t st, const int* cexp) {
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
