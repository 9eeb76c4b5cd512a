// Gaussian draw of Omega (Alg. 3 / Alg. 4 step 1) on the device.
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) turns the counter
// (e / 4, 0, word2, 0) under key (seed, stream) into four 64-bit words; the
// Box-Muller transform turns them into four N(0,1) numbers, of which draw e
// takes number e % 4. log, sin and cos are fixed sequences of IEEE double
// operations (+, -, *, /, sqrt; each rounded once, no fused multiply-add), so
// the draws are bitwise reproducible by any implementation of the same
// sequence, including the library's CPU reference:
//   log u:  u = f 2^e, f in (sqrt(1/2), sqrt(2)];  s = (f-1)/(f+1);  z = s s;
//           p = 1/23;  p = 1/(2j+1) + z p  (j = 10..0);  log u = e LN2 + (2 s) p
//   2 pi u with u = (2t+1) 2^-53:  quadrant qd = (2t+1+2^50) >> 51;
//           f = ((2t+1) - qd 2^51) 2^-51;  x = f PIO2;  z = x x;
//           S = 1 - (z S)/((2j)(2j+1)),  C = 1 - (z C)/((2j-1)(2j))  (j = 10..1);
//           (sin, cos)(x) = (x S, C), rotated by qd quarter turns.
#include "half16.hpp"

namespace sor {

namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;
constexpr double kLn2 = 0.6931471805599453;
constexpr double kPio2 = 1.5707963267948966;
constexpr double kSqrt2 = 1.4142135623730951;

struct Words { uint64_t w[4]; };

__device__ inline Words philox_block(uint64_t c0, uint64_t c2, uint64_t k0, uint64_t k1) {
  uint64_t x0 = c0, x1 = 0, x2 = c2, x3 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = __umul64hi(kM0, x0), lo0 = kM0 * x0;
    uint64_t hi1 = __umul64hi(kM1, x2), lo1 = kM1 * x2;
    uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    if (r != 9) { k0 += kW0; k1 += kW1; }
  }
  Words out;
  out.w[0] = x0; out.w[1] = x1; out.w[2] = x2; out.w[3] = x3;
  return out;
}

__device__ inline double uniform01(uint64_t w) {
  double t = (double)(w >> 12);                     // < 2^52: exact
  return t * 0x1p-52 + 0x1p-53;                     // exact dyadic in (0, 1)
}

__device__ inline double seq_log(double u) {
#pragma clang fp contract(off)
  uint64_t bits = __double_as_longlong(u);
  int e = (int)((bits >> 52) & 0x7ff) - 1023;       // u is normal here (u >= 2^-53)
  double f = __longlong_as_double((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);  // [1, 2)
  if (f > kSqrt2) { f = f * 0.5; e += 1; }
  double s = (f - 1.0) / (f + 1.0);
  double z = s * s;
  double p = 1.0 / 23.0;
  for (int j = 10; j >= 0; --j) {
    double inv = 1.0 / (double)(2 * j + 1);
    double zp = z * p;
    p = inv + zp;
  }
  double ed = (double)e;
  double a = ed * kLn2;
  double b = (2.0 * s) * p;
  return a + b;
}

__device__ inline void seq_sincos_2pi(uint64_t w, double* sn, double* cs) {
#pragma clang fp contract(off)
  int64_t t = (int64_t)(w >> 12);
  int64_t odd = 2 * t + 1;
  int64_t qd = (odd + (1ll << 50)) >> 51;
  double f = (double)(odd - qd * (1ll << 51)) * 0x1p-51;
  double x = f * kPio2;
  double z = x * x;
  double S = 1.0, C = 1.0;
  for (int j = 10; j >= 1; --j) {
    double ds = (double)((2 * j) * (2 * j + 1));
    double dc = (double)((2 * j - 1) * (2 * j));
    double zs = z * S;
    double zc = z * C;
    S = 1.0 - zs / ds;
    C = 1.0 - zc / dc;
  }
  double sx = x * S, cx = C;
  switch (qd & 3) {
    case 0: *sn = sx; *cs = cx; break;
    case 1: *sn = cx; *cs = -sx; break;
    case 2: *sn = -sx; *cs = -cx; break;
    default: *sn = -cx; *cs = sx; break;
  }
}

__device__ inline void normals4(uint64_t block, uint64_t word2, uint64_t seed, uint64_t stream, double z[4]) {
#pragma clang fp contract(off)
  Words w = philox_block(block, word2, seed, stream);
  double u0 = uniform01(w.w[0]);
  double u2 = uniform01(w.w[2]);
  double l0 = seq_log(u0), l2 = seq_log(u2);
  double m0 = -2.0 * l0, m2 = -2.0 * l2;
  double r01 = sqrt(m0), r23 = sqrt(m2);
  double s01, c01, s23, c23;
  seq_sincos_2pi(w.w[1], &s01, &c01);
  seq_sincos_2pi(w.w[3], &s23, &c23);
  z[0] = r01 * c01; z[1] = r01 * s01; z[2] = r23 * c23; z[3] = r23 * s23;
}

// One thread per Philox block. Writes Omega into one of three layouts:
//   mode 0: FP64 column-major rows x cols (ld = rows)
//   mode 1: compute-type row-major rows x ldx (ld = ldx), element (i, j) at i*ldx + j
//   mode 2: BF16 transposed: element (i, j) at j*ldx + i
template <int MODE, typename T>
__global__ void __launch_bounds__(256) k_omega(uint64_t seed, uint64_t stream, uint64_t word2,
                                               int64_t rows, int64_t cols, T* __restrict__ out,
                                               int64_t ldx) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t count = rows * cols;
  if (4 * b >= count) return;
  double z[4];
  normals4((uint64_t)b, word2, seed, stream, z);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    int64_t e = 4 * b + t;
    if (e >= count) break;
    int64_t i = e % rows, j = e / rows;
    if (MODE == 0) {
      out[e] = (T)z[t];
    } else if (MODE == 1) {
      out[i * ldx + j] = (T)z[t];
    } else {
      out[j * ldx + i] = (T)f64_to_bf16(z[t]);
    }
  }
}

// FP16 Omega for an NN pass, transposed (element (i, j) at j * ldx + i, as
// mode 2) and scaled: row i (column i of A) by 2^(nn_base - e_i), the
// scaling of every FP16 NN operand (H16Scale). Same draws as k_omega.
__global__ void __launch_bounds__(256) k_omega_f16_t(uint64_t seed, int64_t rows, int64_t cols,
                                                     uint16_t* __restrict__ out, int64_t ldx,
                                                     const H16Scale* __restrict__ sc,
                                                     const int* __restrict__ cexp) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t count = rows * cols;
  if (4 * b >= count) return;
  double z[4];
  normals4((uint64_t)b, 0, seed, 0, z);
  const int base = sc->nn_base;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t e = 4 * b + t;
    if (e >= count) break;
    const int64_t i = e % rows, j = e / rows;
    out[j * ldx + i] = f64_to_f16(ldexp(z[t], base - (cexp ? cexp[i] : 0)));
  }
}

// Batched Omega: blockIdx.y selects the job; one thread per Philox block,
// element (i, j) of job y is draw i + j * rows of key (seed_y, 0), exactly as
// in the single-problem kernel (mode 1).
template <typename T>
__global__ void __launch_bounds__(256) k_omega_batch(const OmegaJob* __restrict__ jobs) {
  const OmegaJob J = jobs[blockIdx.y];
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t count = J.rows * J.cols;
  if (4 * b >= count) return;
  double z[4];
  normals4((uint64_t)b, 0, J.seed, 0, z);
  T* out = reinterpret_cast<T*>(J.out);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t e = 4 * b + t;
    if (e >= count) break;
    out[(e % J.rows) * J.ldx + e / J.rows] = (T)z[t];
  }
}

}  // namespace

// Host launchers ------------------------------------------------------------

hipError_t launch_omega_f64_colmajor(uint64_t seed, uint64_t stream_id, uint64_t word2,
                                     int64_t rows, int64_t cols, double* out, hipStream_t st) {
  int64_t blocks = ceil_div(ceil_div(rows * cols, 4), 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_omega<0, double>), dim3((unsigned)blocks), dim3(256), 0, st,
                     seed, stream_id, word2, rows, cols, out, rows);
  return hipGetLastError();
}

hipError_t launch_omega_rowmajor_f64(uint64_t seed, int64_t rows, int64_t cols, double* out,
                                     int64_t ldx, hipStream_t st) {
  int64_t blocks = ceil_div(ceil_div(rows * cols, 4), 256);
  hipLaunchKernelGGL((k_omega<1, double>), dim3((unsigned)blocks), dim3(256), 0, st,
                     seed, (uint64_t)0, (uint64_t)0, rows, cols, out, ldx);
  return hipGetLastError();
}

hipError_t launch_omega_rowmajor_f32(uint64_t seed, int64_t rows, int64_t cols, float* out,
                                     int64_t ldx, hipStream_t st) {
  int64_t blocks = ceil_div(ceil_div(rows * cols, 4), 256);
  hipLaunchKernelGGL((k_omega<1, float>), dim3((unsigned)blocks), dim3(256), 0, st,
                     seed, (uint64_t)0, (uint64_t)0, rows, cols, out, ldx);
  return hipGetLastError();
}

hipError_t launch_omega_bf16_t(uint64_t seed, int64_t rows, int64_t cols, bf16_t* out,
                               int64_t ldx, hipStream_t st) {
  int64_t blocks = ceil_div(ceil_div(rows * cols, 4), 256);
  hipLaunchKernelGGL((k_omega<2, bf16_t>), dim3((unsigned)blocks), dim3(256), 0, st,
                     seed, (uint64_t)0, (uint64_t)0, rows, cols, out, ldx);
  return hipGetLastError();
}

hipError_t launch_omega_f16_t(uint64_t seed, int64_t rows, int64_t cols, uint16_t* out, int64_t ldx,
                              const H16Scale* sc, const int* cexp, hipStream_t st) {
  const int64_t blocks = ceil_div(ceil_div(rows * cols, 4), 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_omega_f16_t, dim3((unsigned)blocks), dim3(256), 0, st, seed, rows, cols, out, ldx, sc, cexp);
  return hipGetLastError();
}

// jobs: device array of njobs descriptors; max_count = the largest rows * cols.
hipError_t launch_omega_batch(const OmegaJob* jobs, int njobs, int64_t max_count, int f32,
                              hipStream_t st) {
  const int64_t blocks = ceil_div(ceil_div(max_count, 4), 256);
  if (blocks == 0 || njobs == 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_omega_batch<float>, dim3((unsigned)blocks, (unsigned)njobs), dim3(256), 0, st, jobs);
  else
    hipLaunchKernelGGL(k_omega_batch<double>, dim3((unsigned)blocks, (unsigned)njobs), dim3(256), 0, st, jobs);
  return hipGetLastError();
}

}  // namespace sor
