// Shared device definitions of the SOR-SVD library (gfx950 / CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t bf16_t;  // storage type of BF16 data (raw bits)

namespace sor {

// One Gaussian draw of a batch (Omega of one problem): rows x cols draws of
// key (seed, 0) written row-major into `out` (leading dimension ldx) in the
// compute type of that batch.
struct OmegaJob {
  uint64_t seed;
  int64_t rows, cols, ldx;
  void* out;
};

constexpr int kWave = 64;
constexpr int kTile = 16;  // MFMA output tile edge

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Round-to-nearest-even FP32 -> BF16 (finite inputs; NaN kept quiet).
__device__ inline bf16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(r >> 16);
}
__device__ inline float bf16_to_f32(bf16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// FP64 -> BF16 with a single rounding: round to FP32 with round-to-odd
// (exact results unchanged, inexact ones truncated toward zero with the last
// bit set), then round that to BF16 to nearest-even. FP32 carries more than
// two extra bits beyond BF16, so the result equals direct rounding of d.
__device__ inline bf16_t f64_to_bf16(double d) {
  float f = (float)d;
  double back = (double)f;
  if (back != d && back - back == 0.0) {
    uint32_t u = __float_as_uint(f);
    if (fabs(back) > fabs(d)) u -= 1u;
    u |= 1u;
    f = __uint_as_float(u);
  }
  return f32_to_bf16(f);
}

// 16-byte streaming load that bypasses cache retention (A is read once per pass).
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ inline uint4 load_stream16(const void* p) {
  const u32x4_t t = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
  return uint4{t.x, t.y, t.z, t.w};
}

// Sum over a full wavefront (64 lanes); every lane gets the total.
// v of lane `lane` (uniform), through two scalar reads.
__device__ inline double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// DPP lane exchange of a double within a row of 16 lanes (no LDS traffic).
// Controls: 0xB1 = quad_perm [1,0,3,2] (lane ^ 1), 0x4E = quad_perm [2,3,0,1]
// (lane ^ 2), 0x141 = row_half_mirror (lane i <-> 7 - i within 8),
// 0x140 = row_mirror (lane i <-> 15 - i within 16).
template <int CTRL>
__device__ inline double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  // every control used here has a valid source lane for every lane, so the
  // old value is never kept (and needs no initialising move)
  const int lo2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, false);
  const int hi2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi2, lo2);
}

// All-reduce sums over aligned groups of 4, 8 or 16 lanes by DPP. Each step
// adds two partial sums that are identical up to operand order, and IEEE
// addition is commutative, so every lane of a group ends with the same bits.
__device__ inline double sum4(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  return v;
}
__device__ inline double sum8(double v) {
  v = sum4(v);
  v += dpp_f64<0x141>(v);
  return v;
}
__device__ inline double sum16(double v) {
  v = sum8(v);
  v += dpp_f64<0x140>(v);
  return v;
}

// Sum over aligned groups of `width` lanes (width a power of two <= 64).
__device__ inline double group_sum(double v, int width) {
  for (int off = width >> 1; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

}  // namespace sor
