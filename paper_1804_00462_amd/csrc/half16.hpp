// 16-bit storage formats of A: BF16 (8 significant bits, FP32 range) and
// IEEE binary16 (11 significant bits, normal range 2^-14 .. 65504). Both are
// held as raw 16-bit words; kFmtBF16 / kFmtF16 select the format at compile
// time.
#pragma once
#include <climits>

#include "common.hpp"

namespace sor {

constexpr int kFmtBF16 = 0;
constexpr int kFmtF16 = 1;

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ inline float f16_to_f32(uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); }

// FP64 -> FP16 with a single rounding: round to FP32 with round-to-odd, then
// to FP16 to nearest-even (v_cvt_f16_f32). FP32 keeps at least 13 more bits
// than FP16 (also where the FP16 result is subnormal), so the two steps give
// the correctly rounded result. Values beyond the FP16 range become +-inf.
__device__ inline uint16_t f64_to_f16(double d) {
  float f = (float)d;
  const double back = (double)f;
  if (back != d && back - back == 0.0) {
    uint32_t u = __float_as_uint(f);
    if (fabs(back) > fabs(d)) u -= 1u;
    u |= 1u;
    f = __uint_as_float(u);
  }
  return __builtin_bit_cast(uint16_t, (_Float16)f);
}

template <int FMT> __device__ inline float h16_to_f32(uint16_t h) {
  if constexpr (FMT == kFmtBF16) return bf16_to_f32(h);
  else return f16_to_f32(h);
}

template <int FMT> __device__ inline uint16_t f64_to_h16(double d) {
  if constexpr (FMT == kFmtBF16) return f64_to_bf16(d);
  else return f64_to_f16(d);
}

// Powers of two applied to the 16-bit skinny operands and undone exactly on
// the FP64 outputs (one record per run, in device memory). With column
// exponents e (A = A_stored diag(2^-e_j)), or e = 0:
//   A X pass:    row j of X is stored as X_j 2^(nn_base - e_j); the output is
//                multiplied by 2^-nn_base
//   A^T Y pass:  Y is stored as Y 2^tn_base; output row j is multiplied by
//                2^(-tn_base - e_j)
// nn_base = min_j e_j + shift and tn_base = shift, where shift lifts entries
// of orthonormal (|q| <= 1) or Gaussian skinny operands clear of the FP16
// subnormal range (12 for FP16, 0 for BF16, whose range is FP32's).
struct H16Scale {
  int32_t nn_base, tn_base;
};

// Largest |e_j| accepted (sums of squares weighted by 4^-e_j stay in FP64 range).
constexpr int kMaxColExp = 256;

}  // namespace sor
