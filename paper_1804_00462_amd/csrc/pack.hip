// FP16 storage of A with power-of-two column scaling: A_stored = fp16(A D),
// D = diag(2^e_j). e_j = 14 - floor(log2 max_i |A_ij|) puts the largest
// entry of every column in [2^14, 2^15), so each column uses the top of the
// FP16 range whatever its own scale (a zero column keeps e_j = 0). The
// scaling is exact; the only error is the one rounding to FP16 (relative
// 2^-11 for entries within 2^-29 of their column's peak, absolute below).
#include <algorithm>

#include "half16.hpp"
#include "sorsvd.h"

namespace sor {

namespace {

// One workgroup per 64 columns: four waves walk interleaved rows, each lane
// one column (every row read is 64 consecutive elements), then the four
// maxima of the floor(log2 |a|) are combined in LDS.
template <typename T>
__global__ void __launch_bounds__(256) k_colexp(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                int* __restrict__ cexp) {
  __shared__ int emax_s[4][64];
  const int lane = threadIdx.x % 64, rg = threadIdx.x / 64;
  const int64_t c = (int64_t)blockIdx.x * 64 + lane;
  int emax = INT_MIN;
  if (c < n)
    for (int64_t i = rg; i < m; i += 4) {
      const double v = fabs((double)A[i * lda + c]);
      if (v != 0.0 && v - v == 0.0) emax = max(emax, ilogb(v));
    }
  emax_s[rg][lane] = emax;
  __syncthreads();
  if (rg == 0 && c < n) {
    const int e = max(max(emax_s[0][lane], emax_s[1][lane]), max(emax_s[2][lane], emax_s[3][lane]));
    cexp[c] = e == INT_MIN ? 0 : min(kMaxColExp, max(-kMaxColExp, 14 - e));
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_pack_f16(const T* __restrict__ A, int64_t lda, int64_t m, int64_t n,
                                                  const int* __restrict__ cexp, uint16_t* __restrict__ out,
                                                  int64_t ldo) {
  const int64_t total = m * n;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int64_t i = idx / n, j = idx % n;
    out[i * ldo + j] = f64_to_f16(ldexp((double)A[i * lda + j], cexp[j]));
  }
}

template <typename T>
hipError_t pack(const T* A, int64_t lda, int64_t m, int64_t n, uint16_t* out, int64_t ldo, int* cexp,
                hipStream_t st) {
  hipLaunchKernelGGL(k_colexp<T>, dim3((unsigned)ceil_div(n, 64)), dim3(256), 0, st, A, lda, m, n, cexp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t blocks = std::min<int64_t>(ceil_div(m * n, 256), 8192);
  hipLaunchKernelGGL(k_pack_f16<T>, dim3((unsigned)blocks), dim3(256), 0, st, A, lda, m, n, cexp, out, ldo);
  return hipGetLastError();
}

}  // namespace

}  // namespace sor

using namespace sor;

extern "C" int sorsvd_pack_f16(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, uint16_t* out,
                               int64_t ldo, int32_t* col_exp, void* stream) {
  if (m < 0 || n < 0 || lda < n || ldo < n) return SORSVD_EINVAL;
  if (a_type != SORSVD_F32 && a_type != SORSVD_F64) return SORSVD_EUNSUPPORTED;
  if (m == 0 || n == 0) return SORSVD_OK;
  if (!A || !out || !col_exp) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const hipError_t e = a_type == SORSVD_F64
                           ? pack((const double*)A, lda, m, n, out, ldo, (int*)col_exp, st)
                           : pack((const float*)A, lda, m, n, out, ldo, (int*)col_exp, st);
  return e == hipSuccess ? SORSVD_OK : SORSVD_EHIP;
}
