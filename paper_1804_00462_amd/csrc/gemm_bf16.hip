// 16-bit passes over A: the BF16 instantiations of the pass kernels
// (h16_body.hpp), the kernels around them shared by both formats (the cast of
// the skinny operand, the reductions of the partials, the scale record) and
// the launchers that dispatch on the format.
#include <map>
#include <mutex>
#include <tuple>

#include "h16_body.hpp"

namespace sor {

// gemm_f16.hip: the FP16 instantiations
hipError_t launch_h16_f16(bool trans, const uint16_t* A, int64_t lda, int64_t OUT, int64_t K, const uint16_t* XT,
                          int64_t ldx, int LP, int64_t kchunk, int nsplit, int ncb, float* P, double* normp,
                          double* Tout, int fold, int rt, const H16Scale* sc, const int* cexp, hipStream_t st);
int h16_blocks_f16(bool trans, int rt, int CT);

// ---------------------------------------------------------------------------
// Skinny operand of a 16-bit pass: Q (rows x ncb LP, FP64, row-major) -> the
// transposed 16-bit layout QT (x ldt), optionally with the contraction
// permutation of the TN kernel, optionally with the low part h16(Q' - hi)
// (the refinement split). Column block cb (columns cb LP .. + LP - 1, LP <=
// 128) goes to QT rows cb LP .. (high part only) or to rows 2 cb LP .. (high
// part) and 2 cb LP + LP .. (low part): the operand block of the pass kernel's
// column block cb. With sc, row r is
// scaled first, Q' = Q 2^s_r: s_r = tn_base for a TN operand (`permute`),
// nn_base - e_r for an NN operand (rows of an NN operand are columns of A).
// Rows rows..ldt-1 are written as zeros. A workgroup stages kCastRows rows of
// its column block in LDS (coalesced reads of Q); each thread then forms 8
// consecutive positions of one output row (8 gathered tile rows) and writes
// them as one 16-byte store. 32-row tiles (33 KB of LDS) let four workgroups
// share a CU; the TN permutation stays within aligned groups of 32 rows.
constexpr int kCastRows = 32;
constexpr int kCastLoads = kCastRows * 128 / 2 / 256;  // 16-byte loads per thread at LP = 128

template <int FMT>
__global__ void __launch_bounds__(256)
k_cast_h16_t(const double* __restrict__ Q, int64_t rows, int LP, int ncb, int64_t ldt, int permute,
             int with_lo, uint16_t* __restrict__ QT, const H16Scale* __restrict__ sc,
             const int* __restrict__ cexp) {
  __shared__ double tile[kCastRows][129];
  const int64_t r0 = (int64_t)blockIdx.x * kCastRows;
  const int cb = blockIdx.y;
  const int64_t ldq = (int64_t)ncb * LP;
  Q += (int64_t)cb * LP;
  QT += (int64_t)cb * (with_lo ? 2 : 1) * LP * ldt;
  // the tile as pairs of entries (LP is even): every thread issues all its
  // 16-byte loads before the first LDS store
  double2 v[kCastLoads];
#pragma unroll
  for (int j = 0; j < kCastLoads; ++j) {
    const int e = 2 * (threadIdx.x + 256 * j);
    const int rr = e / LP, c = e % LP;
    const int64_t r = r0 + rr;
    v[j] = double2{0.0, 0.0};
    if (e < kCastRows * LP && r < rows) v[j] = *reinterpret_cast<const double2*>(Q + r * ldq + c);
  }
#pragma unroll
  for (int j = 0; j < kCastLoads; ++j) {
    const int e = 2 * (threadIdx.x + 256 * j);
    if (e < kCastRows * LP) {
      const int rr = e / LP, c = e % LP;
      const int64_t r = r0 + rr;
      double2 w = v[j];
      if (sc && r < rows) {
        const int sh = permute ? sc->tn_base : sc->nn_base - (cexp ? cexp[r] : 0);
        w.x = ldexp(w.x, sh);
        w.y = ldexp(w.y, sh);
      }
      tile[rr][c] = w.x;
      tile[rr][c + 1] = w.y;
    }
  }
  __syncthreads();
  const int parts = with_lo ? 2 : 1;
  // item: (output row cp = part LP + c, group u of 8 positions); consecutive
  // threads cover consecutive positions of one output row
  constexpr int NU = kCastRows / 8;
  for (int it = threadIdx.x; it < parts * LP * NU; it += 256) {
    const int u = it % NU, cp = it / NU;
    const int c = cp % LP, part = cp / LP;
    const int64_t pos0 = r0 + 8 * u;
    if (pos0 >= ldt) continue;  // ldt is a multiple of kCastRows
    uint32_t wv[4];
#pragma unroll
    for (int t2 = 0; t2 < 4; ++t2) {
      uint32_t pair = 0;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = 2 * t2 + h;
        // position 32 J + 8 g + t holds row 32 J + 4 t + g when permuted
        const int pr = 8 * u + t;
        const int rr = permute ? (pr / 32) * 32 + 4 * t + (pr % 32) / 8 : pr;
        const double q = tile[rr][c];
        const uint16_t hi = f64_to_h16<FMT>(q);
        const uint16_t val = part == 0 ? hi : f64_to_h16<FMT>(q - (double)h16_to_f32<FMT>(hi));
        pair |= (uint32_t)val << (16 * h);
      }
      wv[t2] = pair;
    }
    *reinterpret_cast<u32x4_t*>(QT + ((int64_t)part * LP + c) * ldt + pos0) = u32x4_t{wv[0], wv[1], wv[2], wv[3]};
  }
}

// Column of the partial sums that holds the high-part product of output
// column c with `fold` (column blocks of cbw outputs, each stored as cbw
// high-part columns followed by cbw low-part columns); the low-part product
// is cbw further on.
__device__ inline int fold_col(int c, int cbw) { return (c / cbw) * 2 * cbw + c % cbw; }

// out[r][c] = sum_s (P[s][r][hi(c)] + P[s][r][hi(c) + cbw]) for c < ncols:
// the refinement pass adds the products with the high and low parts of Q2.
__global__ void __launch_bounds__(256)
k_reduce_fold(const float* __restrict__ P, int64_t OUT, int LP2, int nsplit, double* __restrict__ out,
              int64_t ldo, int ncols, int cbw) {
  const int LPh = LP2 / 2;
  const int64_t total = OUT * LPh;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int64_t r = idx / LPh;
  const int c = (int)(idx % LPh);
  const int ch = fold_col(c, cbw);
  double acc = 0.0;
  for (int s = 0; s < nsplit; ++s) {
    const float* p = P + ((int64_t)s * OUT + r) * LP2;
    acc += (double)p[ch] + (double)p[ch + cbw];
  }
  if (c < ncols) out[r * ldo + c] = acc;
}

// Scaled reduction of the partials (4 output columns per thread):
// out[r][c] = 2^sh(r) sum_s P[s][r][c], or with `fold`
// 2^sh(r) sum_s (P[s][r][hi(c)] + P[s][r][hi(c) + cbw]) (fold_col), sh(r)
// undoing the operand scaling (out_shift). cbw is a multiple of 4, so the
// four columns of a thread lie in one block.
template <bool TRANS>
__global__ void __launch_bounds__(256)
k_reduce_h16(const float* __restrict__ P, int64_t OUT, int LP2, int nsplit, double* __restrict__ out,
             int64_t ldo, int ncols, int fold, int cbw, const H16Scale* __restrict__ sc,
             const int* __restrict__ cexp) {
  const int LPo = fold ? LP2 / 2 : LP2;
  const int64_t total = OUT * LPo;
  const int64_t idx = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (idx >= total) return;
  const int64_t r = idx / LPo;
  const int c = (int)(idx % LPo);
  const float* p = P + r * LP2 + (fold ? fold_col(c, cbw) : c);
  const int LPo_off = fold ? cbw : 0;  // the low-part product, cbw columns on
  const int64_t stride = OUT * LP2;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  int s = 0;
  for (; s + 4 <= nsplit; s += 4) {
    float4 v[4], w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      v[u] = *reinterpret_cast<const float4*>(p + (int64_t)(s + u) * stride);
      if (fold) w[u] = *reinterpret_cast<const float4*>(p + (int64_t)(s + u) * stride + LPo_off);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (fold) {
        a[0] += (double)v[u].x + (double)w[u].x; a[1] += (double)v[u].y + (double)w[u].y;
        a[2] += (double)v[u].z + (double)w[u].z; a[3] += (double)v[u].w + (double)w[u].w;
      } else {
        a[0] += (double)v[u].x; a[1] += (double)v[u].y; a[2] += (double)v[u].z; a[3] += (double)v[u].w;
      }
    }
  }
  for (; s < nsplit; ++s) {
    const float4 v = *reinterpret_cast<const float4*>(p + (int64_t)s * stride);
    if (fold) {
      const float4 w = *reinterpret_cast<const float4*>(p + (int64_t)s * stride + LPo_off);
      a[0] += (double)v.x + (double)w.x; a[1] += (double)v.y + (double)w.y;
      a[2] += (double)v.z + (double)w.z; a[3] += (double)v.w + (double)w.w;
    } else {
      a[0] += (double)v.x; a[1] += (double)v.y; a[2] += (double)v.z; a[3] += (double)v.w;
    }
  }
  const int sh = out_shift<TRANS>(sc, cexp, r);
  double* o = out + r * ldo + c;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (c + u < ncols) o[u] = ldexp(a[u], sh);
}

// Sets the scale record: nn_base = min_j e_j + shift (shift without
// exponents), tn_base = shift; flags bit 3 of the result record when some
// |e_j| > kMaxColExp (the run goes on with them). One workgroup.
__global__ void __launch_bounds__(256)
k_h16_scale(const int* __restrict__ cexp, int64_t n, int shift, H16Scale* __restrict__ sc, int* __restrict__ flags) {
  __shared__ int smin[256], sbad[256];
  int mn = INT_MAX, bad = 0;
  if (cexp)
    for (int64_t j = threadIdx.x; j < n; j += 256) {
      const int e = cexp[j];
      mn = min(mn, e);
      bad |= (e > kMaxColExp || e < -kMaxColExp) ? 1 : 0;
    }
  smin[threadIdx.x] = mn;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + off]);
      sbad[threadIdx.x] |= sbad[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int emin = (cexp && n > 0) ? smin[0] : 0;
    sc->nn_base = emin + shift;
    sc->tn_base = shift;
    if (sbad[0]) *flags |= 8;
  }
}

// ------------------------------------------------------------------ launchers

// fmt: kFmtBF16 (sc and cexp unused: BF16 operands are not scaled) or
// kFmtF16 (sc required, cexp optional).
// LP: total operand width, in ncb column blocks.
hipError_t launch_h16_pass(int fmt, bool trans, const uint16_t* A, int64_t lda, int64_t OUT, int64_t K,
                           const uint16_t* XT, int64_t ldx, int LP, int64_t kchunk, int nsplit, int ncb, float* P,
                           double* normp, double* Tout, int fold, int rt, const H16Scale* sc, const int* cexp,
                           hipStream_t st) {
  if (fmt == kFmtBF16)
    return launch_h16_fmt<kFmtBF16>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, ncb, P, normp, Tout, fold,
                                    rt, nullptr, nullptr, st);
  if (fmt == kFmtF16 && sc)
    return launch_h16_f16(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, ncb, P, normp, Tout, fold, rt, sc,
                          cexp, st);
  return hipErrorInvalidValue;
}

int h16_slots(int fmt, bool trans, int rt, int LP) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, bool, int, int>, int> cache;
  if (LP % kTile || LP < kTile || (rt != 1 && rt != 2 && rt != 4) || (fmt != kFmtBF16 && fmt != kFmtF16)) return 0;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  std::lock_guard<std::mutex> g(mu);
  const auto key = std::make_tuple(dev, fmt, trans, rt, LP);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  const int CT = LP / kTile;
  const int nb = fmt == kFmtBF16 ? h16_blocks<kFmtBF16>(trans, rt, CT) : h16_blocks_f16(trans, rt, CT);
  (void)hipGetLastError();
  const int slots = cus > 0 && nb > 0 ? cus * nb : 0;
  cache[key] = slots;
  return slots;
}

// contraction step of the 16-bit kernels for a given rt and skinny width LP
// (splits are multiples of it)
int bf16_step(bool trans, int rt, int LP) { return trans ? (rt >= 4 ? 64 : 128) : nn_kb(rt, LP); }

// Q: rows x (ncb LP) FP64; LP: the width of one column block.
hipError_t launch_cast_h16_t(int fmt, const double* Q, int64_t rows, int LP, int ncb, int64_t ldt, int permute,
                             int with_lo, uint16_t* QT, const H16Scale* sc, const int* cexp, hipStream_t st) {
  // the staging loads take Q 16-byte aligned, LP even and at most 128
  if (ldt % kCastRows || LP % 2 || LP > 128 || ncb < 1 || ((uintptr_t)Q % 16)) return hipErrorInvalidValue;
  const int64_t blocks = ceil_div(ldt, kCastRows);
  if (blocks == 0) return hipSuccess;
  const dim3 grid((unsigned)blocks, (unsigned)ncb);
  if (fmt == kFmtBF16)
    hipLaunchKernelGGL(k_cast_h16_t<kFmtBF16>, grid, dim3(256), 0, st, Q, rows, LP, ncb, ldt, permute, with_lo, QT,
                       sc, cexp);
  else
    hipLaunchKernelGGL(k_cast_h16_t<kFmtF16>, grid, dim3(256), 0, st, Q, rows, LP, ncb, ldt, permute, with_lo, QT,
                       sc, cexp);
  return hipGetLastError();
}

// cbw: output columns per column block (the whole width when ncb = 1).
hipError_t launch_reduce_fold(const float* P, int64_t OUT, int LP2, int nsplit, double* out,
                              int64_t ldo, int ncols, int cbw, hipStream_t st) {
  const int64_t total = OUT * (LP2 / 2);
  if (total == 0) return hipSuccess;
  if (cbw < 1 || (LP2 / 2) % cbw) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce_fold, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, P, OUT,
                     LP2, nsplit, out, ldo, ncols, cbw);
  return hipGetLastError();
}

hipError_t launch_reduce_h16(bool trans, const float* P, int64_t OUT, int LP2, int nsplit, double* out, int64_t ldo,
                             int ncols, int fold, int cbw, const H16Scale* sc, const int* cexp, hipStream_t st) {
  const int LPo = fold ? LP2 / 2 : LP2;
  const int64_t total = OUT * LPo;
  if (total == 0) return hipSuccess;
  if (LPo % 4 || (fold && (cbw % 4 || LPo % cbw))) return hipErrorInvalidValue;
  const dim3 grid((unsigned)ceil_div(total / 4, 256));
  if (trans)
    hipLaunchKernelGGL(k_reduce_h16<true>, grid, dim3(256), 0, st, P, OUT, LP2, nsplit, out, ldo, ncols, fold, cbw,
                       sc, cexp);
  else
    hipLaunchKernelGGL(k_reduce_h16<false>, grid, dim3(256), 0, st, P, OUT, LP2, nsplit, out, ldo, ncols, fold, cbw,
                       sc, cexp);
  return hipGetLastError();
}

hipError_t launch_h16_scale(const int* cexp, int64_t n, int shift, H16Scale* sc, int* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_h16_scale, dim3(1), dim3(256), 0, st, cexp, n, shift, sc, flags);
  return hipGetLastError();
}

}  // namespace sor
