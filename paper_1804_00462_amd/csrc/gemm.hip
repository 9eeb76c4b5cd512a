// Launchers of the streaming skinny products over A (the passes of SOR-SVD)
// and their helper kernels: the fixed-order reduction of split partial sums,
// packing and casting of skinny operands.
//
//   NN:  T = A X      (T1 = A Omega, eq. T1; T1 = A T2 and the A Q2 half of eq. M in Alg. 4)
//   TN:  T = A^T Y    (T2 = A^T T1, eq. AT1; Alg. 4's T2 update)
//
// The contraction may be split into `nsplit` chunks whose partial sums are
// added afterwards in a fixed order (deterministic, no atomics). Workgroups
// are renumbered so that each of the 8 XCDs receives a contiguous run of
// (split, tile) pairs: workgroups on one XCD mostly share one split, i.e. one
// slab of the skinny operand, which then stays in that XCD's L2.
#include <algorithm>

#include <map>
#include <mutex>
#include <tuple>

#include "skinny_body.hpp"

namespace sor {

// The skinny operand and the output may be wider than one workgroup's
// columns: they are then cut into ncb column blocks of CT tiles (the output
// and the partial sums have ncb CT 16 columns). The ncb workgroups of one
// (split, row tile) read the same rows of A and get neighbouring logical
// indices, so they run on one XCD at about the same time and A comes from
// HBM about once. The sums of squares of A (normp) are taken by column
// block 0, one slot per (split, row tile).
template <typename T, bool TRANS, int RT, int CT>
__global__ void __launch_bounds__(256, 2)
k_skinny(const T* A, int64_t lda, int64_t OUT, int64_t K,
         const T* __restrict__ X, int64_t ldx, int64_t kchunk, int tiles, int nsplit, int ncb,
         int vec_ok, typename Traits<T>::acc_t* P, double* __restrict__ normp,
         const int* __restrict__ skipflag, double* Tout, int tri) {
  if (skipflag && *skipflag) return;  // product not needed (see the Cholesky QR step)
  constexpr int CB = CT * kTile;
  __shared__ T Xs[xs_elems<T, CT>()];
  __shared__ double red[4];
  const int nb = tiles * nsplit * ncb;
  const int v = ncb > 1 ? xcd_remap_any((int)blockIdx.x, nb) : xcd_remap((int)blockIdx.x, nb);
  const int cb = v % ncb, u = v / ncb;
  const int s = u / tiles, tile = u % tiles;
  const int64_t ldp = (int64_t)ncb * CB, c0 = (int64_t)cb * CB;
  const int64_t k0 = (int64_t)s * kchunk;
  const int64_t k1 = min(K, k0 + kchunk);
  const int64_t base = (int64_t)tile * (64 * RT);
  if constexpr (sizeof(T) == 8 && TRANS) {
    if (tri == 2 && c0 + CB <= base) {
      // the whole tile lies below the diagonal of A^T A, of which only the
      // upper triangle is wanted: zeros, with no pass over the rows
      double* out = Tout ? Tout : P + (int64_t)s * OUT * ldp;
      for (int e = threadIdx.x; e < 64 * RT * CB; e += 256) {
        const int64_t r = base + e / CB;
        if (r < OUT) out[r * ldp + c0 + e % CB] = 0.0;
      }
      return;
    }
  }
  // FP32 A^T Y: A fragments one step ahead (157 instead of 176 VGPRs at CT = 7:
  // three waves per SIMD); FP32 A X: two
  skinny_tile<T, TRANS, RT, CT, (sizeof(T) == 4 && !TRANS) ? 2 : 1>(A, lda, OUT, k0, k1, X + c0, ldx, base, vec_ok,
                                Tout ? nullptr : P + (int64_t)s * OUT * ldp + c0, Tout ? Tout + c0 : nullptr, ldp,
                                (normp && cb == 0) ? normp + u : nullptr, Xs, red, tri, ldp, c0);
}

// Column block cb of T <- T Z in place, for an upper triangular Z (LP x LP,
// LP = ncb CT 16): block cb needs columns [0, c0 + CB) of T (Z is zero below
// its diagonal) and overwrites columns [c0, c0 + CB). The blocks are formed
// from the last to the first (one launch each), so no block reads columns an
// earlier launch has overwritten. (P and nrm are null; taken as arguments,
// since constant null pointers there crash this compiler.)
template <int CT>
__global__ void __launch_bounds__(256, 2)
k_apply_tri_block(double* T, int64_t rows, int64_t LP, const double* __restrict__ Z, int cb, int vec_ok,
                  const int* __restrict__ skipflag, double* P, double* nrm) {
  if (skipflag && *skipflag) return;
  constexpr int CB = CT * kTile;
  __shared__ double Xs[xs_elems<double, CT>()];
  __shared__ double red[4];
  const int64_t base = (int64_t)blockIdx.x * 64;
  const int64_t c0 = (int64_t)cb * CB;
  skinny_tile<double, false, 1, CT>(T, LP, rows, 0, min(LP, c0 + CB), Z + c0, LP, base, vec_ok, P, T + c0,
                                    LP, nrm, Xs, red, 1, LP, c0);
}

// out[r][c] = sum_{s = 0..nsplit-1} P[s][r][c] in FP64, for c < ncols, in a
// fixed order: the kRedWaves waves of a block take s = w, w + kRedWaves, ...
// for the same 64 consecutive outputs (coalesced), eight splits in flight per
// wave, each with its own running sum (s = w + kRedWaves (u + 8 j) goes to
// sum u); the sums are combined pairwise, then the wave sums are added in
// order. skipflag as in the pass kernel (the sum is not needed).
constexpr int kRedWaves = 16;

template <typename Acc>
__global__ void __launch_bounds__(64 * kRedWaves)
k_reduce(const Acc* __restrict__ P, int64_t OUT, int LP, int nsplit, double* __restrict__ out,
         int64_t ldo, int ncols, const int* __restrict__ skipflag) {
  if (skipflag && *skipflag) return;
  __shared__ double part[kRedWaves][64];
  const int64_t total = OUT * LP;
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (idx < total) {
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int s = wv;
    for (; s + 7 * kRedWaves < nsplit; s += 8 * kRedWaves) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (double)P[(int64_t)(s + kRedWaves * u) * total + idx];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += v[u];
    }
    for (int u = 0; s < nsplit; s += kRedWaves, ++u) a[u] += (double)P[(int64_t)s * total + idx];
    acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  }
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && idx < total) {
    double t = part[0][lane];
#pragma unroll
    for (int i = 1; i < kRedWaves; ++i) t += part[i][lane];
    const int64_t r = idx / LP;
    const int c = (int)(idx % LP);
    if (c < ncols) out[r * ldo + c] = t;
  }
}

// FP32 partials: out[r][c] = sum_{s = 0..nsplit-1} P[s][r][c] in FP64, added
// in split order. Each thread takes four consecutive outputs (16-byte loads;
// LP is a multiple of 16, so the four share a row) and issues the loads of
// eight splits before adding them.
__global__ void __launch_bounds__(256)
k_reduce4(const float* __restrict__ P, int64_t OUT, int LP, int nsplit, double* __restrict__ out, int64_t ldo,
          int ncols) {
  const int64_t total = OUT * LP;
  const int64_t idx = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (idx >= total) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int s = 0;
  for (; s + 8 <= nsplit; s += 8) {
    float4 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = *reinterpret_cast<const float4*>(P + (int64_t)(s + u) * total + idx);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a0 += (double)v[u].x; a1 += (double)v[u].y; a2 += (double)v[u].z; a3 += (double)v[u].w;
    }
  }
  for (; s < nsplit; ++s) {
    const float4 v = *reinterpret_cast<const float4*>(P + (int64_t)s * total + idx);
    a0 += (double)v.x; a1 += (double)v.y; a2 += (double)v.z; a3 += (double)v.w;
  }
  const int64_t r = idx / LP;
  const int c = (int)(idx % LP);
  double* o = out + r * ldo + c;
  if (c < ncols) o[0] = a0;
  if (c + 1 < ncols) o[1] = a1;
  if (c + 2 < ncols) o[2] = a2;
  if (c + 3 < ncols) o[3] = a3;
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

// C (rows x cols, ldc) = A - B (both rows x cols, lda / ldb); FP64.
__global__ void __launch_bounds__(256)
k_sub_f64(const double* __restrict__ A, int64_t lda, const double* __restrict__ B, int64_t ldb, int64_t rows,
          int cols, double* __restrict__ C, int64_t ldc) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx / cols;
  const int c = (int)(idx % cols);
  C[r * ldc + c] = A[r * lda + c] - B[r * ldb + c];
}

// dst (cols x rows, ldd) = src^T, src rows x cols (lds); FP64.
__global__ void __launch_bounds__(256)
k_transpose_f64(const double* __restrict__ src, int64_t lds, int64_t rows, int cols, double* __restrict__ dst,
                int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * cols) return;
  const int64_t r = idx % rows;
  const int c = (int)(idx / rows);
  dst[(int64_t)c * ldd + r] = src[r * lds + c];
}

// ------------------------------------------------------------------ launchers

hipError_t launch_sub_f64(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t rows, int cols,
                          double* C, int64_t ldc, hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sub_f64, dim3((unsigned)ceil_div(rows * cols, 256)), dim3(256), 0, st, A, lda, B, ldb, rows,
                     cols, C, ldc);
  return hipGetLastError();
}

hipError_t launch_transpose_f64(const double* src, int64_t lds, int64_t rows, int cols, double* dst, int64_t ldd,
                                hipStream_t st) {
  if (rows * cols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_f64, dim3((unsigned)ceil_div(rows * cols, 256)), dim3(256), 0, st, src, lds, rows,
                     cols, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_zero_lower(double* R, int l, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_lower, dim3((unsigned)ceil_div((int64_t)l * l, 256)), dim3(256), 0, st, R, l);
  return hipGetLastError();
}

template <typename T, bool TRANS, int RT>
static hipError_t launch_ct(int CT, const T* A, int64_t lda, int64_t OUT, int64_t K, const T* X,
                            int64_t ldx, int64_t kchunk, int tiles, int nsplit, int ncb, int vec_ok,
                            typename Traits<T>::acc_t* P, double* normp, const int* skipflag,
                            double* Tout, hipStream_t st, int tri) {
  dim3 grid((unsigned)(tiles * nsplit * ncb)), block(256);
#define SORSVD_CASE(C)                                                                           \
  case C:                                                                                        \
    hipLaunchKernelGGL((k_skinny<T, TRANS, RT, C>), grid, block, 0, st, A, lda, OUT, K, X, ldx, \
                       kchunk, tiles, nsplit, ncb, vec_ok, P, normp, skipflag, Tout, tri);       \
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

// FP64 tiles are 64 rows: 128-row FP64 tiles of the widest operands do not fit the registers
int skinny_rt(int a_type, int64_t OUT) { return a_type == 1 ? 2 : 1; }

template <typename T, int RT>
static hipError_t launch_rt(bool trans, const T* A, int64_t lda, int64_t OUT, int64_t K, const T* X,
                            int64_t ldx, int LP, int64_t kchunk, int nsplit, int ncb,
                            typename Traits<T>::acc_t* P, double* normp, const int* skipflag,
                            double* Tout, hipStream_t st, int tri) {
  const int tiles = (int)ceil_div(OUT, 64 * RT);
  if (tiles == 0 || nsplit == 0) return hipSuccess;
  if (ncb < 1 || LP % (ncb * kTile)) return hipErrorInvalidValue;
  const int vec_ok = ((lda * (int64_t)sizeof(T)) % 16 == 0) && (((uintptr_t)A) % 16 == 0);
  const int CT = LP / ncb / kTile;
  if (trans)
    return launch_ct<T, true, RT>(CT, A, lda, OUT, K, X, ldx, kchunk, tiles, nsplit, ncb, vec_ok, P, normp, skipflag, Tout, st, tri);
  return launch_ct<T, false, RT>(CT, A, lda, OUT, K, X, ldx, kchunk, tiles, nsplit, ncb, vec_ok, P, normp, skipflag, Tout, st, tri);
}

template <typename T>
hipError_t launch_skinny(bool trans, const T* A, int64_t lda, int64_t OUT, int64_t K, const T* X,
                         int64_t ldx, int LP, int64_t kchunk, int nsplit,
                         typename Traits<T>::acc_t* P, double* normp, const int* skipflag,
                         double* Tout, hipStream_t st, int tri = 0, int ncb = 1) {
  // must agree with skinny_rt: FP64 64-row tiles, FP32 128-row tiles
  if constexpr (has_rt1<T>())
    return launch_rt<T, 1>(trans, A, lda, OUT, K, X, ldx, LP, kchunk, nsplit, ncb, P, normp, skipflag, Tout, st, tri);
  else
    return launch_rt<T, 2>(trans, A, lda, OUT, K, X, ldx, LP, kchunk, nsplit, ncb, P, normp, skipflag, Tout, st, tri);
}

// With Tout != null and nsplit == 1 the kernel writes the FP64 result itself.
// tri = 1: X is upper triangular (see skinny_tile); not with ncb > 1 in place
// (launch_apply_tri_blocks). tri = 2 (trans, X = A): only the upper triangle
// of A^T A is formed. ncb: column blocks of X and of the output (LP is their
// total width).
hipError_t launch_skinny_f64(bool trans, const double* A, int64_t lda, int64_t OUT, int64_t K,
                             const double* X, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                             double* P, double* normp, const int* skipflag, hipStream_t st,
                             double* Tout, int tri, int ncb) {
  if (tri == 1 && ncb > 1 && Tout == A) return hipErrorInvalidValue;
  if (tri == 2 && (!trans || X != A)) return hipErrorInvalidValue;
  return launch_skinny<double>(trans, A, lda, OUT, K, X, ldx, LP, kchunk, nsplit, P, normp, skipflag,
                               nsplit == 1 ? Tout : nullptr, st, tri, ncb);
}

hipError_t launch_skinny_f32(bool trans, const float* A, int64_t lda, int64_t OUT, int64_t K,
                             const float* X, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                             float* P, double* normp, const int* skipflag, hipStream_t st,
                             double* Tout, int ncb) {
  return launch_skinny<float>(trans, A, lda, OUT, K, X, ldx, LP, kchunk, nsplit, P, normp, skipflag,
                              nsplit == 1 ? Tout : nullptr, st, 0, ncb);
}

// T (rows x LP, ld LP) <- T Z in place, Z upper triangular LP x LP, LP = ncb
// column blocks of equal width (at most 128).
hipError_t launch_apply_tri_blocks(double* T, int64_t rows, int LP, const double* Z, int ncb,
                                   const int* skipflag, hipStream_t st) {
  if (ncb < 1 || LP % (ncb * kTile)) return hipErrorInvalidValue;
  const int CT = LP / ncb / kTile;
  const int64_t tiles = ceil_div(rows, 64);
  if (tiles == 0) return hipSuccess;
  const int vec_ok = ((LP * 8) % 16 == 0) && (((uintptr_t)T) % 16 == 0);
  dim3 grid((unsigned)tiles), block(256);
  for (int cb = ncb - 1; cb >= 0; --cb) {
#define SORSVD_CASE(C)                                                                                         \
  case C:                                                                                                      \
    hipLaunchKernelGGL((k_apply_tri_block<C>), grid, block, 0, st, T, rows, (int64_t)LP, Z, cb, vec_ok, skipflag, \
                       nullptr, nullptr);                                                                            \
    break;
    switch (CT) {
      SORSVD_CASE(1) SORSVD_CASE(2) SORSVD_CASE(3) SORSVD_CASE(4)
      SORSVD_CASE(5) SORSVD_CASE(6) SORSVD_CASE(7) SORSVD_CASE(8)
      default: return hipErrorInvalidValue;
    }
#undef SORSVD_CASE
  }
  return hipGetLastError();
}

int skinny_rows_per_block(int a_type, int64_t OUT) { return 64 * skinny_rt(a_type, OUT); }

// Workgroups of the pass kernel (FP64 a_type 0 / FP32 a_type 1, LP = 16 CT)
// that the current device holds at once: resident workgroups per CU (from
// the kernel's registers and LDS) times the CUs. 0 when no device answers.
template <typename T, bool TRANS>
static int skinny_blocks_per_cu(int CT) {
  constexpr int RT = has_rt1<T>() ? 1 : 2;
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
#define SORSVD_CASE(C)                                                                                     \
  case C:                                                                                                  \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_skinny<T, TRANS, RT, C>), \
                                                     256, 0);                                              \
    break;
  switch (CT) {
    SORSVD_CASE(1) SORSVD_CASE(2) SORSVD_CASE(3) SORSVD_CASE(4)
    SORSVD_CASE(5) SORSVD_CASE(6) SORSVD_CASE(7) SORSVD_CASE(8)
    default: break;
  }
#undef SORSVD_CASE
  return e == hipSuccess ? nb : 0;
}

// LP: the width of one column block.
int skinny_slots(int a_type, bool trans, int LP) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, bool, int>, int> cache;
  if ((a_type != 0 && a_type != 1) || LP % kTile || LP < kTile || LP > 8 * kTile) return 0;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  std::lock_guard<std::mutex> g(mu);
  const auto key = std::make_tuple(dev, a_type, trans, LP);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
  const int CT = LP / kTile;
  int nb;
  if (a_type == 0) nb = trans ? skinny_blocks_per_cu<double, true>(CT) : skinny_blocks_per_cu<double, false>(CT);
  else nb = trans ? skinny_blocks_per_cu<float, true>(CT) : skinny_blocks_per_cu<float, false>(CT);
  (void)hipGetLastError();
  const int slots = cus > 0 && nb > 0 ? cus * nb : 0;
  cache[key] = slots;
  return slots;
}
int skinny_step(int a_type) { return a_type == 0 ? 32 : (a_type == 1 ? 32 : 128); }

hipError_t launch_reduce_f64(const double* P, int64_t OUT, int LP, int nsplit, double* out,
                             int64_t ldo, int ncols, hipStream_t st, const int* skipflag) {
  const int64_t total = OUT * LP;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL((k_reduce<double>), dim3((unsigned)ceil_div(total, 64)), dim3(64 * kRedWaves), 0, st,
                     P, OUT, LP, nsplit, out, ldo, ncols, skipflag);
  return hipGetLastError();
}

hipError_t launch_reduce_f32(const float* P, int64_t OUT, int LP, int nsplit, double* out,
                             int64_t ldo, int ncols, hipStream_t st) {
  const int64_t total = OUT * LP;
  if (total == 0) return hipSuccess;
  if (LP % 4) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce4, dim3((unsigned)ceil_div(total / 4, 256)), dim3(256), 0, st, P, OUT, LP, nsplit,
                     out, ldo, ncols);
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

// A = diag(sigma) (n x n, given by its diagonal): T = diag(sigma) X, which is
// also A^T X. X and T are n x LP row-major.
__global__ void __launch_bounds__(256) k_diag_pass(const double* __restrict__ sigma, int64_t n, int LP,
                                                   const double* __restrict__ X, double* __restrict__ T) {
  const int64_t tot = n * LP;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (int64_t)gridDim.x * 256)
    T[i] = sigma[i / LP] * X[i];
}

// normp[b] = sum of sigma_r^2 over rows [b rpb, (b + 1) rpb) (the ||A||_F^2 slots of the first pass).
__global__ void __launch_bounds__(256) k_diag_norm(const double* __restrict__ sigma, int64_t n, int64_t rpb,
                                                   double* __restrict__ normp) {
  __shared__ double part[256];
  const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = min(n, r0 + rpb);
  double a = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) a += sigma[r] * sigma[r];
  part[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) normp[blockIdx.x] = part[0];
}

hipError_t launch_diag_pass(const double* sigma, int64_t n, int LP, const double* X, double* T, double* normp,
                            int nparts, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>(8192, ceil_div(n * LP, 256));
  hipLaunchKernelGGL(k_diag_pass, dim3((unsigned)blocks), dim3(256), 0, st, sigma, n, LP, X, T);
  if (normp)
    hipLaunchKernelGGL(k_diag_norm, dim3((unsigned)nparts), dim3(256), 0, st, sigma, n, ceil_div(n, nparts), normp);
  return hipGetLastError();
}

}  // namespace sor
