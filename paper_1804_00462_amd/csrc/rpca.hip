// Robust PCA by the ALM-SOR-SVD iteration (Sec. V, Table III): the
// elementwise kernels around the SOR-SVD of every iteration (FP64).
//
// One iteration, with (U, z, V) the SOR-SVD of W = X - S + Y / mu:
//   L = U shrink_{1/mu}(z) V^T
//   S = shrink_{lambda/mu}(X - L + Y / mu)
//   R = X - L - S,  Y = Y + mu R
//   W' = X - S + Y / mu'   (the next SOR-SVD input, mu' the next penalty)
// k_rpca_step does all of it in one pass over the m x n arrays: a workgroup
// owns a 32 x 32 tile, stages U's 32 rows (times the thresholded z) and V's
// 32 rows transposed in LDS, kRpcaChunk terms at a time, forms its L tile
// with FP64 FMAs (the l terms added in order) and applies the updates; the
// squares of R are summed per workgroup in FP64 (fixed order) for the
// stopping test.
#include <algorithm>

#include "common.hpp"

namespace sor {

namespace {

constexpr int kRT = 32;          // tile rows and columns
constexpr int kRpcaChunk = 128;  // terms of L staged in LDS at a time

// Per-block partial sums of x^2 and maxima of |x| over an m x n array.
__global__ void __launch_bounds__(256) k_rpca_stats(const double* __restrict__ X, int64_t ldx, int64_t m,
                                                    int64_t n, double* __restrict__ psq,
                                                    double* __restrict__ pmax) {
  __shared__ double ssq[4], smx[4];
  const int64_t total = m * n;
  double sq = 0.0, mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const double v = X[(i / n) * ldx + i % n];
    sq += v * v;
    mx = fmax(mx, fabs(v));
  }
  sq = wave_sum(sq);
  for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
  const int w = threadIdx.x / kWave;
  if (threadIdx.x % kWave == 0) {
    ssq[w] = sq;
    smx[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    psq[blockIdx.x] = (ssq[0] + ssq[1]) + (ssq[2] + ssq[3]);
    pmax[blockIdx.x] = fmax(fmax(smx[0], smx[1]), fmax(smx[2], smx[3]));
  }
}

// Y = X / J, S = 0, W = X + Y / mu.
__global__ void __launch_bounds__(256) k_rpca_init(const double* __restrict__ X, int64_t ldx, int64_t m,
                                                   int64_t n, double inv_j, double inv_mu, double* __restrict__ S,
                                                   int64_t lds, double* __restrict__ Y, double* __restrict__ W) {
  const int64_t total = m * n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / n, c = i % n;
    const double x = X[r * ldx + c];
    const double y = x * inv_j;
    S[r * lds + c] = 0.0;
    Y[i] = y;
    W[i] = x + y * inv_mu;
  }
}

__device__ inline double shrink(double x, double e) {
  const double a = fabs(x) - e;
  return a > 0.0 ? copysign(a, x) : 0.0;
}

// One ALM iteration over a 32 x 32 tile (256 threads: thread (ty, tx) takes
// rows ty + 8 i, i < 4, of column tx). U: m x l, V: n x l (row-major, ld l).
__global__ void __launch_bounds__(256) k_rpca_step(const double* __restrict__ X, int64_t ldx, int64_t m, int64_t n,
                                                   const double* __restrict__ U, const double* __restrict__ V,
                                                   const double* __restrict__ z, int l, double inv_mu, double thr_s,
                                                   double mu, double inv_mu_next, double* __restrict__ L,
                                                   double* __restrict__ S, int64_t ld, double* __restrict__ Y,
                                                   double* __restrict__ W, double* __restrict__ rpart) {
  extern __shared__ double sm[];
  const int lc = min(l, kRpcaChunk);
  double* Us = sm;              // lc x 32: Us[t][r] = U[r0 + r][t0 + t] shrink(z_{t0 + t})
  double* Vs = sm + lc * kRT;   // lc x 32: Vs[t][c] = V[c0 + c][t0 + t]
  __shared__ double red[4];
  const int64_t r0 = (int64_t)blockIdx.y * kRT, c0 = (int64_t)blockIdx.x * kRT;
  const int tx = threadIdx.x % kRT, ty = threadIdx.x / kRT;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t0 = 0; t0 < l; t0 += lc) {
    const int nt = min(lc, l - t0);
    if (t0 > 0) __syncthreads();  // the previous chunk has been read
    for (int i = threadIdx.x; i < nt * kRT; i += 256) {
      const int t = i % nt, r = i / nt;  // consecutive threads read consecutive t of one row
      const double zt = fmax(z[t0 + t] - inv_mu, 0.0);
      Us[t * kRT + r] = r0 + r < m ? U[(r0 + r) * l + t0 + t] * zt : 0.0;
      Vs[t * kRT + r] = c0 + r < n ? V[(c0 + r) * l + t0 + t] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < nt; ++t) {
      const double v = Vs[t * kRT + tx];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] += Us[t * kRT + ty + 8 * i] * v;
    }
  }
  double rsq = 0.0;
  const int64_t c = c0 + tx;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + ty + 8 * i;
    if (r < m && c < n) {
      const double x = X[r * ldx + c];
      const int64_t e = r * n + c;
      const double y = Y[e];
      const double lv = acc[i];
      const double s = shrink(x - lv + y * inv_mu, thr_s);
      const double res = x - lv - s;
      const double y2 = y + mu * res;
      L[r * ld + c] = lv;
      S[r * ld + c] = s;
      Y[e] = y2;
      W[e] = x - s + y2 * inv_mu_next;
      rsq += res * res;
    }
  }
  rsq = wave_sum(rsq);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = rsq;
  __syncthreads();
  if (threadIdx.x == 0) rpart[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Per-block counts of nonzero entries of S.
__global__ void __launch_bounds__(256) k_rpca_nnz(const double* __restrict__ S, int64_t ld, int64_t m, int64_t n,
                                                  double* __restrict__ pcount) {
  __shared__ double red[4];
  const int64_t total = m * n;
  double cnt = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
    cnt += S[(i / n) * ld + i % n] != 0.0 ? 1.0 : 0.0;
  cnt = wave_sum(cnt);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) pcount[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace

int rpca_stat_blocks(int64_t m, int64_t n) { return (int)std::min<int64_t>(1024, ceil_div(m * n, 256)); }
int64_t rpca_step_blocks(int64_t m, int64_t n) { return ceil_div(m, kRT) * ceil_div(n, kRT); }

hipError_t launch_rpca_stats(const double* X, int64_t ldx, int64_t m, int64_t n, double* psq, double* pmax,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_rpca_stats, dim3((unsigned)rpca_stat_blocks(m, n)), dim3(256), 0, st, X, ldx, m, n, psq,
                     pmax);
  return hipGetLastError();
}

hipError_t launch_rpca_init(const double* X, int64_t ldx, int64_t m, int64_t n, double inv_j, double inv_mu,
                            double* S, int64_t lds, double* Y, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_rpca_init, dim3((unsigned)rpca_stat_blocks(m, n)), dim3(256), 0, st, X, ldx, m, n, inv_j,
                     inv_mu, S, lds, Y, W);
  return hipGetLastError();
}

hipError_t launch_rpca_step(const double* X, int64_t ldx, int64_t m, int64_t n, const double* U, const double* V,
                            const double* z, int l, double inv_mu, double thr_s, double mu, double inv_mu_next,
                            double* L, double* S, int64_t ld, double* Y, double* W, double* rpart,
                            hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(n, kRT), (unsigned)ceil_div(m, kRT));
  const size_t shm = (size_t)2 * std::min(l, kRpcaChunk) * kRT * sizeof(double);
  hipLaunchKernelGGL(k_rpca_step, grid, dim3(256), shm, st, X, ldx, m, n, U, V, z, l, inv_mu, thr_s, mu,
                     inv_mu_next, L, S, ld, Y, W, rpart);
  return hipGetLastError();
}

hipError_t launch_rpca_nnz(const double* S, int64_t ld, int64_t m, int64_t n, double* pcount, hipStream_t st) {
  hipLaunchKernelGGL(k_rpca_nnz, dim3((unsigned)rpca_stat_blocks(m, n)), dim3(256), 0, st, S, ld, m, n, pcount);
  return hipGetLastError();
}

}  // namespace sor
