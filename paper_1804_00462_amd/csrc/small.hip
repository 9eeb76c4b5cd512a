// Small kernels of the SOR-SVD path: the Cholesky-QR step and the core SVD
// (bodies in small_body.hpp), the sign convention and assembly of the lifted
// factors, and the error record.
#include "small_body.hpp"

namespace sor {

__global__ void __launch_bounds__(kSmallThreads)
k_chol_inv(const double* __restrict__ G, int LP, int l, int64_t rows, int mode,
           double* __restrict__ Rinv, int* __restrict__ skip3, DevInfo* __restrict__ info) {
  extern __shared__ double sm[];
  chol_inv_body(G, 1, 0, LP, l, rows, mode, Rinv, skip3, info, sm);
}

template <bool V_LDS, bool WANT_V, int NRB>
__global__ void __launch_bounds__(kJacThreads)
k_jacobi(const double* __restrict__ Min, int LP, int l, int k, int max_sweeps, double tol2,
         double* __restrict__ Ut, double* __restrict__ sv, double* __restrict__ Vt, int ldk,
         double* __restrict__ Vg, DevInfo* __restrict__ info, double2* __restrict__ rlog,
         int* __restrict__ vperm) {
  extern __shared__ double sm[];
  jacobi_body<V_LDS, WANT_V, NRB>(Min, 1, 0, LP, l, k, max_sweeps, tol2, Ut, sv, Vt, ldk, Vg, info, sm, rlog,
                                  vperm);
}

// V of the core SVD from the rotation log of jacobi_body (rlog, vperm): row r
// of V starts as e_r and receives, step by step, the rotations of that step's
// disjoint column pairs, (v_p, v_q) <- (c v_p - s v_q, s v_p + c v_q), p < q:
// the sequence the columns of M received. Then Vt[r][j] = V[r][vperm[j]].
// A wave owns one row and follows the pair order of jac_slot: lane s is slot
// s and holds, for a level, the entry of its stationary column (a) and of
// its current moving column (b); between steps the moving entries pass from
// slot g + 1 to slot g of each block (a lane gather), and at the end of a
// level (when after R steps every moving entry is back at its first slot)
// the row goes through LDS to the next level's slots. The waves of a
// workgroup share the coefficients, staged through LDS kVapChunk steps at a
// time: the next chunk is loaded into registers while the current one is
// applied.
constexpr int kVapWaves = 4;
constexpr int kVapChunk = 32;
constexpr int kVapLoads = kVapChunk * kWave / (kWave * kVapWaves);
constexpr int kVapGroup = 8;

__global__ void __launch_bounds__(64 * kVapWaves)
k_jacobi_vapply(const double2* __restrict__ rlog, const int* __restrict__ vperm, const DevInfo* __restrict__ info,
                int l, int k, int max_sweeps, double* __restrict__ Vt, int ldk) {
  __shared__ double2 cbuf[2][kVapChunk * kWave];
  __shared__ double rows[kVapWaves][128];
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int r = blockIdx.x * kVapWaves + w;
  const int ng = jac_groups(l), nst = jac_sweep_steps(l), nlev = jac_levels(l);
  // a converged run's last sweep rotated nothing (that is how it ended):
  // it is not replayed; after the sweep cap every sweep is
  const int ran = min(info->sweeps, max_sweeps);
  const int sweeps = (info->flags & kFlagNoConv) ? ran : max(ran - 1, 0);
  const int64_t T = (int64_t)sweeps * nst;
  double* R = rows[w];
  for (int j = lane; j < 128; j += kWave) R[j] = (j == r) ? 1.0 : 0.0;
  __syncthreads();
  if (T > 0) {  // uniform
    // level state (uniform: level d, its step j and length H) and this
    // lane's slot in it
    int d = 0, j = 0, H = jac_level_steps(l, 0);
    JacSlot sl = jac_slot(l, 0, H, lane);
    bool live = lane < ng;
    double a = 0.0, b = 0.0;
    auto enter = [&]() {
      sl = jac_slot(l, d, H, lane);
      a = (live && sl.g < sl.a) ? R[sl.p] : 0.0;
      b = (live && sl.g < sl.m) ? R[sl.s1 + sl.g] : 0.0;
    };
    enter();
    // chunk entry e = s * kWave + slot: coefficients of that slot at step
    // t0 + s. Addresses are clamped so that every load is unconditional
    // (entries past the log, and slots past the groups, are never used)
    const int64_t tlast = T - 1;
    auto load_entry = [&](int64_t t0, int jj) {
      const int e = threadIdx.x + jj * 64 * kVapWaves;
      return rlog[min(t0 + e / kWave, tlast) * ng + min(e % kWave, ng - 1)];
    };
    auto apply = [&](const double2 cs) {
      if (j < sl.R) {  // the block's ring is still turning
        int mi = sl.g + j;
        if (mi >= sl.R) mi -= sl.R;
        if (live && sl.g < sl.a && mi < sl.m) {
          const double c = cs.x, s = cs.y, x = a, y = b;
          a = c * x - s * y;
          b = s * x + c * y;
        }
      }
      // moving entries from slot g + 1 to slot g (ring of R slots)
      int src = sl.g + 1;
      if (src >= sl.R) src = 0;
      src = lane - sl.g + src;
      const double nb = __shfl(b, live ? src : lane, kWave);
      if (live && j < sl.R && sl.g < sl.R) b = nb;
      if (++j == H) {
        // after R steps every moving entry is back at slot g: the row to LDS,
        // then the next level's slots
        if (live && sl.g < sl.a) R[sl.p] = a;
        if (live && sl.g < sl.m) R[sl.s1 + sl.g] = b;
        __syncthreads();
        j = 0;
        if (++d == nlev) d = 0;
        H = jac_level_steps(l, d);
        enter();
        __syncthreads();
      }
    };
#pragma unroll
    for (int jj = 0; jj < kVapLoads; ++jj) cbuf[0][threadIdx.x + jj * 64 * kVapWaves] = load_entry(0, jj);
    __syncthreads();
    const int64_t nch = ceil_div(T, (int64_t)kVapChunk);
    for (int64_t ch = 0; ch < nch; ++ch) {
      const int buf = (int)(ch & 1);
      // the next chunk is loaded even after the last one (clamped, unused) so
      // that the loads need no branch
      double2 st[kVapLoads];
#pragma unroll
      for (int jj = 0; jj < kVapLoads; ++jj) st[jj] = load_entry((ch + 1) * kVapChunk, jj);
      const double2* cb = cbuf[buf] + lane;
      if ((ch + 1) * kVapChunk <= T) {
        // coefficients read from LDS a group of kVapGroup steps ahead of use
        double2 cw[kVapGroup];
#pragma unroll
        for (int s = 0; s < kVapGroup; ++s) cw[s] = cb[s * kWave];
#pragma unroll
        for (int g = 0; g < kVapChunk; g += kVapGroup) {
          double2 nx[kVapGroup];
#pragma unroll
          for (int s = 0; s < kVapGroup; ++s)
            if (g + kVapGroup < kVapChunk) nx[s] = cb[(g + kVapGroup + s) * kWave];
#pragma unroll
          for (int s = 0; s < kVapGroup; ++s) apply(cw[s]);
#pragma unroll
          for (int s = 0; s < kVapGroup; ++s) cw[s] = nx[s];
        }
      } else {
        const int ns = (int)(T - ch * kVapChunk);
        for (int s = 0; s < ns; ++s) apply(cb[s * kWave]);
      }
#pragma unroll
      for (int jj = 0; jj < kVapLoads; ++jj) cbuf[buf ^ 1][threadIdx.x + jj * 64 * kVapWaves] = st[jj];
      __syncthreads();
    }
  }
  // T is a whole number of sweeps: the row is in R (written at the last level end)
  if (r < l)
    for (int j = lane; j < k; j += kWave) Vt[r * ldk + j] = R[vperm[j]];
}

// ---------------------------------------------------------------------------
// Sign convention: for each column j < k of U (rows x ld), the entry of
// largest magnitude (lowest row on ties) is made positive; V's column j is
// flipped with it.  Stage 1: per-block candidates.
__global__ void __launch_bounds__(256)
k_colmax(const double* __restrict__ U, int64_t rows, int ld, int k, int64_t rows_per_block,
         double* __restrict__ pval, int64_t* __restrict__ pidx) {
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(rows, r0 + rows_per_block);
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  for (int c0 = 0; c0 < k; c0 += 64) {
    const int c = c0 + (threadIdx.x % 64);
    const int sub = threadIdx.x / 64;
    double best = -1.0;
    int64_t bidx = -1;
    if (c < k) {
      for (int64_t r = r0 + sub; r < r1; r += 4) {
        const double v = fabs(U[r * ld + c]);
        if (v > best) { best = v; bidx = r; }  // rows visited in increasing order per sub
      }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    if (sub == 0 && c < k) {
      for (int t = 1; t < 4; ++t) {
        const double v = bv[threadIdx.x + 64 * t];
        const int64_t ix = bi[threadIdx.x + 64 * t];
        if (v > best || (v == best && ix >= 0 && (bidx < 0 || ix < bidx))) { best = v; bidx = ix; }
      }
      pval[(int64_t)blockIdx.x * k + c] = best;
      pidx[(int64_t)blockIdx.x * k + c] = bidx;
    }
    __syncthreads();
  }
}

// Stage 2: combine block candidates (max, lowest index on ties) -> signs.
// One workgroup per column; the candidates are combined by a tree in LDS
// (max with lowest index on ties is associative and commutative, so the
// order does not change the result).
__global__ void __launch_bounds__(256)
k_signs(const double* __restrict__ U, int ld, int k, int nblocks, const double* __restrict__ pval,
        const int64_t* __restrict__ pidx, double* __restrict__ sgn) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int c = blockIdx.x;
  double best = -1.0;
  int64_t bidx = -1;
  for (int b = threadIdx.x; b < nblocks; b += 256) {
    const double v = pval[(int64_t)b * k + c];
    const int64_t ix = pidx[(int64_t)b * k + c];
    if (ix < 0) continue;
    if (v > best || (v == best && (bidx < 0 || ix < bidx))) { best = v; bidx = ix; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) {
      const double v = bv[threadIdx.x + off];
      const int64_t ix = bi[threadIdx.x + off];
      const double b0 = bv[threadIdx.x];
      const int64_t i0 = bi[threadIdx.x];
      if (ix >= 0 && (v > b0 || (v == b0 && (i0 < 0 || ix < i0)))) {
        bv[threadIdx.x] = v;
        bi[threadIdx.x] = ix;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t ix = bi[0];
    sgn[c] = (ix >= 0 && U[ix * ld + c] < 0.0) ? -1.0 : 1.0;
  }
}

// Stage 3: out[r][c] = sgn[c] * src[r][c] for c < k, in FP64 or FP32.
template <typename TO>
__global__ void __launch_bounds__(256)
k_apply_signs(const double* __restrict__ src, int64_t rows, int lds, int k,
              const double* __restrict__ sgn, TO* __restrict__ out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * k) return;
  const int64_t r = idx / k;
  const int c = (int)(idx % k);
  out[r * ldo + c] = (TO)(sgn[c] * src[r * lds + c]);
}

// ---------------------------------------------------------------------------
// Result record: ||A||_F from the per-block sums of squares of the first pass
// (summed in a fixed order), and the error by the split of Th. 2:
// ||A - Q1 M_k Q2^T||_F^2 = ||A||_F^2 - sum_{j<=k} sigma_j^2.
__global__ void __launch_bounds__(256)
k_finalize(const double* __restrict__ normp, int nparts, const double* __restrict__ sv, int k,
           DevInfo* __restrict__ info) {
  __shared__ double part[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < nparts; i += 256) a += normp[i];
  part[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double a2 = part[0];
    double s2 = 0.0;
    for (int j = 0; j < k; ++j) s2 += sv[j] * sv[j];
    info->a_fro = sqrt(a2);
    if (!(a2 - a2 == 0.0)) atomicOr(&info->flags, kFlagNonFinite);
    info->err_fro = a2 > 0.0 ? sqrt(fmax(a2 - s2, 0.0)) / sqrt(a2) : 0.0;
  }
}

__global__ void __launch_bounds__(64) k_info_init(DevInfo* info) {
  if (threadIdx.x == 0) {
    info->a_fro = 0.0;
    info->err_fro = 0.0;
    info->err_fro_explicit = -1.0;
    info->sweeps = 0;
    info->flags = 0;
    info->a_noise_rel = 0.0;
  }
}

__global__ void __launch_bounds__(256) k_fill(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_chol_inv(const double* G, int LP, int l, int64_t rows, int mode, double* Rinv,
                           int* skip3, void* info, hipStream_t st) {
  const size_t shm = chol_lds(l);
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kSmallThreads), shm, st, G, LP, l, rows, mode, Rinv,
                     skip3, (DevInfo*)info);
  return hipGetLastError();
}

template <bool V_LDS, bool WANT_V>
static void launch_jacobi_nrb(int nrb, size_t shm, hipStream_t st, const double* M, int LP, int l, int k,
                              int max_sweeps, double tol2, double* Ut, double* sv, double* Vt, int ldk,
                              double* Vg, DevInfo* info, double2* rlog = nullptr, int* vperm = nullptr) {
#define SOR_JAC(R)                                                                                       \
  case R:                                                                                                \
    hipLaunchKernelGGL((k_jacobi<V_LDS, WANT_V, R>), dim3(1), dim3(kJacThreads), shm, st, M, LP, l, k,  \
                       max_sweeps, tol2, Ut, sv, Vt, ldk, Vg, info, rlog, vperm);                        \
    break;
  switch (nrb) {
    SOR_JAC(1) SOR_JAC(2) SOR_JAC(4) SOR_JAC(6) SOR_JAC(8) SOR_JAC(10) SOR_JAC(13) SOR_JAC(16)
    default: break;
  }
#undef SOR_JAC
}

// Bytes of the rotation log of a core SVD of width l with up to max_sweeps
// sweeps, plus the permutation (see jacobi_body).
size_t jacobi_log_bytes(int l, int max_sweeps) {
  return (size_t)max_sweeps * jac_sweep_steps(l) * jac_groups(l) * sizeof(double2) + 128 * sizeof(int);
}

// Whether the core SVD of width l rebuilds V from the rotation log: for
// widths above 32, where moving V through LDS at every step of the Jacobi
// kernel costs more than the replay (l = 100: 1.55 ms for the Jacobi kernel
// with V, 0.96 ms without it plus 0.07 ms of replay; l = 64: 0.47 ms with V,
// 0.39 ms without).
bool jacobi_uses_log(int l) { return l > 32; }

// tol <= 0 selects the default orthogonality threshold sqrt(l) 2^-52. rlog:
// jacobi_log_bytes(l, max_sweeps) bytes of scratch, or null (V kept in the
// Jacobi kernel).
hipError_t launch_jacobi(const double* M, int LP, int l, int k, int max_sweeps, double* Ut,
                         double* sv, double* Vt, int ldk, double* Vg, void* info, hipStream_t st,
                         bool want_v, double tol, void* rlog) {
  if (l < 1 || l > 128) return hipErrorInvalidValue;
  const double tol2 = tol > 0.0 ? tol * tol : (double)l * 0x1p-104;
  const int nrb = jac_nrb(l);
  DevInfo* di = (DevInfo*)info;
  if (want_v && rlog && jacobi_uses_log(l)) {
    bool v_lds = false;
    const size_t shm = jacobi_lds(l, false, &v_lds);
    double2* lg = reinterpret_cast<double2*>(rlog);
    int* perm = reinterpret_cast<int*>(lg + (size_t)max_sweeps * jac_sweep_steps(l) * jac_groups(l));
    launch_jacobi_nrb<false, false>(nrb, shm, st, M, LP, l, k, max_sweeps, tol2, Ut, sv, Vt, ldk, Vg, di, lg, perm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int blocks = (int)ceil_div(l, kVapWaves);
    hipLaunchKernelGGL(k_jacobi_vapply, dim3(blocks), dim3(64 * kVapWaves), 0, st, lg, perm, di, l, k, max_sweeps,
                       Vt, ldk);
    return hipGetLastError();
  }
  bool v_lds = false;
  const size_t shm = jacobi_lds(l, want_v, &v_lds);
  if (!want_v)
    launch_jacobi_nrb<false, false>(nrb, shm, st, M, LP, l, k, max_sweeps, tol2, Ut, sv, Vt, ldk, Vg, di);
  else if (v_lds)
    launch_jacobi_nrb<true, true>(nrb, shm, st, M, LP, l, k, max_sweeps, tol2, Ut, sv, Vt, ldk, Vg, di);
  else
    launch_jacobi_nrb<false, true>(nrb, shm, st, M, LP, l, k, max_sweeps, tol2, Ut, sv, Vt, ldk, Vg, di);
  return hipGetLastError();
}

// U, V: double* (out_f32 = 0) or float* (out_f32 = 1).
hipError_t launch_signfix(const double* U64, int64_t m, const double* V64, int64_t n, int ld, int k,
                          double* pval, int64_t* pidx, int nblocks_max, double* sgn, void* U,
                          int64_t ldu, void* V, int64_t ldv, hipStream_t st, int out_f32) {
  if (k == 0) return hipSuccess;
  int64_t rpb = ceil_div(m, nblocks_max);
  rpb = rpb < 64 ? 64 : rpb;
  const int nb = (int)ceil_div(m, rpb);
  if (nb > 0) {
    hipLaunchKernelGGL(k_colmax, dim3(nb), dim3(256), 0, st, U64, m, ld, k, rpb, pval, pidx);
    hipLaunchKernelGGL(k_signs, dim3(k), dim3(256), 0, st, U64, ld, k, nb, pval, pidx, sgn);
  }
  const dim3 gu((unsigned)ceil_div(m * k, 256)), gv((unsigned)ceil_div(n * k, 256));
  if (out_f32) {
    if (m * k > 0) hipLaunchKernelGGL(k_apply_signs<float>, gu, dim3(256), 0, st, U64, m, ld, k, sgn, (float*)U, ldu);
    if (n * k > 0) hipLaunchKernelGGL(k_apply_signs<float>, gv, dim3(256), 0, st, V64, n, ld, k, sgn, (float*)V, ldv);
  } else {
    if (m * k > 0) hipLaunchKernelGGL(k_apply_signs<double>, gu, dim3(256), 0, st, U64, m, ld, k, sgn, (double*)U, ldu);
    if (n * k > 0) hipLaunchKernelGGL(k_apply_signs<double>, gv, dim3(256), 0, st, V64, n, ld, k, sgn, (double*)V, ldv);
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const double* normp, int nparts, const double* sv, int k, void* info,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, st, normp, nparts, sv, k, (DevInfo*)info);
  return hipGetLastError();
}

hipError_t launch_info_init(void* info, hipStream_t st) {
  hipLaunchKernelGGL(k_info_init, dim3(1), dim3(64), 0, st, (DevInfo*)info);
  return hipGetLastError();
}

hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace sor
