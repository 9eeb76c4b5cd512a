// Small dense FP64 kernels of the SOR-SVD path, each run by one workgroup:
//   * Cholesky factor and inverse of the l x l Gram matrix (the QR step of
//     Alg. 3 / Alg. 4 as Cholesky QR: T = Q R with R^T R = T^T T),
//   * the core SVD of M = Q1^T A Q2 by one-sided (Hestenes) Jacobi rotations
//     with a round-robin pair order (rank-k truncation of Alg. 3 step 6),
//   * sign convention and assembly of the lifted factors, and the error record.
#include "common.hpp"

namespace sor {

constexpr int kSmallThreads = 1024;

// Flags stored in the int32 `flags` word of the result record.
constexpr int kFlagNoConv = 1;
constexpr int kFlagNonFinite = 2;
constexpr int kFlagQrBreakdown = 4;

struct DevInfo {  // mirrors sorsvd_info
  double a_fro;
  double err_fro;
  double err_fro_explicit;
  int32_t sweeps;
  int32_t flags;
};

// ---------------------------------------------------------------------------
// Cholesky QR step. G (ld LP) holds T^T T for the current T (rows x l).
// Computes R with R^T R = G (+ shift I) and writes Rinv = R^{-1} into an
// LP x LP zero-padded buffer; the caller then forms T <- T Rinv.
//   mode 0 (first step): unshifted; if a pivot shows column j nearly in the
//          span of the earlier ones (Schur pivot < 1e-13 G_jj, i.e. a condition
//          number beyond ~3e6, or a breakdown), the factorisation is redone with
//          the shift c u tr(G), c = 11 (rows l + l (l + 1)), u = 2^-53 (shifted
//          Cholesky QR, Fukaya et al.), and a third step is requested through
//          *skip3 = 0; otherwise *skip3 = 1.
//   mode 1 (second step): unshifted.
//   mode 2 (third step): does nothing when *skip3 is set.
// Two unshifted steps leave T orthonormal to rounding when its condition
// number is below ~1e7; the shifted first step brings any T with condition
// number up to ~1/u into that range.
constexpr int kCholRetry = 1;

// LDL^T elimination of the l x l SPD matrix held in the upper triangle of S,
// carrying W = L^{-1} (unit lower triangular) in the strict lower triangle:
// step j subtracts f_a = S[j][a] / S[j][j] times row j from every row a > j,
// on the trailing upper triangle of S and on W's columns 0..j. The pivots
// d_j stay on the diagonal. One barrier per step. Then R = D^{1/2} L^T and
// R^{-1} = L^{-T} D^{-1/2} = W^T D^{-1/2}.
__device__ int ldl_inverse(double* S, int l, double shift, const double* d0, bool check,
                           DevInfo* info) {
  const int tid = threadIdx.x;
  const int tx = tid % 32, ty = tid / 32;
  if (shift != 0.0)
    for (int i = tid; i < l; i += kSmallThreads) S[i * l + i] += shift;
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    double d = S[j * l + j];
    if (check && !(d > 1e-13 * d0[j])) return kCholRetry;  // every thread sees the same d
    if (!(d > 0.0)) {  // breakdown after the shift (or NaN): record it, continue with a tiny pivot
      if (tid == 0) atomicOr(&info->flags, kFlagQrBreakdown);
      d = 0x1p-1000;
    }
    const double dinv = 1.0 / d;
    const double* rowj = S + j * l;
    for (int a = j + 1 + ty; a < l; a += kSmallThreads / 32) {
      const double f = rowj[a] * dinv;
      double* rowa = S + a * l;
#pragma unroll 4
      for (int c = a + tx; c < l; c += 32) rowa[c] -= f * rowj[c];
#pragma unroll 4
      for (int c = tx; c <= j; c += 32) rowa[c] -= f * (c == j ? 1.0 : rowj[c]);
    }
    __syncthreads();
  }
  return 0;
}

__global__ void __launch_bounds__(kSmallThreads)
k_chol_inv(const double* __restrict__ G, int LP, int l, int64_t rows, int mode,
           double* __restrict__ Rinv, int* __restrict__ skip3, DevInfo* __restrict__ info) {
  if (mode == 2 && *skip3) return;
  extern __shared__ double sm[];
  double* S = sm;               // l x l: upper = S, strict lower = W
  double* d0 = sm + l * l;      // l: diagonal of G
  const int tid = threadIdx.x;

  auto load = [&]() {
    for (int i = tid; i < l * l; i += kSmallThreads) {
      const int r = i / l, c = i % l;
      S[i] = (c >= r) ? G[r * LP + c] : 0.0;
    }
  };
  load();
  for (int i = tid; i < l; i += kSmallThreads) d0[i] = G[i * LP + i];
  __syncthreads();
  if (mode == 0) {
    if (ldl_inverse(S, l, 0.0, d0, true, info) == kCholRetry) {
      __syncthreads();
      double tr = 0.0;
      for (int i = 0; i < l; ++i) tr += d0[i];
      const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 0x1p-53 * tr;
      load();
      __syncthreads();
      ldl_inverse(S, l, shift, d0, false, info);
      if (tid == 0) *skip3 = 0;
    } else if (tid == 0) {
      *skip3 = 1;
    }
  } else {
    ldl_inverse(S, l, 0.0, d0, false, info);
  }
  __syncthreads();
  // R^{-1}[r][c] = W[c][r] / sqrt(d_c) for r < c, 1 / sqrt(d_c) on the diagonal.
  for (int i = tid; i < LP * LP; i += kSmallThreads) {
    const int r = i / LP, c = i % LP;
    double v = 0.0;
    if (r < l && c < l && c >= r) {
      double d = S[c * l + c];
      if (!(d > 0.0)) d = 0x1p-1000;
      const double isd = 1.0 / sqrt(d);
      v = (r == c) ? isd : S[c * l + r] * isd;
    }
    Rinv[i] = v;
  }
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of an l x l matrix M (ld LP), FP64, l <= 128.
// Columns are rotated in pairs (p, q): with alpha = |m_p|^2, beta = |m_q|^2,
// gamma = m_p . m_q, zeta = (beta - alpha) / (2 gamma),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t,
// m_p <- c m_p - s m_q, m_q <- s m_p + c m_q (and the same on V), which makes
// the pair orthogonal. A sweep visits every pair once in round-robin order
// (l' - 1 steps of l'/2 disjoint pairs, l' = l rounded up to even); sweeps
// stop when no pair had |gamma| > tol sqrt(alpha beta), tol = sqrt(l) 2^-52,
// or after max_sweeps. Then sigma_j = |m_j|, U~_j = m_j / sigma_j, V~_j = v_j,
// sorted descending; the first k are written (Ut, Vt: l x k, ld ldk; s: k).
// Each pair is handled by a group of 16 lanes (one DPP row); each lane keeps
// its (at most 8) rows of the two columns in registers for the step, and the
// dot products are reduced with DPP. M lives in LDS; V lives in LDS when both
// fit, else in the global scratch `Vg` (l x l).
constexpr int kJacRows = 8;  // rows per lane: l <= 16 * kJacRows

template <bool V_LDS>
__global__ void __launch_bounds__(kSmallThreads)
k_jacobi(const double* __restrict__ Min, int LP, int l, int k, int max_sweeps,
         double* __restrict__ Ut, double* __restrict__ sv, double* __restrict__ Vt, int ldk,
         double* __restrict__ Vg, DevInfo* __restrict__ info) {
  extern __shared__ double sm[];
  double* Mc = sm;                             // column-major: Mc[c * l + r]
  double* Vc;                                  // column-major
  if constexpr (V_LDS) Vc = sm + l * l; else Vc = Vg;
  double* sig = sm + (V_LDS ? 2 * l * l : l * l);  // l
  __shared__ int s_rot;
  const int tid = threadIdx.x;
  const int grp = tid / 16, gl = tid % 16;
  constexpr int ngroups = kSmallThreads / 16;

  for (int i = tid; i < l * l; i += kSmallThreads) {
    const int c = i / l, r = i % l;
    Mc[i] = Min[r * LP + c];
    Vc[i] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();

  const int lp = (l + 1) & ~1;
  const int npairs = lp / 2;
  const double tol2 = (double)l * 0x1p-104;  // (sqrt(l) 2^-52)^2
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int step = 0; step < lp - 1; ++step) {
      for (int pr = grp; pr < npairs; pr += ngroups) {
        // round-robin: position 0 fixed, positions 1..lp-1 rotate
        auto player = [&](int pos) {
          if (pos == 0) return 0;
          int x = pos - 1 + step;
          if (x >= lp - 1) x -= lp - 1;
          return 1 + x;
        };
        int p = player(pr), q = player(lp - 1 - pr);
        if (p >= l || q >= l) continue;
        if (p > q) { int t = p; p = q; q = t; }
        double* mp = Mc + p * l;
        double* mq = Mc + q * l;
        double* vp = Vc + p * l;
        double* vq = Vc + q * l;
        double x[kJacRows], y[kJacRows], vx[kJacRows], vy[kJacRows];
#pragma unroll
        for (int i = 0; i < kJacRows; ++i) {
          // clamped, unconditional loads (all issued before the first use)
          const int r = gl + 16 * i;
          const int rc = r < l ? r : l - 1;
          const double a = mp[rc], b = mq[rc], va = vp[rc], vb = vq[rc];
          const bool in = r < l;
          x[i] = in ? a : 0.0;
          y[i] = in ? b : 0.0;
          vx[i] = in ? va : 0.0;
          vy[i] = in ? vb : 0.0;
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int i = 0; i < kJacRows; ++i) {
          al += x[i] * x[i]; be += y[i] * y[i]; ga += x[i] * y[i];
        }
        al = sum16(al); be = sum16(be); ga = sum16(ga);
        if (!(ga * ga > tol2 * (al * be))) continue;  // orthogonal enough (or zero column)
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
#pragma unroll
        for (int i = 0; i < kJacRows; ++i) {
          const int r = gl + 16 * i;
          if (r < l) {
            mp[r] = c * x[i] - s * y[i];
            mq[r] = s * x[i] + c * y[i];
            vp[r] = c * vx[i] - s * vy[i];
            vq[r] = s * vx[i] + c * vy[i];
          }
        }
        if (gl == 0) s_rot = 1;
      }
      __syncthreads();
    }
    const int rot = s_rot;
    __syncthreads();
    if (!rot) break;
  }
  if (tid == 0) {
    info->sweeps = sweep + (sweep < max_sweeps ? 1 : 0);
    if (sweep >= max_sweeps) atomicOr(&info->flags, kFlagNoConv);
  }
  // column norms -> singular values
  for (int c = grp; c < l; c += ngroups) {
    double a = 0.0;
    for (int r = gl; r < l; r += 16) a += Mc[c * l + r] * Mc[c * l + r];
    a = sum16(a);
    if (gl == 0) sig[c] = sqrt(a);
  }
  __syncthreads();
  // rank of each column in descending order (ties: lower index first)
  for (int c = grp; c < l; c += ngroups) {
    const double sc = sig[c];
    int rank = 0;
    for (int i = gl; i < l; i += 16) rank += (sig[i] > sc || (sig[i] == sc && i < c)) ? 1 : 0;
    for (int off = 8; off >= 1; off >>= 1) rank += __shfl_xor(rank, off, kWave);
    if (rank < k) {
      const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
      for (int r = gl; r < l; r += 16) {
        Ut[r * ldk + rank] = Mc[c * l + r] * inv;
        Vt[r * ldk + rank] = Vc[c * l + r];
      }
      if (gl == 0) sv[rank] = sc;
    }
  }
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

// Stage 3: out[r][c] = sgn[c] * src[r][c] for c < k.
__global__ void __launch_bounds__(256)
k_apply_signs(const double* __restrict__ src, int64_t rows, int lds, int k,
              const double* __restrict__ sgn, double* __restrict__ out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= rows * k) return;
  const int64_t r = idx / k;
  const int c = (int)(idx % k);
  out[r * ldo + c] = sgn[c] * src[r * lds + c];
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
  }
}

__global__ void __launch_bounds__(256) k_fill(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ launchers

hipError_t launch_chol_inv(const double* G, int LP, int l, int64_t rows, int mode, double* Rinv,
                           int* skip3, void* info, hipStream_t st) {
  const size_t shm = ((size_t)l * l + l) * sizeof(double);
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kSmallThreads), shm, st, G, LP, l, rows, mode, Rinv,
                     skip3, (DevInfo*)info);
  return hipGetLastError();
}

static size_t jacobi_lds_bytes(int l, int* v_in_lds) {
  const size_t one = (size_t)l * l * sizeof(double);
  const size_t vec = (size_t)l * sizeof(double);
  const size_t limit = 160 * 1024 - 256;  // room for the static LDS words
  *v_in_lds = (2 * one + vec <= limit) ? 1 : 0;
  return (*v_in_lds ? 2 * one : one) + vec;
}

hipError_t launch_jacobi(const double* M, int LP, int l, int k, int max_sweeps, double* Ut,
                         double* sv, double* Vt, int ldk, double* Vg, void* info, hipStream_t st) {
  int v_in_lds = 0;
  const size_t shm = jacobi_lds_bytes(l, &v_in_lds);
  if (v_in_lds)
    hipLaunchKernelGGL(k_jacobi<true>, dim3(1), dim3(kSmallThreads), shm, st, M, LP, l, k, max_sweeps,
                       Ut, sv, Vt, ldk, Vg, (DevInfo*)info);
  else
    hipLaunchKernelGGL(k_jacobi<false>, dim3(1), dim3(kSmallThreads), shm, st, M, LP, l, k, max_sweeps,
                       Ut, sv, Vt, ldk, Vg, (DevInfo*)info);
  return hipGetLastError();
}

hipError_t launch_signfix(const double* U64, int64_t m, const double* V64, int64_t n, int ld, int k,
                          double* pval, int64_t* pidx, int nblocks_max, double* sgn, double* U,
                          int64_t ldu, double* V, int64_t ldv, hipStream_t st) {
  if (k == 0) return hipSuccess;
  int64_t rpb = ceil_div(m, nblocks_max);
  rpb = rpb < 64 ? 64 : rpb;
  const int nb = (int)ceil_div(m, rpb);
  if (nb > 0) {
    hipLaunchKernelGGL(k_colmax, dim3(nb), dim3(256), 0, st, U64, m, ld, k, rpb, pval, pidx);
    hipLaunchKernelGGL(k_signs, dim3(k), dim3(256), 0, st, U64, ld, k, nb, pval, pidx, sgn);
  }
  if (m * k > 0)
    hipLaunchKernelGGL(k_apply_signs, dim3((unsigned)ceil_div(m * k, 256)), dim3(256), 0, st, U64, m, ld, k, sgn, U, ldu);
  if (n * k > 0)
    hipLaunchKernelGGL(k_apply_signs, dim3((unsigned)ceil_div(n * k, 256)), dim3(256), 0, st, V64, n, ld, k, sgn, V, ldv);
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
