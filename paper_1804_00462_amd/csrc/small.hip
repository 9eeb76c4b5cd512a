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
// Cholesky QR step. G (ldg = LP) holds T^T T for the current T (rows x l).
// Computes R with R^T R = G + shift I (shift = c u tr(G) when `shifted`,
// c = 11 (rows l + l (l + 1)), u = 2^-53: the shifted Cholesky QR of Fukaya et
// al., which keeps the factorisation defined for condition numbers up to
// about 1/u) and writes Rinv = R^{-1} into an LP x LP zero-padded buffer.
// When `may_skip` is set and max |G - I| <= 1e-14, T is already orthonormal:
// Rinv = I and *skip = 1 (the caller's product kernel then leaves T alone).
__global__ void __launch_bounds__(kSmallThreads)
k_chol_inv(const double* __restrict__ G, int LP, int l, int64_t rows, int shifted, int may_skip,
           double* __restrict__ Rinv, int* __restrict__ skip, DevInfo* __restrict__ info) {
  extern __shared__ double sm[];
  double* R = sm;               // l x l, row-major (upper triangle used)
  double* tmp = sm + l * l;     // l
  __shared__ double s_shift;
  __shared__ unsigned long long s_dev;
  __shared__ int s_skip;
  const int tid = threadIdx.x;

  for (int i = tid; i < l * l; i += kSmallThreads) R[i] = G[(i / l) * LP + (i % l)];
  if (tid == 0) { s_dev = 0ull; s_skip = 0; }
  __syncthreads();
  if (may_skip) {
    double dev = 0.0;
    for (int i = tid; i < l * l; i += kSmallThreads) {
      const double e = R[i] - ((i / l == i % l) ? 1.0 : 0.0);
      dev = fmax(dev, fabs(e));
    }
    for (int off = 32; off >= 1; off >>= 1) dev = fmax(dev, __shfl_xor(dev, off, kWave));
    // non-negative doubles order like their bit patterns
    if ((tid & 63) == 0) atomicMax(&s_dev, (unsigned long long)__double_as_longlong(dev));
    __syncthreads();
    if (tid == 0) s_skip = (__longlong_as_double((long long)s_dev) <= 1e-14) ? 1 : 0;
    __syncthreads();
  }
  if (s_skip) {
    for (int i = tid; i < LP * LP; i += kSmallThreads) Rinv[i] = (i / LP == i % LP && i / LP < l) ? 1.0 : 0.0;
    if (tid == 0) *skip = 1;
    return;
  }
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < l; ++i) tr += R[i * l + i];
    s_shift = shifted ? 11.0 * ((double)rows * l + (double)l * (l + 1)) * 0x1p-53 * tr : 0.0;
    if (skip) *skip = 0;
  }
  __syncthreads();
  for (int i = tid; i < l; i += kSmallThreads) R[i * l + i] += s_shift;
  __syncthreads();

  // Right-looking Cholesky on the upper triangle: R[j][j..] becomes row j of R.
  for (int j = 0; j < l; ++j) {
    if (tid == 0) {
      double d = R[j * l + j];
      if (!(d > 0.0)) {  // breakdown (or NaN): record it, continue with a tiny pivot
        atomicOr(&info->flags, kFlagQrBreakdown);
        d = 0x1p-1000;
      }
      R[j * l + j] = sqrt(d);
    }
    __syncthreads();
    const double inv = 1.0 / R[j * l + j];
    for (int c = j + 1 + tid; c < l; c += kSmallThreads) R[j * l + c] *= inv;
    __syncthreads();
    const int m = l - j - 1;  // trailing size
    for (int t = tid; t < m * m; t += kSmallThreads) {
      const int a = j + 1 + t / m, c = j + 1 + t % m;
      if (c >= a) R[a * l + c] -= R[j * l + a] * R[j * l + c];
    }
    __syncthreads();
  }
  // In-place inverse of the upper triangular R, column by column:
  // with R = [[R11, r], [0, rho]], R^{-1} = [[R11^{-1}, -R11^{-1} r / rho], [0, 1/rho]].
  for (int j = 0; j < l; ++j) {
    for (int i = tid; i < j; i += kSmallThreads) {
      double acc = 0.0;
      for (int t = i; t < j; ++t) acc += R[i * l + t] * R[t * l + j];
      tmp[i] = acc;
    }
    __syncthreads();
    const double rinv = 1.0 / R[j * l + j];
    for (int i = tid; i < j; i += kSmallThreads) R[i * l + j] = -tmp[i] * rinv;
    __syncthreads();
    if (tid == 0) R[j * l + j] = rinv;
    __syncthreads();
  }
  for (int i = tid; i < LP * LP; i += kSmallThreads) {
    const int r = i / LP, c = i % LP;
    Rinv[i] = (r < l && c < l && c >= r) ? R[r * l + c] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of an l x l matrix M (ld LP), FP64.
// Columns are rotated in pairs (p, q): with alpha = |m_p|^2, beta = |m_q|^2,
// gamma = m_p . m_q, zeta = (beta - alpha) / (2 gamma),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t,
// m_p <- c m_p - s m_q, m_q <- s m_p + c m_q (and the same on V), which makes
// the pair orthogonal. A sweep visits every pair once in round-robin order
// (l' - 1 steps of l'/2 disjoint pairs, l' = l rounded up to even); sweeps
// stop when no pair had |gamma| > tol sqrt(alpha beta), tol = sqrt(l) 2^-52,
// or after max_sweeps. Then sigma_j = |m_j|, U~_j = m_j / sigma_j, V~_j = v_j,
// sorted descending; the first k are written (Ut, Vt: l x k, ld ldk; s: k).
// Each pair is handled by a group of 16 lanes. M lives in LDS; V lives in LDS
// when both fit, else in the global scratch `Vg` (l x l).
__global__ void __launch_bounds__(kSmallThreads)
k_jacobi(const double* __restrict__ Min, int LP, int l, int k, int max_sweeps,
         double* __restrict__ Ut, double* __restrict__ sv, double* __restrict__ Vt, int ldk,
         double* __restrict__ Vg, int v_in_lds, DevInfo* __restrict__ info) {
  extern __shared__ double sm[];
  double* Mc = sm;                             // column-major: Mc[c * l + r]
  double* Vc = v_in_lds ? sm + l * l : Vg;     // column-major
  double* sig = sm + (v_in_lds ? 2 * l * l : l * l);  // l
  __shared__ int s_rot;
  __shared__ int s_sweeps;
  const int tid = threadIdx.x;
  const int grp = tid / 16, gl = tid % 16;
  constexpr int ngroups = kSmallThreads / 16;

  for (int i = tid; i < l * l; i += kSmallThreads) {
    const int c = i / l, r = i % l;
    Mc[i] = Min[r * LP + c];
    Vc[i] = (r == c) ? 1.0 : 0.0;
  }
  if (tid == 0) s_sweeps = 0;
  __syncthreads();

  const int lp = (l + 1) & ~1;
  const int npairs = lp / 2;
  const double tol = sqrt((double)l) * 0x1p-52;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int step = 0; step < lp - 1; ++step) {
      for (int pr = grp; pr < npairs; pr += ngroups) {
        // round-robin: position 0 fixed, positions 1..lp-1 rotate
        auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + step) % (lp - 1); };
        int p = player(pr), q = player(lp - 1 - pr);
        if (p >= l || q >= l) continue;
        if (p > q) { int t = p; p = q; q = t; }
        double* mp = Mc + p * l;
        double* mq = Mc + q * l;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int r = gl; r < l; r += 16) {
          const double x = mp[r], y = mq[r];
          al += x * x; be += y * y; ga += x * y;
        }
        al = group_sum(al, 16); be = group_sum(be, 16); ga = group_sum(ga, 16);
        if (!(fabs(ga) > tol * sqrt(al * be))) continue;  // orthogonal enough (or zero column)
        const double zeta = (be - al) / (2.0 * ga);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
        for (int r = gl; r < l; r += 16) {
          const double x = mp[r], y = mq[r];
          mp[r] = c * x - s * y;
          mq[r] = s * x + c * y;
        }
        double* vp = Vc + p * l;
        double* vq = Vc + q * l;
        for (int r = gl; r < l; r += 16) {
          const double x = vp[r], y = vq[r];
          vp[r] = c * x - s * y;
          vq[r] = s * x + c * y;
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
    a = group_sum(a, 16);
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
__global__ void __launch_bounds__(256)
k_signs(const double* __restrict__ U, int ld, int k, int nblocks, const double* __restrict__ pval,
        const int64_t* __restrict__ pidx, double* __restrict__ sgn) {
  for (int c = threadIdx.x; c < k; c += 256) {
    double best = -1.0;
    int64_t bidx = -1;
    for (int b = 0; b < nblocks; ++b) {
      const double v = pval[(int64_t)b * k + c];
      const int64_t ix = pidx[(int64_t)b * k + c];
      if (ix < 0) continue;
      if (v > best || (v == best && ix < bidx)) { best = v; bidx = ix; }
    }
    sgn[c] = (bidx >= 0 && U[bidx * ld + c] < 0.0) ? -1.0 : 1.0;
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

hipError_t launch_chol_inv(const double* G, int LP, int l, int64_t rows, int shifted, int may_skip,
                           double* Rinv, int* skip, void* info, hipStream_t st) {
  const size_t shm = ((size_t)l * l + l) * sizeof(double);
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(kSmallThreads), shm, st, G, LP, l, rows, shifted,
                     may_skip, Rinv, skip, (DevInfo*)info);
  return hipGetLastError();
}

size_t jacobi_lds_bytes(int l, int* v_in_lds) {
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
  hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(kSmallThreads), shm, st, M, LP, l, k, max_sweeps, Ut,
                     sv, Vt, ldk, Vg, v_in_lds, (DevInfo*)info);
  return hipGetLastError();
}

hipError_t launch_signfix(const double* U64, int64_t m, const double* V64, int64_t n, int ld, int k,
                          double* pval, int64_t* pidx, int nblocks_max, double* sgn, double* U,
                          int64_t ldu, double* V, int64_t ldv, hipStream_t st) {
  if (k == 0) return hipSuccess;
  int64_t rpb = ceil_div(m, nblocks_max);
  rpb = rpb < 256 ? 256 : rpb;
  const int nb = (int)ceil_div(m, rpb);
  if (nb > 0) {
    hipLaunchKernelGGL(k_colmax, dim3(nb), dim3(256), 0, st, U64, m, ld, k, rpb, pval, pidx);
    hipLaunchKernelGGL(k_signs, dim3(1), dim3(256), 0, st, U64, ld, k, nb, pval, pidx, sgn);
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
