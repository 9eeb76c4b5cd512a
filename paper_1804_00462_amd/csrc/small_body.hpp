// Device bodies of the small dense FP64 steps of the SOR-SVD path, each run
// by one workgroup of kSmallThreads threads (shared by the single-problem
// kernels and the batched kernels, which run one workgroup per problem):
//   * Cholesky factor and inverse of the l x l Gram matrix (the QR step of
//     Alg. 3 / Alg. 4 as Cholesky QR: T = Q R with R^T R = T^T T),
//   * the core SVD of M = Q1^T A Q2 by one-sided (Hestenes) Jacobi rotations
//     with a round-robin pair order (rank-k truncation of Alg. 3 step 6).
#pragma once
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
  double a_noise_rel;
};

// ---------------------------------------------------------------------------
// Cholesky QR step. G (ld LP) holds T^T T for the current T (rows x l).
// Computes R with R^T R = G (+ shift I) and writes Rinv = R^{-1} into an
// LP x LP zero-padded buffer; the caller then forms T <- T Rinv.
// Every step first factors G unshifted; if a pivot shows column j nearly in
// the span of the earlier ones (Schur pivot < 1e-13 G_jj, i.e. a condition
// number beyond ~3e6, or a breakdown), it factors again with the shift
// c u tr(G), c = 11 (rows l + l (l + 1)), u = 2^-53 (shifted Cholesky QR,
// Fukaya et al.), and asks for the third step through *skip3 = 0.
//   mode 0 (first step): sets *skip3 = 1 when no shift was needed;
//   mode 1 (second step): leaves *skip3 alone unless it shifted;
//   mode 2 (third step): does nothing when *skip3 is set.
// Two unshifted steps leave T orthonormal to rounding when its condition
// number is below ~1e7; the shifted step brings any T with condition number
// up to ~1/u into that range. A pivot that is still not positive after the
// shift (a column dependent to rounding, or NaN) drops its column: it
// eliminates nothing and its column of R^{-1} is zero (flag bit 2).

// LDL^T elimination of the l x l SPD matrix G (+ shift on the diagonal),
// carrying W = L^{-1} (unit lower triangular) in the strict lower part of each
// row: step j subtracts f_a = S[j][a] / S[j][j] times row j from every row
// a > j, on the trailing upper part (columns >= a) and on W's columns 0..j.
// The pivots d_j stay on the diagonal. Then R = D^{1/2} L^T and
// R^{-1} = L^{-T} D^{-1/2} = W^T D^{-1/2}.
//
// Dataflow form: wave w holds rows a = w + 16 i in registers (lane holds
// columns lane and lane + 64) and finishes them in increasing order, each by
// applying the steps j < a in order from the published rows j (left-looking:
// the same operations in the same order as the row-by-row elimination). A
// finished row is published to LDS with 1 in place of its pivot d_a (the
// unit diagonal of W, which is what the later steps subtract) and with
// 1/d_a beside it, and a counter of published
// rows is raised; rows finish in index order, so the chain costs one step and
// one hand-off per row instead of a workgroup barrier per step. Every wait is
// bounded: after ~1e6 polls a wave stops waiting and the result is flagged as
// a breakdown.
constexpr int kCholWaves = kSmallThreads / 64;
constexpr int kCholRowsPerWave = (128 + kCholWaves - 1) / kCholWaves;  // l <= 128

struct CholRows {
  double v[kCholRowsPerWave][2];
};

__device__ inline double chol_gval(const double* __restrict__ G, int nparts, int64_t pstride, int LP, int r,
                                   int c) {
  double v = 0.0;
  for (int p = 0; p < nparts; ++p) v += G[p * pstride + r * LP + c];
  return v;
}

// check: a pivot below 1e-13 of the original diagonal sets *retry (every
// wave finishes its rows regardless, so that no wait is left open). Pub: LDS
// of l * l doubles; pinv: l doubles; *nready and *retry zero on entry.
__device__ inline void ldl_flow(const double* __restrict__ G, int nparts, int64_t pstride, int LP, int l,
                                double shift, const double* d0, bool check, double* Pub, double* pinv,
                                int* nready, int* retry, DevInfo* info, CholRows& R) {
  // (the wave index through readfirstlane: known uniform, so that row and
  // step bounds live in scalar registers and the loops are not divergent)
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  bool bail = false;
  int known = 0;  // rows known to be published
  // this wave's rows of G (upper part), the parts added in order: all loads of
  // a part are issued before the first is used (entries outside the upper
  // part read a valid address and are dropped)
#pragma unroll
  for (int i = 0; i < kCholRowsPerWave; ++i)
#pragma unroll
    for (int h = 0; h < 2; ++h) R.v[i][h] = 0.0;
  for (int p = 0; p < nparts; ++p) {
    double gv[kCholRowsPerWave][2];
#pragma unroll
    for (int i = 0; i < kCholRowsPerWave; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int a = w + kCholWaves * i, c = lane + 64 * h;
        const bool in = a < l && c < l && c >= a;
        gv[i][h] = G[p * pstride + (in ? a * LP + c : 0)];
      }
#pragma unroll
    for (int i = 0; i < kCholRowsPerWave; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int a = w + kCholWaves * i, c = lane + 64 * h;
        if (a < l && c < l && c >= a) R.v[i][h] += gv[i][h];
      }
  }
#pragma unroll
  for (int i = 0; i < kCholRowsPerWave; ++i)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int a = w + kCholWaves * i;
      if (a < l && lane + 64 * h == a) R.v[i][h] += shift;
    }
#pragma unroll
  for (int i = 0; i < kCholRowsPerWave; ++i) {
    const int a = w + kCholWaves * i;
    if (a < l) {
    // steps j < a in chunks of published rows: the multipliers f_j of a chunk
    // (at most 64) are read at once, one per lane, and broadcast from there
    bool ge_a[2];
    int cc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      ge_a[h] = lane + 64 * h >= a;
      cc[h] = min(lane + 64 * h, l - 1);  // clamped column: loads stay in row t
    }
    int j = 0;
    while (j < a) {
      if (j >= known) {
        int spins = 0;
        while (!bail) {
          known = __builtin_amdgcn_readfirstlane(
              __hip_atomic_load(nready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
          if (known > j) break;
          if (spins > 64) __builtin_amdgcn_s_sleep(1);  // poll tightly for a while first
          if (++spins > (1 << 20)) bail = true;
        }
        if (bail) known = a;
      }
      const int jend = min(min(known, a), j + 64);
      const int jl = j + lane;
      const double fv = jl < jend ? Pub[jl * l + a] * pinv[jl] : 0.0;
      const int flo = __double2loint(fv), fhi = __double2hiint(fv);
      // published row t holds W[t][c] (c < t), 1 (c = t), S[t][c] (c > t):
      // lane c < a takes it for c <= t, lane c >= a always. Loads and FMAs
      // are unconditional with the mask on the multiplier (v - 0 p = v), and
      // the loads of four steps are issued before their FMAs.
      double v0 = R.v[i][0], v1 = R.v[i][1];
      int t = j;
      for (; t + 4 <= jend; t += 4) {
        double p0[4], p1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          p0[u] = Pub[(t + u) * l + cc[0]];
          p1[u] = Pub[(t + u) * l + cc[1]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double f = __hiloint2double(__builtin_amdgcn_readlane(fhi, t + u - j),
                                            __builtin_amdgcn_readlane(flo, t + u - j));
          v0 = fma(-((lane <= t + u || ge_a[0]) ? f : 0.0), p0[u], v0);
          v1 = fma(-((lane + 64 <= t + u || ge_a[1]) ? f : 0.0), p1[u], v1);
        }
      }
      for (; t < jend; ++t) {
        const double f = __hiloint2double(__builtin_amdgcn_readlane(fhi, t - j), __builtin_amdgcn_readlane(flo, t - j));
        v0 = fma(-((lane <= t || ge_a[0]) ? f : 0.0), Pub[t * l + cc[0]], v0);
        v1 = fma(-((lane + 64 <= t || ge_a[1]) ? f : 0.0), Pub[t * l + cc[1]], v1);
      }
      R.v[i][0] = v0;
      R.v[i][1] = v1;
      j = jend;
    }
    // row a is final: its pivot, then publish
    const double dsrc = a < 64 ? R.v[i][0] : R.v[i][1];
    const double d = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(dsrc), a % 64),
                                      __builtin_amdgcn_readlane(__double2loint(dsrc), a % 64));
    double dinv = 1.0 / d;
    if (check) {
      if (!(d > 1e-13 * d0[a]) && lane == 0) *retry = 1;
    } else if (!(d > 0.0)) {  // not positive after the shift (or NaN): drop column a
      if (lane == 0) atomicOr(&info->flags, kFlagQrBreakdown);
      dinv = 0.0;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int c = lane + 64 * h;
      if (c < l) Pub[a * l + c] = c == a ? 1.0 : R.v[i][h];
    }
    if (lane == 0) pinv[a] = dinv;
    __hip_atomic_store(nready, a + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  if (bail && lane == 0) atomicOr(&info->flags, kFlagQrBreakdown);
}

// LDS of the Cholesky body: published rows, 1/d, the diagonal of G, and two
// counters.
__host__ __device__ inline size_t chol_lds(int l) { return ((size_t)l * l + 2 * l) * 8 + 16; }

// G is given as nparts partial sums (stride pstride elements), added here in
// order; sm: LDS of chol_lds(l) bytes.
__device__ inline void chol_inv_body(const double* __restrict__ G, int nparts, int64_t pstride, int LP,
                                     int l, int64_t rows, int mode, double* __restrict__ Rinv,
                                     int* __restrict__ skip3, DevInfo* __restrict__ info, double* sm) {
  if (mode == 2 && *skip3) return;
  double* Pub = sm;             // l x l: published final rows
  double* pinv = sm + l * l;    // l: 1 / d
  double* d0 = pinv + l;        // l: diagonal of G
  int* nready = reinterpret_cast<int*>(d0 + l);
  int* retry = nready + 1;
  const int tid = threadIdx.x;
  for (int i = tid; i < l; i += kSmallThreads) d0[i] = chol_gval(G, nparts, pstride, LP, i, i);
  if (tid == 0) { *nready = 0; *retry = 0; }
  __syncthreads();
  CholRows R;
  ldl_flow(G, nparts, pstride, LP, l, 0.0, d0, true, Pub, pinv, nready, retry, info, R);
  __syncthreads();
  bool shifted = false;
  if (*retry) {
    double tr = 0.0;
    for (int i = 0; i < l; ++i) tr += d0[i];
    const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 0x1p-53 * tr;
    __syncthreads();
    if (tid == 0) *nready = 0;
    __syncthreads();
    ldl_flow(G, nparts, pstride, LP, l, shift, d0, false, Pub, pinv, nready, retry, info, R);
    shifted = true;
  }
  if (tid == 0) {
    if (shifted) *skip3 = 0;
    else if (mode == 0) *skip3 = 1;
  }
  // R^{-1}[r][c] = W[c][r] / sqrt(d_c) for r < c, 1 / sqrt(d_c) on the diagonal;
  // a dropped column (d_c not positive) is zero. Zeros first, then each wave
  // writes the columns of its rows.
  for (int i = tid; i < LP * LP; i += kSmallThreads) Rinv[i] = 0.0;
  __syncthreads();
  const int w = tid / 64, lane = tid % 64;
#pragma unroll
  for (int i = 0; i < kCholRowsPerWave; ++i) {
    const int c = w + kCholWaves * i;  // row c of the factor = column c of R^{-1}
    if (c >= l) continue;
    const double dc = __shfl(c < 64 ? R.v[i][0] : R.v[i][1], c % 64, kWave);
    const double isd = dc > 0.0 ? 1.0 / sqrt(dc) : 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = lane + 64 * h;
      if (r < c) Rinv[r * LP + c] = R.v[i][h] * isd;
      else if (r == c) Rinv[r * LP + c] = isd;
    }
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
// stop when no pair had |gamma| > tol sqrt(alpha beta), or after max_sweeps.
// Then sigma_j = |m_j|, U~_j = m_j / sigma_j, V~_j = v_j, sorted descending;
// the first k are written (Ut, and Vt if WANT_V: l x k, ld ldk; s: k).
//
// One workgroup of kJacThreads. Each pair is handled by a group of 8 lanes;
// lane g of a group holds rows g, g + 8, ... of the two columns in registers
// for the step (NRB of them, a compile-time row-block count), and the three
// dot products are reduced with DPP. The step cost is VALU issue on one CU,
// so the layout avoids per-row masks: M lives in LDS column-major with its
// columns padded with zero rows to ldm = 8 NRB (rotations keep them zero).
// V, when wanted, lives in LDS when it fits: column stride ldm, or, where
// only the unpadded form fits, stride l followed by one dummy word that takes
// the rows past l of the last row block; else in the global scratch `Vg`
// (at least l x ldm, stride ldm). V is not needed for singular values alone
// (WANT_V = false).
constexpr int kJacThreads = 512;

// Row blocks per lane for a given l (a few sizes, to bound the number of
// compiled variants): M's padded column length is 8 jac_nrb(l).
__host__ __device__ constexpr int jac_nrb(int l) {
  return l <= 8 ? 1 : l <= 16 ? 2 : l <= 32 ? 4 : l <= 48 ? 6 : l <= 64 ? 8 : l <= 80 ? 10 : l <= 104 ? 13 : 16;
}
__host__ __device__ constexpr int jac_ldm(int l) { return 8 * jac_nrb(l); }
// Column stride of the global scratch Vg (LP x this): holds V with padded
// columns, or the singular values.
__host__ __device__ constexpr int jac_vg_ld(int l) { return jac_ldm(l) > ((l + 15) & ~15) ? jac_ldm(l) : ((l + 15) & ~15); }
constexpr size_t kJacLdsLimit = 160 * 1024 - 256;  // room for the static LDS words
// V in LDS with padded columns / with unpadded columns (+ the dummy word).
__host__ __device__ inline bool jac_vpad_fits(int l) {
  return (size_t)l * jac_ldm(l) * 16 <= kJacLdsLimit;
}
__host__ __device__ inline bool jac_vtail_fits(int l) {
  return ((size_t)l * jac_ldm(l) + (size_t)l * l + 1) * 8 <= kJacLdsLimit;
}
// Dynamic LDS of the Jacobi body and whether V is in it.
__host__ __device__ inline size_t jacobi_lds(int l, bool want_v, bool* v_lds) {
  const size_t mbytes = (size_t)l * jac_ldm(l) * 8;
  *v_lds = want_v && (jac_vpad_fits(l) || jac_vtail_fits(l));
  if (!*v_lds) return mbytes + (size_t)l * 8;  // M and the singular values
  return jac_vpad_fits(l) ? 2 * mbytes : mbytes + ((size_t)l * l + 1) * 8;
}

// (c, s) of the pair rotation above for gamma != 0, with t in one division:
// multiplying the numerator and the denominator of t by 2 |gamma| gives
// t = sign(zeta) 2 |gamma| / (|d| + sqrt(d^2 + 4 gamma^2)), d = beta - alpha,
// evaluated on d and 2 gamma scaled by the same power of two (the squares can
// neither overflow nor underflow, and t does not change); sign(zeta) = +1
// for d = 0. c = rsqrt(1 + t^2) with 1 + t^2 in [1, 2].
__device__ inline void jac_rotation(double al, double be, double ga, double& c, double& s) {
  const double d = be - al, g2 = 2.0 * ga;
  const int e = ilogb(fmax(fabs(d), fabs(g2)));
  const double ds = ldexp(d, -e), gs = ldexp(g2, -e);
  const double t0 = fabs(gs) / (fabs(ds) + sqrt(fma(ds, ds, gs * gs)));
  const double t = (d == 0.0 || (d > 0.0) == (ga > 0.0)) ? t0 : -t0;
  c = rsqrt(fma(t, t, 1.0));
  s = c * t;
}

// Min is given as nparts partial sums (stride pstride elements), added in
// order. tol2 = tol^2 (the main path takes tol = sqrt(l) 2^-52).
//
// rlog != null (with WANT_V false): V is not kept here. Instead the (c, s)
// of every pair of every step is written to rlog (double2, (1, 0) where the
// pair was not rotated; entry (sweep (lp - 1) + step) npairs + pr), and the
// column of rank j < k to vperm[j]: every row of V receives the same
// sequence of column rotations, so k_jacobi_vapply rebuilds V afterwards, one
// row per wave and many rows at once, instead of moving V through this one
// CU's LDS at every step (which doubles its LDS traffic). rlog holds
// max_sweeps (lp - 1) npairs entries.
template <bool V_LDS, bool WANT_V, int NRB>
__device__ inline void jacobi_body(const double* __restrict__ Min, int nparts, int64_t pstride, int LP,
                                   int l, int k, int max_sweeps, double tol2, double* __restrict__ Ut,
                                   double* __restrict__ sv, double* __restrict__ Vt, int ldk,
                                   double* __restrict__ Vg, DevInfo* __restrict__ info, double* sm,
                                   double2* __restrict__ rlog = nullptr, int* __restrict__ vperm = nullptr) {
  static_assert(WANT_V || !V_LDS, "V in LDS only when wanted");
  constexpr int ldm = 8 * NRB;
  const bool vtail = V_LDS && !jac_vpad_fits(l);  // V columns unpadded (stride l)
  double* Mc = sm;                              // column-major: Mc[c * ldm + r]
  double* Vc = V_LDS ? sm + (size_t)l * ldm : Vg;
  const int vld = vtail ? l : ldm;              // column stride of V
  const int vdummy = l * vld;                   // (vtail) the dummy word
  // singular values: after M (and V) in LDS, or in the unused global scratch
  double* sig = V_LDS ? Vg : sm + (size_t)l * ldm;
  __shared__ int s_rot;
  const int tid = threadIdx.x;
  const int grp = tid / 8, gl = tid % 8;
  constexpr int ngroups = kJacThreads / 8;

  // M (row-major, ld LP, as nparts partial sums added in order) into LDS
  // column-major with rows l .. ldm - 1 zero: read row-major (a wave reads
  // consecutive columns), kMLoad entries per thread in flight at a time
  {
    constexpr int kMLoad = 8;
    const int tot = ldm * l;
    for (int i0 = 0; i0 < tot; i0 += kJacThreads * kMLoad) {
      double mv[kMLoad];
#pragma unroll
      for (int u = 0; u < kMLoad; ++u) mv[u] = 0.0;
      for (int p = 0; p < nparts; ++p) {
        double t[kMLoad];
#pragma unroll
        for (int u = 0; u < kMLoad; ++u) {
          const int i = i0 + tid + kJacThreads * u;
          const int r = i / l, c = i % l;
          t[u] = Min[p * pstride + ((i < tot && r < l) ? r * LP + c : 0)];
        }
#pragma unroll
        for (int u = 0; u < kMLoad; ++u) {
          const int i = i0 + tid + kJacThreads * u;
          if (i < tot && i / l < l) mv[u] += t[u];
        }
      }
#pragma unroll
      for (int u = 0; u < kMLoad; ++u) {
        const int i = i0 + tid + kJacThreads * u;
        if (i < tot) Mc[(i % l) * ldm + i / l] = mv[u];
      }
    }
  }
  if (WANT_V)
    for (int i = tid; i < l * vld; i += kJacThreads) {
      const int c = i / vld, r = i % vld;
      Vc[i] = (r == c) ? 1.0 : 0.0;
    }
  __syncthreads();

  const int lp = (l + 1) & ~1;
  const int npairs = lp / 2;
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
        double2* lg = (!WANT_V && rlog && gl == 0)
                          ? rlog + ((size_t)sweep * (lp - 1) + step) * npairs + pr : nullptr;
        int p = player(pr), q = player(lp - 1 - pr);
        if (p >= l || q >= l) {
          if (lg) *lg = double2{1.0, 0.0};
          continue;
        }
        if (p > q) { int t = p; p = q; q = t; }
        double* mp = Mc + p * ldm + gl;
        double* mq = Mc + q * ldm + gl;
        double x[NRB], y[NRB];
#pragma unroll
        for (int i = 0; i < NRB; ++i) { x[i] = mp[8 * i]; y[i] = mq[8 * i]; }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int i = 0; i < NRB; ++i) { al += x[i] * x[i]; be += y[i] * y[i]; ga += x[i] * y[i]; }
        al = sum8(al); be = sum8(be); ga = sum8(ga);
        if (!(ga * ga > tol2 * (al * be))) {  // orthogonal enough (or zero column)
          if (lg) *lg = double2{1.0, 0.0};
          continue;
        }
        // V: the row blocks before the last one are whole; in the last one
        // (registers vxl, vyl) rows past l go to the dummy word when V's
        // columns are not padded
        double vx[NRB], vy[NRB], vxl = 0.0, vyl = 0.0;
        int ipl = 0, iql = 0;
        if (WANT_V) {
          // read before the rotation is formed, so that the latency overlaps
          // the division and square roots
#pragma unroll
          for (int i = 0; i < NRB - 1; ++i) {
            vx[i] = Vc[p * vld + gl + 8 * i];
            vy[i] = Vc[q * vld + gl + 8 * i];
          }
          const int rl = gl + 8 * (NRB - 1);
          const bool okl = !vtail || rl < l;
          ipl = okl ? p * vld + rl : vdummy;
          iql = okl ? q * vld + rl : vdummy;
          vxl = Vc[ipl];
          vyl = Vc[iql];
        }
        double c, s;
        jac_rotation(al, be, ga, c, s);
        if (lg) *lg = double2{c, s};
#pragma unroll
        for (int i = 0; i < NRB; ++i) {
          mp[8 * i] = c * x[i] - s * y[i];
          mq[8 * i] = s * x[i] + c * y[i];
        }
        if (WANT_V) {
#pragma unroll
          for (int i = 0; i < NRB - 1; ++i) {
            Vc[p * vld + gl + 8 * i] = c * vx[i] - s * vy[i];
            Vc[q * vld + gl + 8 * i] = s * vx[i] + c * vy[i];
          }
          Vc[ipl] = c * vxl - s * vyl;
          Vc[iql] = s * vxl + c * vyl;
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
    for (int r = gl; r < l; r += 8) a += Mc[c * ldm + r] * Mc[c * ldm + r];
    a = sum8(a);
    if (gl == 0) sig[c] = sqrt(a);
  }
  __syncthreads();
  // rank of each column in descending order (ties: lower index first)
  for (int c = grp; c < l; c += ngroups) {
    const double sc = sig[c];
    int rank = 0;
    for (int i = gl; i < l; i += 8) rank += (sig[i] > sc || (sig[i] == sc && i < c)) ? 1 : 0;
    for (int off = 4; off >= 1; off >>= 1) rank += __shfl_xor(rank, off, kWave);
    if (rank < k) {
      const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
      for (int r = gl; r < l; r += 8) {
        Ut[r * ldk + rank] = Mc[c * ldm + r] * inv;
        if (WANT_V) Vt[r * ldk + rank] = Vc[c * vld + r];
      }
      if (gl == 0) sv[rank] = sc;
      if (!WANT_V && vperm && gl == 0) vperm[rank] = c;
    }
  }
}

}  // namespace sor
