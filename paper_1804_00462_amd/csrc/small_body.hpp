// Device bodies of the small dense FP64 steps of the SOR-SVD path, each run
// by one workgroup of kSmallThreads threads (shared by the single-problem
// kernels and the batched kernels, which run one workgroup per problem):
//   * Cholesky factor and inverse of the l x l Gram matrix (the QR step of
//     Alg. 3 / Alg. 4 as Cholesky QR: T = Q R with R^T R = T^T T),
//   * the core SVD of M = Q1^T A Q2 by one-sided (Hestenes) Jacobi rotations
//     in a pair order of levels with stationary columns (rank-k truncation
//     of Alg. 3 step 6).
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
// carrying W = L^{-1} (unit lower triangular): step j subtracts
// f_a = S[j][a] / S[j][j] times row j from every row a > j, on the trailing
// upper part (columns >= a) and on W's columns 0..j. Row a holds W[a][c] for
// c < a and S[a][c] for c >= a (the pivots d_a on the diagonal). Then
// R = D^{1/2} L^T and R^{-1} = L^{-T} D^{-1/2} = W^T D^{-1/2}.
//
// Blocked in panels of 16 rows over X, the matrix padded to lp = 16
// ceil(l / 16) with the identity (its pivots are 1 and it meets no other
// row). Per panel J = [j0, j0 + 16), with M[j][a] = S[j][a] / d_j taken from
// the final row j (the trailing matrix is symmetric, so the multiplier of
// row a at step j is row j's entry at column a):
//   1. wave 0 runs the 16 steps on the 16 x 16 diagonal block (each lane
//      holds a 2 x 2 tile of it; the pivot is read from its lane, the
//      multipliers and the row subtracted come by lane shuffles; no
//      barrier);
//   2. every other column c of the panel rows receives the same steps: they
//      act on the rows J as left multiplication by L11^{-1}, which is the
//      W part of the diagonal block after step 1 (row j's entry at c is S
//      for c >= j0 + 16 and W for c < j0), so X[J][c] <- W11 X[J][c] on
//      FP64 MFMA;
//   3. the rows below the panel receive all 16 steps at once on FP64 MFMA:
//      X[a][c] -= sum_j M[j][a] Y[j][c] over 16 x 16 tiles, where Y[j] is
//      row j with its W part taken as W[j][c] (c < j), 1 (c = j), 0 (j < c
//      < j0 + 16); only the S part (c >= a) and the W part (c < j0 + 16) of
//      a row are written (its entries j0 + 16 <= c < a are W entries of
//      later panels, still zero).
// The pivots are checked against 1e-13 of G's diagonal after the factor
// (check), or a pivot that is not positive is dropped at its step (after
// the shift).
constexpr int kCholP = 16;  // panel height
__host__ __device__ inline int chol_lp(int l) { return (l + kCholP - 1) & ~(kCholP - 1); }
__host__ __device__ inline int chol_ldx(int l) { return chol_lp(l) + 8; }  // LDS row stride (bank spread)

// X (lp x ldx), dinv (lp), d0 (lp: G's diagonal, 1 on the padding; written
// here when fill_d0), *retry zero on entry.
constexpr int kCholLoad = 8;  // entries of X per thread and batch of loads
__device__ __forceinline__ void ldl_blocked(const double* __restrict__ G, int nparts, int64_t pstride, int LP,
                                            int l, double shift, double* __restrict__ d0, bool fill_d0, bool check,
                                            double* X, double* dinv, int* retry, DevInfo* info) {
  const int lp = chol_lp(l), ldx = chol_ldx(l), nt = lp / kCholP;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  // X: G's upper part (+ shift), zero below, the identity on the padding; the
  // parts are added in order, the loads of a batch of kCholLoad entries per
  // thread issued before any is used (entries outside the upper part read a
  // valid address and are dropped)
  for (int e0 = 0; e0 < lp * lp; e0 += kSmallThreads * kCholLoad) {
    double v[kCholLoad];
    int off[kCholLoad];
#pragma unroll
    for (int i = 0; i < kCholLoad; ++i) {
      const int e = e0 + tid + kSmallThreads * i, a = e / lp, c = e % lp;
      const bool in = e < lp * lp && a < l && c < l && c >= a;
      off[i] = in ? a * LP + c : 0;
      v[i] = G[off[i]];
    }
    for (int p = 1; p < nparts; ++p)
#pragma unroll
      for (int i = 0; i < kCholLoad; ++i) v[i] += G[p * pstride + off[i]];
#pragma unroll
    for (int i = 0; i < kCholLoad; ++i) {
      const int e = e0 + tid + kSmallThreads * i, a = e / lp, c = e % lp;
      if (e < lp * lp) {
        const bool in = a < l && c < l && c >= a;
        if (fill_d0 && a == c) d0[a] = in ? v[i] : 1.0;
        X[a * ldx + c] = in ? v[i] + (a == c ? shift : 0.0) : (a == c ? 1.0 : 0.0);
      }
    }
  }
  __syncthreads();
  for (int k = 0; k < nt; ++k) {
    const int j0 = kCholP * k, j1 = j0 + kCholP;
    // 1. the diagonal block, wave 0: lane (r2, c2) = (lane / 8, lane % 8)
    // holds rows j0 + 2 r2 + {0, 1}, columns j0 + 2 c2 + {0, 1}
    if (w == 0) {
      const int r2 = lane / 8, c2 = lane % 8;
      double x[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) x[a][b] = X[(j0 + 2 * r2 + a) * ldx + j0 + 2 * c2 + b];
      double mydi = 0.0;  // lane j: 1 / d of step j
#pragma unroll
      for (int j = 0; j < kCholP; ++j) {
        const int jr = j / 2, jb = j % 2;
        const double d = readlane_f64(x[jb][jb], 8 * jr + jr);
        // 1 / d: the hardware estimate and two Newton steps (a pivot that is
        // not positive is checked after the factor, or dropped here)
        double di = __builtin_amdgcn_rcp(d);
        di = fma(di, fma(-d, di, 1.0), di);
        di = fma(di, fma(-d, di, 1.0), di);
        if (!check && !(d > 0.0)) {  // not positive after the shift (or NaN): drop column j0 + j
          if (lane == 0) atomicOr(&info->flags, kFlagQrBreakdown);
          di = 0.0;
        }
        if (lane == j) mydi = di;
        // row j at my rows' columns (the multipliers: S[j][i] = S[i][j]) and
        // at my columns (the row subtracted)
        double f[2], rj[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          f[a] = __shfl(x[jb][a], 8 * jr + r2, kWave) * di;
          rj[a] = __shfl(x[jb][a], 8 * jr + c2, kWave);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const int i = 2 * r2 + a;
          if (i > j) {
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              const int c = 2 * c2 + b;
              const double y = (c >= i || c < j) ? rj[b] : (c == j ? 1.0 : 0.0);
              x[a][b] = fma(-f[a], y, x[a][b]);
            }
          }
        }
      }
      if (lane < kCholP) dinv[j0 + lane] = mydi;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) X[(j0 + 2 * r2 + a) * ldx + j0 + 2 * c2 + b] = x[a][b];
    }
    __syncthreads();
    const int li = lane % 16, g = lane / 16;
    // 2. the other columns of the panel rows receive the panel's steps: the
    // steps on rows J are left multiplication by W11 = L11^{-1}, the W part
    // of the diagonal block (unit diagonal), so X[J][c] <- W11 X[J][c], one
    // 16-column tile per wave on FP64 MFMA
    for (int it = w; it < nt - 1; it += kSmallThreads / kWave) {
      const int c0 = kCholP * (it < k ? it : it + 1);
      double bv[4], av[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * s + g;
        bv[s] = X[(j0 + kk) * ldx + c0 + li];
        av[s] = li > kk ? X[(j0 + li) * ldx + j0 + kk] : (li == kk ? 1.0 : 0.0);  // W11[li][kk]
      }
      f64x4 acc = f64x4{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
#pragma unroll
      for (int r4 = 0; r4 < 4; ++r4) X[(j0 + 4 * r4 + g) * ldx + c0 + li] = acc[r4];
    }
    __syncthreads();
    if (k == nt - 1) break;
    // 3. the rows below the panel: tiles (ta, tc), ta > k, tc <= k (W part)
    // or tc >= ta (S part), dealt round-robin to the waves; a tile's loads
    // are all issued before its products
    {
      int ntile = 0;
      for (int ta = k + 1; ta < nt; ++ta) ntile += (k + 1) + (nt - ta);
      for (int it = w; it < ntile; it += kSmallThreads / kWave) {
        int ta = k + 1, rem = it;
        for (;;) {
          const int n = (k + 1) + (nt - ta);
          if (rem < n) break;
          rem -= n;
          ++ta;
        }
        const int tc = rem <= k ? rem : ta + (rem - (k + 1));
        const int a0 = kCholP * ta, c0 = kCholP * tc, c = c0 + li;
        f64x4 acc;
        double am[4], bm[4];
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) acc[r4] = X[(a0 + 4 * r4 + g) * ldx + c];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int j = j0 + 4 * s + g;
          am[s] = -X[j * ldx + a0 + li] * dinv[j];  // -M[j][a0 + li]
          const double xb = X[j * ldx + c];
          bm[s] = (tc < k || c < j || c >= j1) ? xb : (c == j ? 1.0 : 0.0);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(am[s], bm[s], acc, 0, 0, 0);
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          const int a = a0 + 4 * r4 + g;
          if (c < j1 || c >= a) X[a * ldx + c] = acc[r4];
        }
      }
    }
    __syncthreads();
  }
  // the unshifted factor: every pivot (the final diagonal) against 1e-13 of
  // G's diagonal
  if (check)
    for (int j = tid; j < l; j += kSmallThreads)
      if (!(X[j * ldx + j] > 1e-13 * d0[j])) *retry = 1;
  __syncthreads();
}

// LDS of the Cholesky body: X, 1/d, the diagonal of G and the retry word.
__host__ __device__ inline size_t chol_lds(int l) {
  const size_t lp = chol_lp(l);
  return (lp * chol_ldx(l) + 2 * lp) * 8 + 16;
}

// G is given as nparts partial sums (stride pstride elements), added here in
// order; sm: LDS of chol_lds(l) bytes.
__device__ inline void chol_inv_body(const double* __restrict__ G, int nparts, int64_t pstride, int LP,
                                     int l, int64_t rows, int mode, double* __restrict__ Rinv,
                                     int* __restrict__ skip3, DevInfo* __restrict__ info, double* sm) {
  if (mode == 2 && *skip3) return;
  const int lp = chol_lp(l), ldx = chol_ldx(l);
  double* X = sm;                        // lp x ldx
  double* dinv = X + (size_t)lp * ldx;   // lp: 1 / d (0: dropped)
  double* d0 = dinv + lp;                // lp: diagonal of G
  int* retry = reinterpret_cast<int*>(d0 + lp);
  const int tid = threadIdx.x;
  if (tid == 0) *retry = 0;
  __syncthreads();
  ldl_blocked(G, nparts, pstride, LP, l, 0.0, d0, true, true, X, dinv, retry, info);
  bool shifted = false;
  if (*retry) {
    double tr = 0.0;
    for (int i = 0; i < l; ++i) tr += d0[i];
    const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 0x1p-53 * tr;
    __syncthreads();
    ldl_blocked(G, nparts, pstride, LP, l, shift, d0, false, false, X, dinv, retry, info);
    shifted = true;
  }
  if (tid == 0) {
    if (shifted) *skip3 = 0;
    else if (mode == 0) *skip3 = 1;
  }
  // R^{-1}[r][c] = W[c][r] / sqrt(d_c) for r < c, 1 / sqrt(d_c) on the
  // diagonal, zero below and outside l; a dropped column (d_c not positive)
  // is zero. 1 / sqrt(d_c) first (into dinv, no longer needed).
  for (int c = tid; c < lp; c += kSmallThreads) {
    const double dc = X[c * ldx + c];
    dinv[c] = dc > 0.0 ? 1.0 / sqrt(dc) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < LP * LP; e += kSmallThreads) {
    const int r = e / LP, c = e % LP;
    double v = 0.0;
    if (r <= c && c < l) v = r == c ? dinv[c] : X[c * ldx + r] * dinv[c];
    Rinv[e] = v;
  }
}


// ---------------------------------------------------------------------------
// One-sided Jacobi SVD of an l x l matrix M (ld LP), FP64, l <= 128.
// Columns are rotated in pairs (p, q): with alpha = |m_p|^2, beta = |m_q|^2,
// gamma = m_p . m_q, zeta = (beta - alpha) / (2 gamma),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t,
// m_p <- c m_p - s m_q, m_q <- s m_p + c m_q (and the same on V), which makes
// the pair orthogonal. A sweep visits every pair once, in steps of disjoint
// pairs (the order of jac_slot below); sweeps
// stop when no pair had |gamma| > tol sqrt(alpha beta), or after max_sweeps.
// Then sigma_j = |m_j|, U~_j = m_j / sigma_j, V~_j = v_j, sorted descending;
// the first k are written (Ut, and Vt if WANT_V: l x k, ld ldk; s: k).
//
// One workgroup of kJacThreads. Each pair is handled by a group of GL lanes
// (16 for widths 33 .. 64, else 8: the pairs of a step then fill two waves
// per SIMD, which hide each other's latency; at widths above 64 groups of 8
// already do, and groups of 4 (one wave per SIMD) are slower); lane g of a
// group holds rows g, g + GL, ... of its columns in registers (8 NRB / GL of
// them, NRB a compile-time row-block count), and the dot products are
// reduced with DPP. A group keeps its stationary column (and that column of
// V) in registers for a whole level of the order and reads and writes only
// the moving column at each step: one column through LDS per pair and step
// instead of two (LDS traffic, not arithmetic, sets the step time). When V is not in LDS, alpha and beta are
// not formed at every step: the squared column norms are computed at the
// start of each sweep and carried through it by the exact update of a
// rotation (alpha - t gamma, beta + t gamma), recomputed from the rotated
// column where that update cancels (the scheme of Drmac and Veselic's
// one-sided Jacobi SVD), which leaves one dot product per pair and step.
// The step cost is VALU issue on one
// CU, so the layout avoids per-row masks: M lives in LDS column-major with its
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
// Lane groups of the Jacobi workgroup (one pair slot each): 8 lanes per
// group, 16 for the row-block counts 6 and 8.
__host__ __device__ constexpr int jac_groups(int l) {
  return kJacThreads / ((jac_nrb(l) == 6 || jac_nrb(l) == 8) ? 16 : 8);
}
// Column stride of M in LDS when V is not there: with groups of 8 lanes
// (every row-block count but 6 and 8) ldm rounded up to 16 doubles, so that
// column starts fall on bank 0 (see jacobi_body); else ldm.
__host__ __device__ constexpr int jac_mstride(int l) {
  return (jac_nrb(l) == 6 || jac_nrb(l) == 8) ? jac_ldm(l) : ((jac_ldm(l) + 15) & ~15);
}
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
  if (!*v_lds) return (size_t)l * jac_mstride(l) * 8 + (size_t)l * 8;  // M and the singular values
  return jac_vpad_fits(l) ? 2 * mbytes : mbytes + ((size_t)l * l + 1) * 8;
}

// Pair order of a sweep, shared by the Jacobi kernel and the V replay. Level
// d (for 2^d < l) cuts the columns into the 2^(d+1) ranges
// J(d + 1, i) = [ceil(i l / 2^(d+1)), ceil((i + 1) l / 2^(d+1))); in block
// b < 2^d every column of range 2b (stationary) meets every column of range
// 2b + 1 (moving): slot g of the block keeps stationary column g for the
// whole level and meets moving column (g + j) mod R at step j, R the larger
// range size, so that the moving columns pass from slot g + 1 to slot g
// between steps. The level takes H = ceil(l / 2^(d+1)) steps (the largest R),
// block b owns slots b H .. b H + R - 1 (2^d H <= 64 for l <= 128, <= 32
// for l <= 64). Two columns meet at the first level that puts them in
// different ranges, so a sweep meets every pair once: sum_d H steps, 127 at
// l = 128, 102 at l = 100 (round-robin takes l - 1 or l), each with at most
// one pair per slot.
struct JacSlot {
  int p;   // stationary column (valid when g < a)
  int s1;  // first moving column
  int a;   // stationary columns of the block
  int m;   // moving columns of the block
  int R;   // ring length max(a, m) (0: slot outside every block)
  int g;   // position in the block
};
__host__ __device__ inline int jac_levels(int l) {
  int d = 0;
  while ((1 << d) < l) ++d;
  return d;
}
__host__ __device__ inline int jac_level_steps(int l, int d) { return (l + (2 << d) - 1) >> (d + 1); }
__host__ __device__ inline int jac_sweep_steps(int l) {
  int n = 0;
  for (int d = 0; (1 << d) < l; ++d) n += jac_level_steps(l, d);
  return n;
}
__host__ __device__ inline JacSlot jac_slot(int l, int d, int H, int slot) {
  JacSlot r;
  const int b = slot / H;
  r.g = slot - b * H;
  if (b >= (1 << d)) {
    r.p = r.s1 = r.a = r.m = r.R = 0;
    return r;
  }
  const int sh = d + 1, rnd = (1 << sh) - 1;
  const int s0 = (2 * b * l + rnd) >> sh, s1 = ((2 * b + 1) * l + rnd) >> sh, e1 = ((2 * b + 2) * l + rnd) >> sh;
  r.a = s1 - s0;
  r.m = e1 - s1;
  r.R = r.a > r.m ? r.a : r.m;
  r.p = s0 + r.g;
  r.s1 = s1;
  return r;
}

// (c, s) of the pair rotation above for gamma != 0. Multiplying the
// numerator and the denominator of t by 2 |gamma| gives
// t = sign(zeta) 2 |gamma| / (|d| + sqrt(d^2 + 4 gamma^2)), d = beta - alpha,
// evaluated on d and 2 gamma scaled by the same power of two into [1, 2) for
// the larger (the squares can neither overflow nor underflow, and t does not
// change); sign(zeta) = +1 for d = 0. With the arguments in fixed ranges,
// the square root (of [1, 8)), the reciprocal (of [1, 5)) and
// c = 1 / sqrt(1 + t^2) (of [1, 2]) take the hardware estimates and Newton
// steps (a short dependency chain: the rotation sits on the critical path of
// every Jacobi step); from estimates within 2^-14 the steps reach full
// precision. Then (c, s) take one Newton step to unit length.
__device__ inline void jac_rotation(double al, double be, double ga, double& c, double& s, double& t) {
  const double d = be - al, g2 = 2.0 * ga;
  const int e = ilogb(fmax(fabs(d), fabs(g2)));
  const double ds = ldexp(d, -e), gs = fabs(ldexp(g2, -e));
  const double r2 = fma(ds, ds, gs * gs);  // [1, 8)
  // sqrt(r2): g ~ sqrt, h ~ 1 / (2 sqrt), one coupled step, then a Newton
  // step on g
  const double y0 = __builtin_amdgcn_rsq(r2);
  double g = r2 * y0, h = 0.5 * y0;
  const double rr = fma(-h, g, 0.5);
  g = fma(g, rr, g);
  h = fma(h, rr, h);
  g = fma(fma(-g, g, r2), h, g);
  // t0 = gs / den, den = |ds| + sqrt(r2) in [1, 5)
  const double den = fabs(ds) + g;
  double q = __builtin_amdgcn_rcp(den);
  q = fma(q, fma(-den, q, 1.0), q);
  q = fma(q, fma(-den, q, 1.0), q);
  double t0 = gs * q;
  t0 = fma(fma(-den, t0, gs), q, t0);
  t = (d == 0.0 || (d > 0.0) == (ga > 0.0)) ? t0 : -t0;
  // c = 1 / sqrt(u), u = 1 + t^2 in [1, 2]: two Newton steps
  const double u = fma(t, t, 1.0);
  double cy = __builtin_amdgcn_rsq(u);
  cy = fma(0.5 * cy, fma(-u * cy, cy, 1.0), cy);
  cy = fma(0.5 * cy, fma(-u * cy, cy, 1.0), cy);
  c = cy;
  s = c * t;
  // one Newton step towards c^2 + s^2 = 1 (eu = c^2 + s^2 - 1 with one
  // rounding of c^2 - 1): a rounding of the same sign in every rotation
  // would otherwise grow the columns' norms
  const double eu = fma(s, s, fma(c, c, -1.0));
  const double f = fma(-0.5, eu, 1.0);
  c *= f;
  s *= f;
}
__device__ inline void jac_rotation(double al, double be, double ga, double& c, double& s) {
  double t;
  jac_rotation(al, be, ga, c, s, t);
}

// Below this ratio of a carried squared column norm to its value before the
// rotation, the norm is recomputed from the rotated column (the update
// subtracts nearly equal numbers there).
constexpr double kJacNormKeep = 0.1;

// Min is given as nparts partial sums (stride pstride elements), added in
// order. tol2 = tol^2 (the main path takes tol = sqrt(l) 2^-52).
//
// rlog != null (with WANT_V false): V is not kept here. Instead the (c, s)
// of every pair of every step is written to rlog (double2, (1, 0) where the
// slot had no pair or did not rotate it; entry (sweep S + step) G + slot,
// S = jac_sweep_steps(l), G = jac_groups(l)), and the
// column of rank j < k to vperm[j]: every row of V receives the same
// sequence of column rotations, so k_jacobi_vapply rebuilds V afterwards, one
// row per wave and many rows at once, instead of moving V through this one
// CU's LDS at every step (which doubles its LDS traffic). rlog holds
// max_sweeps S G entries.
template <bool V_LDS, bool WANT_V, int NRB>
__device__ inline void jacobi_body(const double* __restrict__ Min, int nparts, int64_t pstride, int LP,
                                   int l, int k, int max_sweeps, double tol2, double* __restrict__ Ut,
                                   double* __restrict__ sv, double* __restrict__ Vt, int ldk,
                                   double* __restrict__ Vg, DevInfo* __restrict__ info, double* sm,
                                   double2* __restrict__ rlog = nullptr, int* __restrict__ vperm = nullptr) {
  static_assert(WANT_V || !V_LDS, "V in LDS only when wanted");
  constexpr int ldm = 8 * NRB;
  constexpr int GL = (NRB == 6 || NRB == 8) ? 16 : 8;  // lanes per pair
  constexpr int RPL = ldm / GL;                         // rows per lane
  // Column stride of M: ldm, or with V out of LDS and groups of 8 lanes,
  // ldm rounded up to 16 doubles (jac_mstride): every column then starts on
  // bank 0, and the odd group of each 16-lane half-row takes its row blocks
  // one block later (register i holds row block i + 1, the last one block
  // 0), so the two groups that one LDS cycle serves always use the two
  // opposite 16-bank halves, whatever their columns are
  constexpr bool SWZ = !V_LDS && GL == 8;
  constexpr int cst = SWZ ? ((ldm + 15) & ~15) : ldm;
  const bool vtail = V_LDS && !jac_vpad_fits(l);  // V columns unpadded (stride l)
  double* Mc = sm;                              // column-major: Mc[c * cst + r]
  double* Vc = V_LDS ? sm + (size_t)l * ldm : Vg;
  const int vld = vtail ? l : ldm;              // column stride of V
  const int vdummy = l * vld;                   // (vtail) the dummy word
  // singular values: after M (and V) in LDS, or in the unused global scratch
  double* sig = V_LDS ? Vg : sm + (size_t)l * cst;
  // Squared column norms carried through a sweep when V is not in LDS (in
  // the singular values' LDS words, which are written only after the sweeps)
  constexpr bool CARRY = !V_LDS;
  double* nrm = sig;
  __shared__ int s_rot;
  const int tid = threadIdx.x;
  const int grp = tid / GL, gl = tid % GL;
  constexpr int ngroups = kJacThreads / GL;

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
        if (i < tot) Mc[(i % l) * cst + i / l] = mv[u];
      }
    }
  }
  if (WANT_V)
    for (int i = tid; i < l * vld; i += kJacThreads) {
      const int c = i / vld, r = i % vld;
      Vc[i] = (r == c) ? 1.0 : 0.0;
    }
  __syncthreads();

  const int nlev = jac_levels(l);
  const int nst = jac_sweep_steps(l);
  // offset of register i's row block (rotated by one block in odd groups)
  const int odd = SWZ ? (grp & 1) : 0;
  auto roff = [&](int i) { return i + odd < RPL ? GL * (i + odd) : 0; };
  auto gsum = [](double v) { return GL == 16 ? sum16(v) : sum8(v); };
  // V: the row blocks before the last one are whole; in the last one (row
  // rl of this lane) rows past l go to the dummy word when V's columns are
  // not padded
  const int rl = gl + GL * (RPL - 1);
  const bool okl = !vtail || rl < l;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    if constexpr (CARRY) {
      // exact squared norms at the start of every sweep (groups of 8 lanes)
      const int g8 = tid / 8, l8 = tid % 8;
      for (int c = g8; c < l; c += kJacThreads / 8) {
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < NRB; ++i) a += Mc[c * cst + l8 + 8 * i] * Mc[c * cst + l8 + 8 * i];
        a = sum8(a);
        if (l8 == 0) nrm[c] = a;
      }
    }
    __syncthreads();
    int tstep = 0;  // step within the sweep
    for (int d = 0; d < nlev; ++d) {
      const int H = jac_level_steps(l, d);
      const JacSlot sl = jac_slot(l, d, H, grp);
      const bool has_p = sl.g < sl.a;
      const int p = has_p ? sl.p : 0;
      double* mp = Mc + p * cst + gl;
      // the stationary column (and its squared norm, and its column of V)
      double x[RPL], vx[RPL], al = 0.0;
      const int ipl = okl ? p * vld + rl : vdummy;
      if (has_p) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) x[i] = mp[roff(i)];
        if constexpr (CARRY) al = nrm[p];
        if (WANT_V) {
#pragma unroll
          for (int i = 0; i < RPL - 1; ++i) vx[i] = Vc[p * vld + gl + GL * i];
          vx[RPL - 1] = Vc[ipl];
        }
      }
      for (int j = 0; j < H; ++j, ++tstep) {
        double2* lg = (!WANT_V && rlog && gl == 0)
                          ? rlog + ((size_t)sweep * nst + tstep) * ngroups + grp : nullptr;
        int mi = sl.g + j;
        if (mi >= sl.R) mi -= sl.R;
        double c = 1.0, s = 0.0;
        if (has_p && j < sl.R && mi < sl.m) {
          const int q = sl.s1 + mi;
          double* mq = Mc + q * cst + gl;
          double y[RPL];
#pragma unroll
          for (int i = 0; i < RPL; ++i) y[i] = mq[roff(i)];
          double alx, be, ga;
          if constexpr (CARRY) {
            // alpha and beta from the carried norms; gamma in three partial
            // sums (three independent FMA chains instead of one)
            alx = al;
            be = nrm[q];
            double g3[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < RPL; ++i) g3[i % 3] += x[i] * y[i];
            ga = gsum((g3[0] + g3[1]) + g3[2]);
          } else {
            alx = 0.0; be = 0.0; ga = 0.0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) { alx += x[i] * x[i]; be += y[i] * y[i]; ga += x[i] * y[i]; }
            alx = gsum(alx); be = gsum(be); ga = gsum(ga);
          }
          if (ga * ga > tol2 * (alx * be)) {  // else orthogonal enough (or a zero column)
            double vy[RPL];
            const int iql = okl ? q * vld + rl : vdummy;
            if (WANT_V) {
              // read before the rotation is formed, so that the latency
              // overlaps the division and square roots
#pragma unroll
              for (int i = 0; i < RPL - 1; ++i) vy[i] = Vc[q * vld + gl + GL * i];
              vy[RPL - 1] = Vc[iql];
            }
            double tr;
            jac_rotation(alx, be, ga, c, s, tr);
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
              const double xi = x[i];
              x[i] = c * xi - s * y[i];
              y[i] = s * xi + c * y[i];
              mq[roff(i)] = y[i];
            }
            if constexpr (CARRY) {
              // the rotated pair's squared norms are the eigenvalues of its
              // 2 x 2 Gram matrix: alpha - t gamma and beta + t gamma
              double a2 = fma(-tr, ga, alx), b2 = fma(tr, ga, be);
              if (!(a2 >= kJacNormKeep * alx && b2 >= kJacNormKeep * be)) {
                double sa = 0.0, sb = 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i) { sa += x[i] * x[i]; sb += y[i] * y[i]; }
                a2 = gsum(sa);
                b2 = gsum(sb);
              }
              al = a2;
              if (gl == 0) nrm[q] = b2;
            }
            if (WANT_V) {
#pragma unroll
              for (int i = 0; i < RPL; ++i) {
                const double xi = vx[i];
                vx[i] = c * xi - s * vy[i];
                vy[i] = s * xi + c * vy[i];
              }
#pragma unroll
              for (int i = 0; i < RPL - 1; ++i) Vc[q * vld + gl + GL * i] = vy[i];
              Vc[iql] = vy[RPL - 1];
            }
            if (gl == 0) s_rot = 1;
          }
        }
        if (lg) *lg = double2{c, s};
        if (j == H - 1 && has_p) {
          // end of the level: the stationary column back to LDS (no other
          // group reads it during this level)
#pragma unroll
          for (int i = 0; i < RPL; ++i) mp[roff(i)] = x[i];
          if constexpr (CARRY) if (gl == 0) nrm[p] = al;
          if (WANT_V) {
#pragma unroll
            for (int i = 0; i < RPL - 1; ++i) Vc[p * vld + gl + GL * i] = vx[i];
            Vc[ipl] = vx[RPL - 1];
          }
        }
        __syncthreads();
      }
    }
    const int rot = s_rot;
    __syncthreads();
    if (!rot) break;
  }
  if (tid == 0) {
    info->sweeps = sweep + (sweep < max_sweeps ? 1 : 0);
    if (sweep >= max_sweeps) atomicOr(&info->flags, kFlagNoConv);
  }
  // column norms -> singular values (groups of 8 lanes from here on)
  const int g8 = tid / 8, l8 = tid % 8;
  for (int c = g8; c < l; c += kJacThreads / 8) {
    double a = 0.0;
    for (int r = l8; r < l; r += 8) a += Mc[c * cst + r] * Mc[c * cst + r];
    a = sum8(a);
    if (l8 == 0) sig[c] = sqrt(a);
  }
  __syncthreads();
  // rank of each column in descending order (ties: lower index first)
  for (int c = g8; c < l; c += kJacThreads / 8) {
    const double sc = sig[c];
    int rank = 0;
    for (int i = l8; i < l; i += 8) rank += (sig[i] > sc || (sig[i] == sc && i < c)) ? 1 : 0;
    for (int off = 4; off >= 1; off >>= 1) rank += __shfl_xor(rank, off, kWave);
    if (rank < k) {
      const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
      for (int r = l8; r < l; r += 8) {
        Ut[r * ldk + rank] = Mc[c * cst + r] * inv;
        if (WANT_V) Vt[r * ldk + rank] = Vc[c * vld + r];
      }
      if (l8 == 0) sv[rank] = sc;
      if (!WANT_V && vperm && l8 == 0) vperm[rank] = c;
    }
  }
}

}  // namespace sor
