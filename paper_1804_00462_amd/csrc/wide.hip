// The l x l steps of the method for sketch widths l > 128, spread over many
// workgroups (the one-workgroup kernels of small.hip hold l <= 128):
//
//   * the Cholesky factor of the Gram matrix G = T^T T of a sketch (the QR
//     step of Alg. 3 / Alg. 4 as Cholesky QR, T = Q R with R^T R = G) and
//     Z = R^{-1}, blocked in 64 x 64 blocks, with the same shift rule as the
//     one-workgroup factor;
//   * the core SVD of M = Q1^T A Q2 (Alg. 3 step 6) by one-sided Jacobi
//     rotations, with the columns grouped in blocks that meet in pairs.
//
// Matrices are FP64, row-major l x l inside LP x LP buffers (ld LP); entries
// at indices >= l are zero on input and stay zero.
#include <algorithm>

#include "small_body.hpp"

namespace sor {

namespace {

constexpr int kWB = 64;        // Cholesky block edge
constexpr int kWLd = kWB + 2;  // LDS row stride of a 64 x 64 block

__device__ inline bool gate_off(const int* skip, const int* need) {
  return (skip && *skip) || (need && !*need);
}

// A 64 x 64 block (rows r0.., columns c0..) of an LP x LP matrix into LDS
// (row stride kWLd), zero outside the buffer.
__device__ inline void load_block64(const double* __restrict__ M, int LP, int r0, int c0, double* S) {
  for (int i = threadIdx.x; i < kWB * kWB; i += 256) {
    const int r = i / kWB, c = i % kWB;
    const int gr = r0 + r, gc = c0 + c;
    S[r * kWLd + c] = (gr < LP && gc < LP) ? M[(int64_t)gr * LP + gc] : 0.0;
  }
}

// acc[ct] += sum_{k in [k0, k1)} A(16 w + i, k) B(k, 16 ct + j) for the 16-row
// strip of wave w, on FP64 MFMA (16 x 16 x 4); A(i, k) = As[k][i] when TA,
// else As[i][k]; both operands in LDS with row stride kWLd. Result layout:
// acc[ct][r] holds C(16 w + 4 r + l / 16, 16 ct + l % 16) for lane l.
template <bool TA>
__device__ inline void mm64(const double* As, const double* Bs, int k0, int k1, f64x4 (&acc)[4]) {
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int li = l % 16, g = l / 16;
  const int i = 16 * w + li;
  for (int kb = k0; kb < k1; kb += 4) {
    const int k = kb + g;
    const double a = TA ? As[k * kWLd + i] : As[i * kWLd + k];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[k * kWLd + 16 * ct + li], acc[ct], 0, 0, 0);
  }
}

__device__ inline void store_acc64(const f64x4 (&acc)[4], double* S) {
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  const int li = l % 16, g = l / 16;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) S[(16 * w + 4 * r + g) * kWLd + 16 * ct + li] = acc[ct][r];
}

}  // namespace

// Small state of a blocked factorization (in the workspace).
struct WideChol {
  int32_t retry;  // a pivot of the unshifted factor failed the check
  int32_t pad_;
  double tr;      // trace of G
};

// ---------------------------------------------------------------------------
// Blocked Cholesky factor. With S the current Schur complement, panel p
// (rows / columns J = [64 p, 64 p + 64)) factors S_JJ = R_JJ^T R_JJ and forms
// R_JI = R_JJ^{-T} S_JI for the trailing blocks I and S_IK <- S_IK - R_JI^T R_JK
// (right-looking; one launch per panel, one workgroup per trailing block
// (I, K), I <= K, each forming the diagonal factor itself). The pivot rule is
// the one-workgroup factor's: an unshifted factor whose pivot d_j falls below
// 1e-13 G_jj (column j nearly in the span of the earlier ones) raises
// `retry`, and the factor is taken again from G + c u tr(G) I (c = 11 (rows
// l + l (l + 1)), u = 2^-53); a pivot that is still not positive then drops
// its column (zero row of R, zero row and column of Z; flag bit 2).
// Z = R^{-1} is then formed by doubling: with Z known on diagonal blocks of
// edge s, the block above the diagonal of each pair is
// Z_12 = -Z_11 R_12 Z_22 (two launches per level).

// Copies G to G0, clears R and Z, takes the diagonal and trace of G (block 0).
__global__ void __launch_bounds__(256)
k_wchol_prep(const double* __restrict__ G, int LP, int l, double* __restrict__ G0, double* __restrict__ Rb,
             double* __restrict__ Z, double* __restrict__ d0, WideChol* __restrict__ st, const int* skip) {
  if (skip && *skip) return;
  const int64_t tot = (int64_t)LP * LP;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (int64_t)gridDim.x * 256) {
    G0[i] = G[i];
    Rb[i] = 0.0;
    Z[i] = 0.0;
  }
  if (blockIdx.x == 0) {
    __shared__ double part[256];
    double a = 0.0;
    for (int j = threadIdx.x; j < l; j += 256) {
      const double d = G[(int64_t)j * LP + j];
      d0[j] = d;
      a += d;
    }
    part[threadIdx.x] = a;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
      if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      st->tr = part[0];
      st->retry = 0;
    }
  }
}

// G <- G0 + shift I (the shifted factor).
__global__ void __launch_bounds__(256)
k_wchol_restore(double* __restrict__ G, const double* __restrict__ G0, int LP, int l, int64_t rows,
                const WideChol* __restrict__ st, const int* skip, const int* need) {
  if (gate_off(skip, need)) return;
  const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * 0x1p-53 * st->tr;
  const int64_t tot = (int64_t)LP * LP;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / LP, c = i % LP;
    G[i] = G0[i] + ((r == c && r < l) ? shift : 0.0);
  }
}

__global__ void __launch_bounds__(256)
k_wchol_panel(double* __restrict__ G, int LP, int l, int p, const double* __restrict__ d0, int check,
              double* __restrict__ Rb, double* __restrict__ Z, WideChol* __restrict__ st, DevInfo* __restrict__ info,
              const int* skip, const int* need) {
  if (gate_off(skip, need)) return;
  __shared__ double Zs[kWB * kWLd], Si[kWB * kWLd], Sj[kWB * kWLd];
  const int nbk = (l + kWB - 1) / kWB;
  const int T = nbk - p - 1;  // trailing blocks
  int I = p, K = p;
  if (T > 0) {  // block index -> (i, k), 0 <= i <= k < T; row i holds T - i of them
    int b = blockIdx.x, i = 0;
    while (b >= T - i) {
      b -= T - i;
      ++i;
    }
    I = p + 1 + i;
    K = I + b;
  }
  const int r0 = kWB * p;
  load_block64(G, LP, r0, r0, Zs);
  if (T > 0) {
    load_block64(G, LP, r0, kWB * I, Si);
    if (K != I) load_block64(G, LP, r0, kWB * K, Sj);
  }
  __syncthreads();
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const bool lead = blockIdx.x == 0;
  if (w == 0) {
    // Wave 0: lane c holds column c of the diagonal block, s[i] = S(i, c),
    // and runs the elimination: step j scales row j by 1 / sqrt(d_j) (lane
    // c >= j then holds R(j, c)) and subtracts R(j, i) R(j, c) from S(i, c),
    // i > j. The R(j, i) come from lane i by readlane.
    double s[kWB];
#pragma unroll
    for (int i = 0; i < kWB; ++i) s[i] = Zs[i * kWLd + lane];
    bool bad = false, drop = false;
#pragma unroll
    for (int j = 0; j < kWB; ++j) {
      const double d = readlane_f64(s[j], j);
      const int gj = r0 + j;
      const bool pad = gj >= l;
      if (!pad && check && !(d > 1e-13 * d0[min(gj, l - 1)])) bad = true;
      const bool ok = !pad && d > 0.0;
      if (!pad && !check && !ok) drop = true;
      const double isd = ok ? 1.0 / sqrt(d) : 0.0;
      s[j] = lane >= j ? s[j] * isd : 0.0;
#pragma unroll
      for (int i = j + 1; i < kWB; ++i) s[i] = fma(-readlane_f64(s[j], i), s[j], s[i]);
    }
    // R_JJ into LDS (rows j, lane = column) and, by the lead workgroup, to Rb
#pragma unroll
    for (int j = 0; j < kWB; ++j) {
      Zs[j * kWLd + lane] = s[j];
      if (lead && r0 + j < LP && r0 + lane < LP) Rb[(int64_t)(r0 + j) * LP + r0 + lane] = s[j];
    }
    // Z_JJ = R_JJ^{-1} by back substitution, lane c forming column c:
    // z_i = (delta_ic - sum_{t > i} R(i, t) z_t) / R(i, i) (0 for a dropped i)
    double z[kWB];
#pragma unroll
    for (int i = kWB - 1; i >= 0; --i) {
      double a = i == lane ? 1.0 : 0.0;
#pragma unroll
      for (int t = i + 1; t < kWB; ++t) a = fma(-Zs[i * kWLd + t], z[t], a);
      const double rii = Zs[i * kWLd + i];
      z[i] = rii != 0.0 ? a / rii : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kWB; ++i) {
      Zs[i * kWLd + lane] = z[i];
      if (lead && r0 + i < LP && r0 + lane < LP) Z[(int64_t)(r0 + i) * LP + r0 + lane] = z[i];
    }
    if (lead && lane == 0) {
      if (bad) st->retry = 1;
      if (drop) atomicOr(&info->flags, kFlagQrBreakdown);
    }
  }
  __syncthreads();
  if (T == 0) return;
  // R_JI = Z_JJ^T S_JI (Z_JJ(k, i) = 0 for k > i: the strip of wave w needs k < 16 (w + 1))
  f64x4 ri[4], rk[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) ri[ct] = rk[ct] = f64x4{0, 0, 0, 0};
  mm64<true>(Zs, Si, 0, 16 * (w + 1), ri);
  if (K != I) mm64<true>(Zs, Sj, 0, 16 * (w + 1), rk);
  __syncthreads();
  store_acc64(ri, Si);
  if (K != I) store_acc64(rk, Sj);
  __syncthreads();
  if (K == I) {  // the diagonal trailing block publishes R_JI
    for (int e = threadIdx.x; e < kWB * kWB; e += 256) {
      const int r = e / kWB, c = e % kWB;
      const int gr = r0 + r, gc = kWB * I + c;
      if (gr < LP && gc < LP) Rb[(int64_t)gr * LP + gc] = Si[r * kWLd + c];
    }
  }
  // S_IK -= R_JI^T R_JK
  f64x4 u[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) u[ct] = f64x4{0, 0, 0, 0};
  mm64<true>(Si, K != I ? Sj : Si, 0, kWB, u);
  const int li = lane % 16, g = lane / 16;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = kWB * I + 16 * w + 4 * r + g, gc = kWB * K + 16 * ct + li;
      if (gr < LP && gc < LP) G[(int64_t)gr * LP + gc] -= u[ct][r];
    }
}

// One launch of a doubling level of Z = R^{-1} (pairs of diagonal blocks of
// edge s, the first starting at a0 = 2 s pair, the second at b0 = a0 + s):
//   step 0: X_12 = R_12 Z_22     (Z_22 upper triangular: k < c + 1)
//   step 1: Z_12 = -Z_11 X_12    (Z_11 upper triangular: k >= r)
// One workgroup per 64 x 64 output tile; operands staged through LDS in
// slices of 32 contraction indices.
__global__ void __launch_bounds__(256)
k_wchol_inv(int LP, int l, int s, int step, const double* __restrict__ Rb, double* __restrict__ Z,
            double* __restrict__ X, const int* skip) {
  if (skip && *skip) return;
  __shared__ double As[kWB * 34], Bs[32 * kWLd];
  const int lw = (l + kWB - 1) / kWB * kWB;
  const int tpb = s / kWB;
  const int pair = blockIdx.x / (tpb * tpb), t = blockIdx.x % (tpb * tpb);
  const int ti = t / tpb, tj = t % tpb;
  const int a0 = 2 * s * pair, b0 = a0 + s;
  const int b1 = min(b0 + s, lw);
  if (b0 + kWB * tj >= b1) return;  // beyond a ragged second block (uniform)
  const int row0 = a0 + kWB * ti, col0 = b0 + kWB * tj;
  const double* A = step == 0 ? Rb : Z;
  const double* B = step == 0 ? Z : X;
  const int k0 = step == 0 ? b0 : row0;
  const int k1 = step == 0 ? col0 + kWB : a0 + s;
  const double alpha = step == 0 ? 1.0 : -1.0;
  double* C = step == 0 ? X : Z;
  const int w = threadIdx.x / kWave, l64 = threadIdx.x % kWave;
  const int li = l64 % 16, g = l64 / 16;
  f64x4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = f64x4{0, 0, 0, 0};
  for (int kb = k0; kb < k1; kb += 32) {
    for (int e = threadIdx.x; e < kWB * 32; e += 256) {
      const int r = e / 32, k = e % 32;
      const int gr = row0 + r, gk = kb + k;
      As[r * 34 + k] = (gr < LP && gk < LP && gk < k1) ? A[(int64_t)gr * LP + gk] : 0.0;
    }
    for (int e = threadIdx.x; e < 32 * kWB; e += 256) {
      const int k = e / kWB, c = e % kWB;
      const int gk = kb + k, gc = col0 + c;
      Bs[k * kWLd + c] = (gk < LP && gc < LP && gk < k1) ? B[(int64_t)gk * LP + gc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4) {
      const double a = As[(16 * w + li) * 34 + kk + g];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
        acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[(kk + g) * kWLd + 16 * ct + li], acc[ct], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gr = row0 + 16 * w + 4 * r + g, gc = col0 + 16 * ct + li;
      if (gr < LP && gc < LP) C[(int64_t)gr * LP + gc] = alpha * acc[ct][r];
    }
}

// The third Cholesky-QR step is needed only after a shifted factor (see
// chol_inv_body): mode 0 sets *skip3 when the factor was unshifted, mode 1
// clears it when it was shifted.
__global__ void __launch_bounds__(64) k_wchol_skipset(const WideChol* __restrict__ st, int mode, int* skip3) {
  if (threadIdx.x) return;
  if (mode == 0) *skip3 = st->retry ? 0 : 1;
  else if (mode == 1 && st->retry) *skip3 = 0;
}

// Scratch of launch_chol_wide: G0, R (LP x LP each), X (LP x LP), the
// diagonal of G (LP) and the state record.
size_t chol_wide_bytes(int LP) { return ((size_t)3 * LP * LP + LP) * 8 + 256; }

hipError_t launch_chol_wide(double* G, int LP, int l, int64_t rows, int mode, double* Z, int* skip3, void* info,
                            void* scratch, hipStream_t st) {
  if (l <= 0 || l > LP) return hipErrorInvalidValue;
  double* G0 = reinterpret_cast<double*>(scratch);
  double* Rb = G0 + (size_t)LP * LP;
  double* X = Rb + (size_t)LP * LP;
  double* d0 = X + (size_t)LP * LP;
  WideChol* wc = reinterpret_cast<WideChol*>(d0 + LP);
  const int* skip = mode == 2 ? skip3 : nullptr;
  DevInfo* di = (DevInfo*)info;
  const int64_t tot = (int64_t)LP * LP;
  const unsigned cblocks = (unsigned)std::min<int64_t>(1024, ceil_div(tot, 256));
  hipLaunchKernelGGL(k_wchol_prep, dim3(cblocks), dim3(256), 0, st, G, LP, l, G0, Rb, Z, d0, wc, skip);
  const int nbk = (int)ceil_div(l, kWB);
  for (int pass = 0; pass < 2; ++pass) {
    const int* need = pass == 0 ? nullptr : &wc->retry;
    if (pass == 1)
      hipLaunchKernelGGL(k_wchol_restore, dim3(cblocks), dim3(256), 0, st, G, G0, LP, l, rows, wc, skip, need);
    for (int p = 0; p < nbk; ++p) {
      const int T = nbk - p - 1;
      const unsigned blocks = (unsigned)std::max(1, T * (T + 1) / 2);
      hipLaunchKernelGGL(k_wchol_panel, dim3(blocks), dim3(256), 0, st, G, LP, l, p, d0, pass == 0 ? 1 : 0, Rb, Z,
                         wc, di, skip, need);
    }
  }
  const int lw = nbk * kWB;
  for (int s = kWB; s < lw; s *= 2) {
    const int pairs = (int)ceil_div(lw - s, 2 * s);  // pairs whose second block starts below lw
    const int tpb = s / kWB;
    for (int step = 0; step < 2; ++step)
      hipLaunchKernelGGL(k_wchol_inv, dim3((unsigned)(pairs * tpb * tpb)), dim3(256), 0, st, LP, l, s, step, Rb, Z,
                         X, skip);
  }
  if (mode != 2) hipLaunchKernelGGL(k_wchol_skipset, dim3(1), dim3(64), 0, st, wc, mode, skip3);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Core SVD for l > 128: one-sided Jacobi on the columns of M, blocked. The
// columns (zero-padded to nbe blocks of B, nbe even) are held column-major
// in global memory (Mc, V in Vc, column stride ldc >= l, rows >= l zero). A
// sweep pairs the blocks by the round-robin order (nbe - 1 steps of nbe / 2
// disjoint block pairs; block 0 stays, the others move one place per step).
// Per step one workgroup takes each block pair: its 2B columns go to LDS and
// their Gram matrix G is formed; one round-robin sweep of pair rotations runs
// on G (the rotation of the one-workgroup kernel, jac_rotation, applied when
// gamma^2 > tol^2 alpha beta, as G <- J^T G J), while the product W of the
// rotations (2B x 2B) is accumulated; then the columns are multiplied by W
// and W is published. V is not touched by these workgroups: the same launch
// carries further workgroups that multiply the columns of V of the previous
// step's block pairs by that step's W (V is read by no step, so its update
// can trail by one launch and runs on CUs the block pairs leave idle; one
// launch after the last step applies the last W). Every pair of columns meets at
// least once per sweep. A sweep in which no workgroup rotated ends the
// iteration (the later launches return at once); then sigma_j = |m_j|,
// U~_j = m_j / sigma_j, V~_j = v_j, in descending order (ties: lower index).

struct WideJacDims {
  int B, nbe, ldc;
};

WideJacDims wjac_dims(int l) {
  WideJacDims d;
  d.ldc = (int)round_up(l, 32);
  d.B = ((size_t)32 * d.ldc + 2 * 32 * 32) * 8 <= 150 * 1024 ? 16 : 8;
  const int nb = (int)ceil_div(l, d.B);
  d.nbe = nb + (nb & 1);
  if (d.nbe < 2) d.nbe = 2;
  return d;
}

// Scratch of launch_jacobi_wide: Mc, Vc (nbe B x ldc each), the singular
// values (l), the W of every block pair for two consecutive steps (2 x nbe/2
// x (2B)^2), the per-sweep rotation counters (up to kWideMaxSweeps), the
// convergence word, and the step tags of the published W (2 x nbe/2).
constexpr int kWideMaxSweeps = 64;
size_t jacobi_wide_bytes(int l) {
  const WideJacDims d = wjac_dims(l);
  const size_t npair = (size_t)d.nbe / 2, nl = 2 * (size_t)d.B;
  return ((size_t)2 * d.nbe * d.B * d.ldc + l + 2 * npair * nl * nl) * 8 + ((size_t)kWideMaxSweeps + 64) * 4 +
         2 * npair * 4;
}

__global__ void __launch_bounds__(256)
k_wjac_init(const double* __restrict__ M, int LPm, int l, int trans, int ncp, int ldc, double* __restrict__ Mc,
            double* __restrict__ Vc, int* __restrict__ cnt, int max_sweeps, int* __restrict__ wtag, int ntag) {
  const int64_t tot = (int64_t)ncp * ldc;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < tot; e += (int64_t)gridDim.x * 256) {
    const int j = (int)(e / ldc), i = (int)(e % ldc);
    Mc[e] = (i < l && j < l) ? M[trans ? (int64_t)j * LPm + i : (int64_t)i * LPm + j] : 0.0;
    Vc[e] = (i == j && j < l) ? 1.0 : 0.0;
  }
  if (blockIdx.x == 0) {
    for (int s = threadIdx.x; s <= max_sweeps; s += 256) cnt[s] = 0;  // cnt[max_sweeps]: convergence word
    for (int s = threadIdx.x; s < ntag; s += 256) wtag[s] = 0;         // no W published yet
  }
}

// V <- V W for the block pair pr of step tp (W column-major, from the step's
// published buffer), rows [r0, r1) in 16-row tiles: wave w takes the tiles
// w, w + 4, ..., four at a time, all their loads in flight before any store;
// the product as (V W)^T = W^T V^T, as for the columns (128-byte stores).
template <int B>
__device__ void wjac_apply_v(double* __restrict__ Vc, int ldc, int nbe, int pr, int tp,
                             const double* __restrict__ W, int r0, int r1) {
  constexpr int NL = 2 * B, NT = NL / 16, TB = 4;
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave, li = lane % 16, g = lane / 16;
  auto player = [](int pos, int step, int n) {
    if (pos == 0) return 0;
    int x = pos - 1 + step;
    if (x >= n - 1) x -= n - 1;
    return 1 + x;
  };
  const int bp = player(pr, tp, nbe), bq = player(nbe - 1 - pr, tp, nbe);
  auto gcol = [&](int c) { return c < B ? bp * B + c : bq * B + (c - B); };
  double wb[NT][NL / 4];
#pragma unroll
  for (int ct = 0; ct < NT; ++ct)
#pragma unroll
    for (int s4 = 0; s4 < NL / 4; ++s4) wb[ct][s4] = W[(16 * ct + li) * NL + 4 * s4 + g];  // W(4 s + g, 16 ct + li)
  for (int rb = r0 + 16 * w; rb < r1; rb += 64 * TB) {
    double va[TB][NL / 4];
#pragma unroll
    for (int tb = 0; tb < TB; ++tb) {
      const int rt = rb + 64 * tb;
      if (rt < r1) {
#pragma unroll
        for (int s4 = 0; s4 < NL / 4; ++s4) va[tb][s4] = Vc[(int64_t)gcol(4 * s4 + g) * ldc + rt + li];
      }
    }
#pragma unroll
    for (int tb = 0; tb < TB; ++tb) {
      const int rt = rb + 64 * tb;
      if (rt >= r1) break;
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) {
        f64x4 av = f64x4{0, 0, 0, 0};
#pragma unroll
        for (int s4 = 0; s4 < NL / 4; ++s4) av = __builtin_amdgcn_mfma_f64_16x16x4f64(wb[ct][s4], va[tb][s4], av, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) Vc[(int64_t)gcol(16 * ct + 4 * r + g) * ldc + rt + li] = av[r];
      }
    }
  }
}

// One launch per step t of sweep `sweep` (global step s = sweep (nbe - 1) + t).
// Workgroups [0, xparts) take the block pairs of step s (xparts = nbe / 2, or
// 0 for the launch that only applies the last W); workgroup xparts + pr
// vchunks + ch applies the W of pair pr of step s - 1 to row chunk ch of V,
// if that step published it: W of step s goes to buffer s % 2 of Wg with tag
// s + 1 in wtag (tags are unique within a run and cleared at its start, so a
// buffer left from step s - 2 never matches).
template <int B>
__global__ void __launch_bounds__(256)
k_wjac_step(double* __restrict__ Mc, double* __restrict__ Vc, int ldc, int l, int nbe, int t, int sweep,
            int* __restrict__ cnt, const int* __restrict__ conv, double tol2, double* __restrict__ Wg,
            int* __restrict__ wtag, int xparts, int vchunks) {
  constexpr int NL = 2 * B, NP = NL / 2, NT = NL / 16;  // columns, pairs per round, 16-column tiles
  const int npair = nbe / 2, gs = sweep * (nbe - 1) + t;
  if ((int)blockIdx.x >= xparts) {
    const int vb = (int)blockIdx.x - xparts, pr = vb / vchunks, ch = vb % vchunks;
    const int pb = (gs - 1) & 1;
    if (gs == 0 || wtag[pb * npair + pr] != gs) return;
    const int crow = (int)round_up(ceil_div(ldc, vchunks), 16);
    const int r0 = ch * crow, r1 = min(ldc, r0 + crow);
    if (r0 < r1)
      wjac_apply_v<B>(Vc, ldc, nbe, pr, t == 0 ? nbe - 2 : t - 1, Wg + ((size_t)pb * npair + pr) * NL * NL, r0, r1);
    return;
  }
  if (*conv) return;
  extern __shared__ double sm[];
  double* Ms = sm;              // NL columns of ldc
  double* Gs = sm + NL * ldc;   // Gram matrix of the columns, row-major NL x NL
  double* Ws = Gs + NL * NL;    // W, column-major: W(r, c) = Ws[c NL + r]
  double* Gp = Ws + NL * NL;    // per-wave partial Gram (NL = 16: the waves split the rows)
  __shared__ int s_rot;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave, li = lane % 16, g = lane / 16;
  auto player = [](int pos, int step, int n) {
    if (pos == 0) return 0;
    int x = pos - 1 + step;
    if (x >= n - 1) x -= n - 1;
    return 1 + x;
  };
  const int bp = player(blockIdx.x, t, nbe), bq = player(nbe - 1 - blockIdx.x, t, nbe);
  auto gcol = [&](int c) { return c < B ? bp * B + c : bq * B + (c - B); };
  // columns to LDS: a thread loads its rows of all NL columns before storing
  // any (2 NL loads in flight per thread for B = 8; ldc is a multiple of 32)
  constexpr int RR = NL == 16 ? 2 : 1;
  for (int r = tid; r < ldc; r += 256 * RR) {
    double v[RR][NL];
#pragma unroll
    for (int u = 0; u < RR; ++u)
#pragma unroll
      for (int c = 0; c < NL; ++c) v[u][c] = r + 256 * u < ldc ? Mc[(int64_t)gcol(c) * ldc + r + 256 * u] : 0.0;
#pragma unroll
    for (int u = 0; u < RR; ++u)
      if (r + 256 * u < ldc)
#pragma unroll
        for (int c = 0; c < NL; ++c) Ms[c * ldc + r + 256 * u] = v[u][c];
  }
  for (int e = tid; e < NL * NL; e += 256) Ws[e] = (e / NL == e % NL) ? 1.0 : 0.0;
  if (tid == 0) s_rot = 0;
  __syncthreads();
  // Gram matrix G = X^T X on FP64 MFMA (16 x 16 x 4): lane (li, g) feeds
  // X(k0 + g, col) as both operands. NL = 16: one tile, the four waves take
  // a quarter of the rows each and the partial tiles are added in wave
  // order; NL = 32: wave w forms tile (w / 2, w % 2) over all rows.
  {
    f64x4 acc = f64x4{0, 0, 0, 0};
    int ti, tj, r0, r1;
    if constexpr (NT == 1) {
      ti = tj = 0;
      r0 = w * (ldc / 4);
      r1 = r0 + ldc / 4;
    } else {
      ti = w / 2;
      tj = w % 2;
      r0 = 0;
      r1 = ldc;
    }
    const double* xa = Ms + (16 * ti + li) * ldc;
    const double* xb = Ms + (16 * tj + li) * ldc;
    for (int kb = r0; kb < r1; kb += 4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[kb + g], xb[kb + g], acc, 0, 0, 0);
    if constexpr (NT == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Gp[w * 256 + (4 * r + g) * 16 + li] = acc[r];
      __syncthreads();
      const double v = (Gp[tid] + Gp[256 + tid]) + (Gp[512 + tid] + Gp[768 + tid]);
      Gs[tid] = v;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) Gs[(16 * ti + 4 * r + g) * NL + 16 * tj + li] = acc[r];
    }
  }
  __syncthreads();
  // One round-robin sweep of rotations on G (the rotations one-sided Jacobi
  // would apply to the columns: G is their Gram matrix, updated as
  // G <- J^T G J), accumulated in W <- W J; the NP pairs of a round are
  // disjoint. Wave 0 alone runs it. Lane b takes the 2 x 2 blocks (pair i,
  // pair j) with j = b % NP and i = b / NP, b / NP + 64 / NP, ...: it forms
  // the rotation of pair j itself (every lane with the same j gets the same
  // bits) and takes that of pair i from lane i, then rotates its blocks of G
  // by both (columns by pair j, rows by pair i) and its blocks of W by pair
  // j. The blocks cover G and W once. A wave performs its LDS accesses in
  // order, so a round only waits for its own LDS writes before the next
  // round reads them (no workgroup barrier inside the sweep).
  if (w == 0) {
    constexpr int NI = NP * NP / kWave;  // blocks per lane
    auto wave_lds_sync = [] { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); };
    auto pair_of = [&](int i, int step, int& p, int& q) {
      p = player(i, step, NL);
      q = player(NL - 1 - i, step, NL);
      if (p > q) {
        const int x = p;
        p = q;
        q = x;
      }
    };
    const int j = lane % NP;
    bool rotated = false;
    for (int step = 0; step < NL - 1; ++step) {
      int pj, qj, pi[NI], qi[NI];
      pair_of(j, step, pj, qj);
      const double al = Gs[pj * NL + pj], be = Gs[qj * NL + qj], ga = Gs[pj * NL + qj];
      double g[NI][4], wv[NI][4];
#pragma unroll
      for (int u = 0; u < NI; ++u) {
        pair_of(lane / NP + u * (kWave / NP), step, pi[u], qi[u]);
        g[u][0] = Gs[pi[u] * NL + pj];
        g[u][1] = Gs[pi[u] * NL + qj];
        g[u][2] = Gs[qi[u] * NL + pj];
        g[u][3] = Gs[qi[u] * NL + qj];
        wv[u][0] = Ws[pj * NL + pi[u]];
        wv[u][1] = Ws[qj * NL + pi[u]];
        wv[u][2] = Ws[pj * NL + qi[u]];
        wv[u][3] = Ws[qj * NL + qi[u]];
      }
      double cj = 1.0, sj = 0.0;
      if (ga * ga > tol2 * (al * be)) {
        jac_rotation(al, be, ga, cj, sj);
        rotated = true;
      }
#pragma unroll
      for (int u = 0; u < NI; ++u) {
        const int src = lane / NP + u * (kWave / NP);  // a lane whose j is pair i
        const double ci = __shfl(cj, src), si = __shfl(sj, src);
        if (si == 0.0 && sj == 0.0) continue;
        const double a0 = cj * g[u][0] - sj * g[u][1], b0 = sj * g[u][0] + cj * g[u][1];  // row p_i
        const double a1 = cj * g[u][2] - sj * g[u][3], b1 = sj * g[u][2] + cj * g[u][3];  // row q_i
        Gs[pi[u] * NL + pj] = ci * a0 - si * a1;
        Gs[qi[u] * NL + pj] = si * a0 + ci * a1;
        Gs[pi[u] * NL + qj] = ci * b0 - si * b1;
        Gs[qi[u] * NL + qj] = si * b0 + ci * b1;
        if (sj != 0.0) {  // W(r, p_j), W(r, q_j) for rows r = p_i, q_i
          Ws[pj * NL + pi[u]] = cj * wv[u][0] - sj * wv[u][1];
          Ws[qj * NL + pi[u]] = sj * wv[u][0] + cj * wv[u][1];
          Ws[pj * NL + qi[u]] = cj * wv[u][2] - sj * wv[u][3];
          Ws[qj * NL + qi[u]] = sj * wv[u][2] + cj * wv[u][3];
        }
      }
      wave_lds_sync();
    }
    if (__any(rotated) && lane == 0) s_rot = 1;
  }
  __syncthreads();
  if (!s_rot) return;  // the columns (and V) stay as they are
  // X <- X W (X from LDS) on FP64 MFMA, as (X W)^T = W^T X^T so that a
  // lane's four outputs are one column's rows and each store instruction
  // writes four columns x 16 rows (128-byte runs): wave w takes the 16-row
  // tiles w, w + 4, ...
  for (int r0 = 16 * w; r0 < ldc; r0 += 64) {
    double xa[NL / 4];
#pragma unroll
    for (int s4 = 0; s4 < NL / 4; ++s4) xa[s4] = Ms[(4 * s4 + g) * ldc + r0 + li];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      f64x4 ax = f64x4{0, 0, 0, 0};
#pragma unroll
      for (int s4 = 0; s4 < NL / 4; ++s4) {
        const double b = Ws[(16 * ct + li) * NL + 4 * s4 + g];  // W(4 s + g, 16 ct + li)
        ax = __builtin_amdgcn_mfma_f64_16x16x4f64(b, xa[s4], ax, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Mc[(int64_t)gcol(16 * ct + 4 * r + g) * ldc + r0 + li] = ax[r];
    }
  }
  // publish W for the next launch's V workgroups
  double* Wo = Wg + ((size_t)(gs & 1) * npair + blockIdx.x) * NL * NL;
  for (int e = tid; e < NL * NL; e += 256) Wo[e] = Ws[e];
  if (tid == 0) {
    wtag[(gs & 1) * npair + blockIdx.x] = gs + 1;
    atomicAdd(&cnt[sweep], 1);
  }
}

__global__ void __launch_bounds__(64)
k_wjac_sweep_end(int* __restrict__ cnt, int sweep, int max_sweeps, DevInfo* __restrict__ info) {
  if (threadIdx.x) return;
  int* conv = cnt + max_sweeps;
  if (*conv) return;
  if (cnt[sweep] == 0) {
    *conv = 1;
    info->sweeps = sweep + 1;
  } else if (sweep == max_sweeps - 1) {
    info->sweeps = max_sweeps;
    atomicOr(&info->flags, kFlagNoConv);
  }
}

// sig[j] = |m_j| (fixed-order tree sum), one workgroup per column.
__global__ void __launch_bounds__(256)
k_wjac_norms(const double* __restrict__ Mc, int ldc, int l, double* __restrict__ sig) {
  __shared__ double part[256];
  const int j = blockIdx.x;
  double a = 0.0;
  for (int r = threadIdx.x; r < l; r += 256) {
    const double x = Mc[(int64_t)j * ldc + r];
    a = fma(x, x, a);
  }
  part[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sig[j] = sqrt(part[0]);
}

// Rank of column j by descending sigma (ties: lower index first); the first
// k go to Ut, Vt (l x k, ld ldk) and sv.
__global__ void __launch_bounds__(256)
k_wjac_out(const double* __restrict__ Mc, const double* __restrict__ Vc, int ldc, int l, int k,
           const double* __restrict__ sig, double* __restrict__ Ut, double* __restrict__ sv, double* __restrict__ Vt,
           int ldk) {
  __shared__ int part[256];
  const int j = blockIdx.x;
  const double sj = sig[j];
  int cntr = 0;
  for (int i = threadIdx.x; i < l; i += 256) cntr += (sig[i] > sj || (sig[i] == sj && i < j)) ? 1 : 0;
  part[threadIdx.x] = cntr;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  const int rank = part[0];
  if (rank >= k) return;
  const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
  for (int r = threadIdx.x; r < l; r += 256) {
    Ut[(int64_t)r * ldk + rank] = Mc[(int64_t)j * ldc + r] * inv;
    Vt[(int64_t)r * ldk + rank] = Vc[(int64_t)j * ldc + r];
  }
  if (threadIdx.x == 0) sv[rank] = sj;
}

// M: l x l in an LPm-wide row-major buffer. tol <= 0: sqrt(l) 2^-52.
// max_sweeps <= kWideMaxSweeps; trans: the SVD of M^T.
hipError_t launch_jacobi_wide(const double* M, int LPm, int l, int k, int max_sweeps, double* Ut, double* sv,
                              double* Vt, int ldk, void* scratch, void* info, hipStream_t st, double tol, bool trans) {
  if (l < 2 || k < 1 || k > l || max_sweeps < 1 || max_sweeps > kWideMaxSweeps) return hipErrorInvalidValue;
  const WideJacDims d = wjac_dims(l);
  const int ncp = d.nbe * d.B;
  double* Mc = reinterpret_cast<double*>(scratch);
  double* Vc = Mc + (size_t)ncp * d.ldc;
  double* sig = Vc + (size_t)ncp * d.ldc;
  const int npair = d.nbe / 2;
  double* Wg = sig + l;
  int* cnt = reinterpret_cast<int*>(Wg + (size_t)2 * npair * (2 * d.B) * (2 * d.B));
  const int* conv = cnt + max_sweeps;
  int* wtag = cnt + kWideMaxSweeps + 64;
  // row chunks of V per block pair: the V workgroups fill the CUs the
  // npair block-pair workgroups leave (one workgroup per CU: the LDS of the
  // block pairs is sized for one), chunks of at least 64 rows
  const int vchunks = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(d.ldc, 64), (256 - npair) / npair));
  const double tol2 = tol > 0.0 ? tol * tol : (double)l * 0x1p-104;
  DevInfo* di = (DevInfo*)info;
  const int64_t tot = (int64_t)ncp * d.ldc;
  hipLaunchKernelGGL(k_wjac_init, dim3((unsigned)std::min<int64_t>(1024, ceil_div(tot, 256))), dim3(256), 0, st, M,
                     LPm, l, trans ? 1 : 0, ncp, d.ldc, Mc, Vc, cnt, max_sweeps, wtag, 2 * npair);
  // columns, G, W and the per-wave partial Gram (B = 8)
  const size_t shm = ((size_t)2 * d.B * d.ldc + 8 * d.B * d.B + (d.B == 8 ? 4 * 256 : 0)) * 8;
  auto step = [&](int xparts, int t, int sw) {
    const dim3 grid((unsigned)(xparts + npair * vchunks));
    if (d.B == 16)
      hipLaunchKernelGGL(k_wjac_step<16>, grid, dim3(256), shm, st, Mc, Vc, d.ldc, l, d.nbe, t, sw, cnt, conv, tol2,
                         Wg, wtag, xparts, vchunks);
    else
      hipLaunchKernelGGL(k_wjac_step<8>, grid, dim3(256), shm, st, Mc, Vc, d.ldc, l, d.nbe, t, sw, cnt, conv, tol2,
                         Wg, wtag, xparts, vchunks);
  };
  for (int sw = 0; sw < max_sweeps; ++sw) {
    for (int t = 0; t < d.nbe - 1; ++t) step(npair, t, sw);
    hipLaunchKernelGGL(k_wjac_sweep_end, dim3(1), dim3(64), 0, st, cnt, sw, max_sweeps, di);
  }
  step(0, 0, max_sweeps);  // V by the W of the last step
  hipLaunchKernelGGL(k_wjac_norms, dim3((unsigned)l), dim3(256), 0, st, Mc, d.ldc, l, sig);
  hipLaunchKernelGGL(k_wjac_out, dim3((unsigned)l), dim3(256), 0, st, Mc, Vc, d.ldc, l, k, sig, Ut, sv, Vt, ldk);
  return hipGetLastError();
}

}  // namespace sor
