// Batched SOR-SVD of many matrices of uneven sizes (Alg. 3 / Alg. 4 on each).
//
// Every step runs as ONE launch over all problems of the batch:
//   * passes over A, Gram products, T <- T R^{-1} and the lifts: a persistent
//     grid walks a host-built work list (largest items first) in a fixed
//     round-robin order, with the tile body of the single-problem path; the
//     start index is spread so that neighbouring items (row tiles of one
//     problem, sharing its skinny operand) run on the same XCD and its L2;
//   * Cholesky factor + inverse and the core SVD: one workgroup per problem;
//   * element-wise steps: a 2-D grid (grid column = problem).
// Every output element is accumulated in the same order whatever the tile
// height or grid size, so the results are bitwise independent of the launch
// configuration the autotuner picks. The launch sequence contains no memset
// and no allocation, so it can be captured in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sorsvd.h"
#include "skinny_body.hpp"
#include "small_body.hpp"

namespace sor {

hipError_t launch_omega_batch(const OmegaJob* jobs, int njobs, int64_t max_count, int f32, hipStream_t st);
hipEvent_t pass_timer_begin(hipStream_t st, double bytes, double flops);

namespace {

constexpr int kGramRows = 512;  // rows of T per Gram work item
constexpr int kMaxBatchLP = 128;
constexpr int kMaxBatch = 65535;
constexpr int kElemsPerBlock = 4096;  // element-wise kernels: elements per workgroup
// dynamic LDS of a tile kernel: its staged operand, then 4 doubles of reductions
template <typename T, int CT>
constexpr size_t xs_bytes() { return (size_t)xs_elems<T, CT>() * sizeof(T); }
template <typename T, int CT>
constexpr size_t tile_lds() { return xs_bytes<T, CT>() + 64; }

struct BProb {
  int64_t m, n;
  int k, l, LP, KP, q, vec_ok;
  const void* A;
  int64_t lda;
  double* U;
  int64_t ldu;
  double* S;
  double* V;
  int64_t ldv;
  void* Xc;       // skinny operand in A's type, max(m, n) x LP
  double* T1;     // m x LP: T1, then Q1
  double* T2;     // n x LP: T2, then Q2
  double* W;      // m x LP: A Q2
  double* U64;    // m x KP
  double* V64;    // n x KP
  double* Rinv;   // LP x LP
  double* Ut;     // LP x KP
  double* Vt;     // LP x KP
  double* Vg;     // LP x LP (Jacobi scratch)
  double* gpart;  // max(gch_m, gch_n) partial LP x LP products
  int gch_m, gch_n;
  double* normp;  // one sum of squares per 64-row tile of the first pass
  int ntile1;
  int sblocks;    // row blocks of the sign search
  double* pval;   // sblocks x KP
  int64_t* pidx;  // sblocks x KP
  double* sgn;    // KP
  int* skip3;
  DevInfo* info;
};

struct BItem {
  int32_t prob;
  int32_t chunk;  // tile index (row tiles) or row chunk (Gram)
  int64_t base;   // first output row of the tile
};

enum Mode : int {
  M_SKETCH = 0, M_ORBIT, M_PROJ,         // passes over A
  M_GRAM1, M_GRAM2, M_PGRAM,             // LP x LP products over row chunks
  M_APPLY1, M_APPLY2, M_LIFTU, M_LIFTV,  // row tiles times a small right operand
  M_COUNT
};

// ------------------------------------------------------------------ kernels

template <typename TA, bool TRANS, int RT, int CT>
__device__ void pass_item(const BProb& P, const BItem& I, int mode, bool want_norm, char* lds) {
  TA* Xs = reinterpret_cast<TA*>(lds);
  double* red = reinterpret_cast<double*>(lds + xs_bytes<TA, CT>());
  const int64_t OUT = TRANS ? P.n : P.m;
  const int64_t K = TRANS ? P.m : P.n;
  double* out = mode == M_SKETCH ? P.T1 : (mode == M_ORBIT ? P.T2 : P.W);
  double* nrm = want_norm ? P.normp + I.chunk : nullptr;
  // one step of prefetch for the widest 128-row tiles: two do not fit the
  // registers next to the persistent loop's state
  constexpr int PD = (sizeof(TA) == 4 && (CT <= 4 || (RT == 1 && CT == 5))) ? 2 : 1;
  skinny_tile<TA, TRANS, RT, CT, PD>(reinterpret_cast<const TA*>(P.A), P.lda, OUT, 0, K,
                                 reinterpret_cast<const TA*>(P.Xc), P.LP, I.base, P.vec_ok, nullptr, out, P.LP,
                                 nrm, Xs, red);
}

// Passes over A of the problems with LP = 16 CT. qiter >= 0: power-loop
// iteration qiter (problems with q <= qiter sit it out). want_norm: the first
// sketch pass also records the sum of squares of A per tile (with RT = 2 the
// tiles fill the first half of the slots, the rest stay zero).
template <typename TA, bool TRANS, int RT, int CT>
__global__ void __launch_bounds__(256, 2)
k_bpass(const BProb* __restrict__ probs, const BItem* __restrict__ items, int nitems, int mode, int qiter,
        int want_norm) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  for (int it = xcd_remap(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const BItem I = items[it];
    const BProb& P = probs[I.prob];
    if (qiter >= 0 && qiter >= P.q) continue;
    pass_item<TA, TRANS, RT, CT>(P, I, mode, want_norm != 0, lds);
  }
}

// Passes over A = diag(sigma) (given by its diagonal, m = n): out = diag(sigma) X
// for one 64-row tile, the same product for A and A^T; the first sketch also
// records the sum of sigma_r^2 over the tile.
__global__ void __launch_bounds__(256)
k_bdiag(const BProb* __restrict__ probs, const BItem* __restrict__ items, int nitems, int mode, int qiter,
        int want_norm) {
  __shared__ double red[4];
  for (int it = xcd_remap(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const BItem I = items[it];
    const BProb& P = probs[I.prob];
    if (qiter >= 0 && qiter >= P.q) continue;
    const double* sig = reinterpret_cast<const double*>(P.A);
    const double* X = reinterpret_cast<const double*>(P.Xc);
    double* out = mode == M_SKETCH ? P.T1 : (mode == M_ORBIT ? P.T2 : P.W);
    const int64_t r0 = I.base, r1 = min(P.n, r0 + 64);
    for (int64_t e = threadIdx.x; e < (r1 - r0) * P.LP; e += 256) {
      const int64_t r = r0 + e / P.LP;
      out[r * P.LP + e % P.LP] = sig[r] * X[r * P.LP + e % P.LP];
    }
    if (want_norm) {
      double a = 0.0;
      for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) a += sig[r] * sig[r];
      a = wave_sum(a);
      if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = a;
      __syncthreads();
      if (threadIdx.x == 0) P.normp[I.chunk] = (red[0] + red[1]) + (red[2] + red[3]);
      __syncthreads();
    }
  }
}

// Whether a problem skips Cholesky-QR step `step` of the QR at power step
// qiter (-1: before the loop): the third step runs only where the first one
// shifted; a basis that only feeds the next product (every QR but those of
// the problem's last power step) skips the second step as well, which leaves
// it orthonormal to ~cond^2 u, a well-conditioned basis of the same span.
__device__ inline bool qr_step_skipped(const BProb& P, int step, int qiter) {
  if (step == 2) return *P.skip3 != 0;
  return step == 1 && qiter != P.q - 1;
}

// FP64 products on the tall sketches, 64-row tiles, problems with LP = 16 CT
// (lifts: KP = 16 CT).
// Gram: T^T T (or Q1^T W) over one 512-row chunk, output rows [base, base + 64)
// of that chunk's LP x LP partial. step: the Cholesky-QR step (0 for the
// projection); see qr_step_skipped.
template <int CT>
__global__ void __launch_bounds__(256, 2)
k_bgram(const BProb* __restrict__ probs, const BItem* __restrict__ items, int nitems, int mode, int qiter,
        int step) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  double* Xs = reinterpret_cast<double*>(lds);
  double* red = reinterpret_cast<double*>(lds + xs_bytes<double, CT>());
  for (int it = xcd_remap(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const BItem I = items[it];
    const BProb& P = probs[I.prob];
    if (qiter >= 0 && qiter >= P.q) continue;
    if (qr_step_skipped(P, step, qiter)) continue;
    const double* T = mode == M_GRAM2 ? P.T2 : P.T1;
    const double* Y = mode == M_PGRAM ? P.W : T;
    const int64_t rows = mode == M_GRAM2 ? P.n : P.m;
    const int64_t r0 = (int64_t)I.chunk * kGramRows;
    const int64_t r1 = min(rows, r0 + kGramRows);
    // (T^T T: only its upper triangle, which the Cholesky factor reads)
    skinny_tile<double, true, 1, CT>(T, P.LP, P.LP, r0, r1, Y, P.LP, I.base, 1, nullptr,
                                     P.gpart + (int64_t)I.chunk * P.LP * P.LP, P.LP, nullptr, Xs, red,
                                     mode == M_PGRAM ? 0 : 2);
  }
}

// T <- T R^{-1} in place, one 64-row tile per item (a workgroup writes only
// the rows it has finished reading).
template <int CT>
__global__ void __launch_bounds__(256, 2)
k_bapply(const BProb* __restrict__ probs, const BItem* __restrict__ items, int nitems, int which, int qiter,
         int step) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  double* Xs = reinterpret_cast<double*>(lds);
  double* red = reinterpret_cast<double*>(lds + xs_bytes<double, CT>());
  for (int it = xcd_remap(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const BItem I = items[it];
    const BProb& P = probs[I.prob];
    if (qiter >= 0 && qiter >= P.q) continue;
    if (qr_step_skipped(P, step, qiter)) continue;
    double* T = which == 2 ? P.T2 : P.T1;
    skinny_tile<double, false, 1, CT>(T, P.LP, which == 2 ? P.n : P.m, 0, P.LP, P.Rinv, P.LP, I.base, 1,
                                      nullptr, T, P.LP, nullptr, Xs, red, 1);  // R^{-1} is upper triangular
  }
}

// Lift: U64 = Q1 U~ (which = 1) or V64 = Q2 V~ (which = 2), one 64-row tile per item.
template <int CT>
__global__ void __launch_bounds__(256, 2)
k_blift(const BProb* __restrict__ probs, const BItem* __restrict__ items, int nitems, int which) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  double* Xs = reinterpret_cast<double*>(lds);
  double* red = reinterpret_cast<double*>(lds + xs_bytes<double, CT>());
  for (int it = xcd_remap(blockIdx.x, gridDim.x); it < nitems; it += gridDim.x) {
    const BItem I = items[it];
    const BProb& P = probs[I.prob];
    skinny_tile<double, false, 1, CT>(which == 2 ? P.T2 : P.T1, P.LP, which == 2 ? P.n : P.m, 0, P.LP,
                                      which == 2 ? P.Vt : P.Ut, P.KP, I.base, 1, nullptr,
                                      which == 2 ? P.V64 : P.U64, P.KP, nullptr, Xs, red);
  }
}

// Result records, the skinny operand (Omega's padding columns must be zero),
// the padded core factors and the norm slots of every problem.
template <typename TA>
__global__ void __launch_bounds__(256) k_bclear(const BProb* __restrict__ probs) {
  const BProb& P = probs[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i0 == 0) {
    P.info->a_fro = 0.0;
    P.info->err_fro = 0.0;
    P.info->err_fro_explicit = -1.0;
    P.info->sweeps = 0;
    P.info->flags = 0;
    P.info->a_noise_rel = 0.0;
    *P.skip3 = 1;
  }
  TA* Xc = reinterpret_cast<TA*>(P.Xc);
  for (int64_t i = i0; i < P.n * P.LP; i += stride) Xc[i] = TA(0);
  for (int64_t i = i0; i < (int64_t)P.LP * P.KP; i += stride) {
    P.Ut[i] = 0.0;
    P.Vt[i] = 0.0;
  }
  for (int64_t i = i0; i < P.ntile1; i += stride) P.normp[i] = 0.0;
}

// Skinny operand of the next pass: Q (T1 or T2, FP64) in A's type.
template <typename TA>
__global__ void __launch_bounds__(256) k_bcast(const BProb* __restrict__ probs, int which, int qiter) {
  const BProb& P = probs[blockIdx.y];
  if (qiter >= 0 && qiter >= P.q) return;
  const double* Q = which == 2 ? P.T2 : P.T1;
  const int64_t tot = (which == 2 ? P.n : P.m) * P.LP;
  TA* Xc = reinterpret_cast<TA*>(P.Xc);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (int64_t)gridDim.x * 256)
    Xc[i] = TA(Q[i]);
}

__global__ void __launch_bounds__(kSmallThreads) k_bchol(const BProb* __restrict__ probs,
                                                         const int32_t* __restrict__ order, int which, int mode,
                                                         int qiter) {
  extern __shared__ double sm[];
  const BProb& P = probs[order[blockIdx.x]];
  if (qiter >= 0 && qiter >= P.q) return;
  const int nparts = which == 2 ? P.gch_n : P.gch_m;
  const int64_t rows = which == 2 ? P.n : P.m;
  if (mode == 1 && qr_step_skipped(P, 1, qiter)) return;
  chol_inv_body(P.gpart, nparts, (int64_t)P.LP * P.LP, P.LP, P.l, rows, mode, P.Rinv, P.skip3, P.info, sm);
}

// One workgroup per problem; the row-block count follows the problem's l.
template <bool V_LDS>
__global__ void __launch_bounds__(kJacThreads) k_bjacobi(const BProb* __restrict__ probs,
                                                          const int32_t* __restrict__ order, int max_sweeps) {
  extern __shared__ double sm[];
  const BProb& P = probs[order[blockIdx.x]];
  const double tol2 = (double)P.l * 0x1p-104;
#define SOR_BJAC(R)                                                                                          \
  case R:                                                                                                    \
    jacobi_body<V_LDS, true, R>(P.gpart, P.gch_m, (int64_t)P.LP * P.LP, P.LP, P.l, P.k, max_sweeps, tol2,   \
                                P.Ut, P.S, P.Vt, P.KP, P.Vg, P.info, sm);                                    \
    break;
  switch (jac_nrb(P.l)) {
    SOR_BJAC(1) SOR_BJAC(2) SOR_BJAC(4) SOR_BJAC(6) SOR_BJAC(8) SOR_BJAC(10) SOR_BJAC(13) SOR_BJAC(16)
    default: break;
  }
#undef SOR_BJAC
}

// Sign convention: the largest-|.| entry of each U column (lowest row on
// ties) is made positive, V's column flipped with it. Stage 1: per row block.
__global__ void __launch_bounds__(256) k_bcolmax(const BProb* __restrict__ probs) {
  const BProb& P = probs[blockIdx.y];
  if ((int)blockIdx.x >= P.sblocks) return;
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int64_t rpb = (P.m + P.sblocks - 1) / P.sblocks;
  const int64_t r0 = (int64_t)blockIdx.x * rpb, r1 = min(P.m, r0 + rpb);
  const int sub = threadIdx.x / 64;
  for (int c0 = 0; c0 < P.k; c0 += 64) {
    const int c = c0 + (threadIdx.x % 64);
    double best = -1.0;
    int64_t bidx = -1;
    if (c < P.k)
      for (int64_t r = r0 + sub; r < r1; r += 4) {
        const double v = fabs(P.U64[r * P.KP + c]);
        if (v > best) { best = v; bidx = r; }
      }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    if (sub == 0 && c < P.k) {
      for (int t = 1; t < 4; ++t) {
        const double v = bv[threadIdx.x + 64 * t];
        const int64_t ix = bi[threadIdx.x + 64 * t];
        if (ix < 0) continue;
        if (bidx < 0 || v > best || (v == best && ix < bidx)) { best = v; bidx = ix; }
      }
      P.pval[(int64_t)blockIdx.x * P.KP + c] = best;
      P.pidx[(int64_t)blockIdx.x * P.KP + c] = bidx;
    }
    __syncthreads();
  }
}

// Stage 2: per column, over the row blocks.
__global__ void __launch_bounds__(64) k_bsigns(const BProb* __restrict__ probs) {
  const BProb& P = probs[blockIdx.y];
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= P.k) return;
  double best = -1.0;
  int64_t bidx = -1;
  for (int b = 0; b < P.sblocks; ++b) {
    const double v = P.pval[(int64_t)b * P.KP + c];
    const int64_t ix = P.pidx[(int64_t)b * P.KP + c];
    if (ix < 0) continue;
    if (bidx < 0 || v > best || (v == best && ix < bidx)) { best = v; bidx = ix; }
  }
  P.sgn[c] = (bidx >= 0 && P.U64[bidx * P.KP + c] < 0.0) ? -1.0 : 1.0;
}

// Signed, truncated factors into the caller's U (m x k) and V (n x k).
__global__ void __launch_bounds__(256) k_bout(const BProb* __restrict__ probs) {
  const BProb& P = probs[blockIdx.y];
  const int64_t nu = P.m * P.k, nv = P.n * P.k;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nu + nv; i += (int64_t)gridDim.x * 256) {
    if (i < nu) {
      const int64_t r = i / P.k;
      const int c = (int)(i % P.k);
      P.U[r * P.ldu + c] = P.sgn[c] * P.U64[r * P.KP + c];
    } else {
      const int64_t j = i - nu;
      const int64_t r = j / P.k;
      const int c = (int)(j % P.k);
      P.V[r * P.ldv + c] = P.sgn[c] * P.V64[r * P.KP + c];
    }
  }
}

// ||A||_F and the error identity sqrt(||A||_F^2 - sum s_j^2) / ||A||_F (Th. 2).
__global__ void __launch_bounds__(256) k_bfinal(const BProb* __restrict__ probs) {
  const BProb& P = probs[blockIdx.x];
  __shared__ double part[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < P.ntile1; i += 256) a += P.normp[i];
  part[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double a2 = part[0];
    double s2 = 0.0;
    for (int j = 0; j < P.k; ++j) s2 += P.S[j] * P.S[j];
    P.info->a_fro = sqrt(a2);
    if (!(a2 - a2 == 0.0)) atomicOr(&P.info->flags, kFlagNonFinite);
    P.info->err_fro = a2 > 0.0 ? sqrt(fmax(a2 - s2, 0.0)) / sqrt(a2) : 0.0;
  }
}

// ------------------------------------------------------------------ host side

struct Cfg {
  int rt = 1;       // passes over A: 64 rt output rows per tile
  int grid = 1024;  // persistent workgroups
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace
}  // namespace sor

using namespace sor;

struct sorsvd_batch {
  int count = 0;
  int a_type = 0;
  int es = 4;
  int max_sweeps = 40;
  int max_q = 0;
  int max_l = 0, max_k = 0, max_sblocks = 0;
  int64_t max_elems = 0, max_omega = 0;
  std::vector<BProb> probs;              // device addresses filled in by upload
  std::vector<OmegaJob> omega;
  std::vector<size_t> off_prob;          // start of each problem's region
  // work lists [mode][rt - 1][CT - 1]; rt only varies for passes over A; CT = LP / 16
  // (KP / 16 for the lifts): one launch per non-empty list
  std::vector<BItem> items[M_COUNT][2][8];
  // problems by descending l (the cost of the one-workgroup steps grows as
  // l^3): workgroup i of those launches takes problem order[i], so that the
  // largest start first
  std::vector<int32_t> order;
  size_t off_table = 0, off_omega = 0, off_order = 0, off_items[M_COUNT][2][8] = {}, total = 0;
  Cfg cfg[3];                            // passes: sketch, orbit, projection
  bool uploaded = false;
  // side streams of the CT groups of a step and their fork / join events
  // (made at the first run, on the device current then)
  mutable hipStream_t aux[8] = {};
  mutable hipEvent_t ev_fork = nullptr, ev_join[8] = {};
  mutable bool forked = false;
  ~sorsvd_batch() {
    for (int c = 0; c < 8; ++c) {
      if (aux[c]) hipStreamDestroy(aux[c]);
      if (ev_join[c]) hipEventDestroy(ev_join[c]);
    }
    if (ev_fork) hipEventDestroy(ev_fork);
  }
};

namespace {

void build_items(sorsvd_batch* b) {
  std::vector<std::pair<double, BItem>> tmp[8];
  auto flush = [&](std::vector<BItem>* dst) {
    for (int c = 0; c < 8; ++c) {
      std::stable_sort(tmp[c].begin(), tmp[c].end(),
                       [](const auto& x, const auto& y) { return x.first > y.first; });
      dst[c].clear();
      for (auto& t : tmp[c]) dst[c].push_back(t.second);
      tmp[c].clear();
    }
  };
  for (int r = 0; r < 2; ++r) {
    const int rt = r + 1;
    for (int mode : {M_SKETCH, M_ORBIT, M_PROJ}) {
      for (int i = 0; i < b->count; ++i) {
        const BProb& P = b->probs[i];
        const int64_t rows = mode == M_ORBIT ? P.n : P.m;
        const int64_t K = mode == M_ORBIT ? P.m : P.n;
        const int64_t tiles = (rows + 64 * rt - 1) / (64 * rt);
        for (int64_t t = 0; t < tiles; ++t)
          tmp[P.LP / kTile - 1].push_back({(double)K * P.LP, BItem{i, (int32_t)t, t * 64 * rt}});
      }
      flush(b->items[mode][r]);
    }
  }
  for (int mode : {M_GRAM1, M_GRAM2, M_PGRAM}) {
    for (int i = 0; i < b->count; ++i) {
      const BProb& P = b->probs[i];
      const int gch = mode == M_GRAM2 ? P.gch_n : P.gch_m;
      const int64_t rows = mode == M_GRAM2 ? P.n : P.m;
      for (int c = 0; c < gch; ++c) {
        const double len = (double)std::min<int64_t>(kGramRows, rows - (int64_t)c * kGramRows);
        for (int h = 0; h * 64 < P.LP; ++h)
          tmp[P.LP / kTile - 1].push_back({len * P.LP * std::min(64, P.LP - 64 * h), BItem{i, c, 64 * h}});
      }
    }
    flush(b->items[mode][0]);
  }
  for (int mode : {M_APPLY1, M_APPLY2, M_LIFTU, M_LIFTV}) {
    for (int i = 0; i < b->count; ++i) {
      const BProb& P = b->probs[i];
      const int64_t rows = (mode == M_APPLY2 || mode == M_LIFTV) ? P.n : P.m;
      const int64_t tiles = (rows + 63) / 64;
      const int ct = (mode >= M_LIFTU ? P.KP : P.LP) / kTile;
      for (int64_t t = 0; t < tiles; ++t)
        tmp[ct - 1].push_back({(double)P.LP * ct * kTile, BItem{i, (int32_t)t, t * 64}});
    }
    flush(b->items[mode][0]);
  }
}

#define SORSVD_TRY(expr)                      \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return SORSVD_EHIP; \
  } while (0)

const BProb* dev_table(const sorsvd_batch* b, void* ws) {
  return reinterpret_cast<const BProb*>((char*)ws + b->off_table);
}

#define SORSVD_CT_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

const BItem* dev_items(const sorsvd_batch* b, void* ws, int mode, int r, int c) {
  return reinterpret_cast<const BItem*>((char*)ws + b->off_items[mode][r][c]);
}

// The launches of the CT groups of one step are independent (disjoint
// problems): the first non-empty group runs on the call's stream, the others
// on side streams forked from it and joined back before the step ends, so
// that their tails overlap. Under stream capture this records a fork / join
// of graph nodes. Per problem the arithmetic is the same as on one stream.
struct GroupFork {
  const sorsvd_batch* b;
  hipStream_t st;
  int ngroups = 0, used = 0;
  bool joined[8] = {};
  hipError_t err = hipSuccess;
  GroupFork(const sorsvd_batch* bb, hipStream_t s, int ng) : b(bb), st(s), ngroups(ng) {
    if (ngroups > 1) err = hipEventRecord(b->ev_fork, st);
  }
  hipStream_t stream(int ci) {
    if (ngroups <= 1 || used++ == 0) return st;
    if (err == hipSuccess) err = hipStreamWaitEvent(b->aux[ci], b->ev_fork, 0);
    joined[ci] = true;
    return b->aux[ci];
  }
  hipError_t join() {
    for (int c = 0; c < 8 && err == hipSuccess; ++c)
      if (joined[c]) {
        err = hipEventRecord(b->ev_join[c], b->aux[c]);
        if (err == hipSuccess) err = hipStreamWaitEvent(st, b->ev_join[c], 0);
      }
    return err;
  }
};

int nonempty_groups(const sorsvd_batch* b, int mode, int r) {
  int n = 0;
  for (int ci = 0; ci < 8; ++ci) n += b->items[mode][r][ci].empty() ? 0 : 1;
  return n;
}

hipError_t make_fork_streams(const sorsvd_batch* b) {
  if (b->forked) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  for (int c = 0; c < 8 && e == hipSuccess; ++c) {
    e = hipStreamCreateWithFlags(&b->aux[c], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join[c], hipEventDisableTiming);
  }
  if (e == hipSuccess) b->forked = true;
  return e;
}

// One pass over A of every problem (one launch per CT group). timed: bracket
// the launches with the library's pass-timing events (when timing is on).
template <typename TA>
int launch_pass(const sorsvd_batch* b, void* ws, int mode, int qiter, const Cfg& c, bool timed, hipStream_t st) {
  if (b->a_type == SORSVD_DIAG) {  // A = diag(sigma): one element-wise launch per LP group
    GroupFork fk(b, st, nonempty_groups(b, mode, 0));
    for (int ci = 0; ci < 8; ++ci) {
      const int n = (int)b->items[mode][0][ci].size();
      if (n == 0) continue;
      hipLaunchKernelGGL(k_bdiag, dim3((unsigned)std::min(2048, n)), dim3(256), 0, fk.stream(ci), dev_table(b, ws),
                         dev_items(b, ws, mode, 0, ci), n, mode, qiter, (mode == M_SKETCH && qiter < 0) ? 1 : 0);
      SORSVD_TRY(hipGetLastError());
    }
    SORSVD_TRY(fk.join());
    return SORSVD_OK;
  }
  // FP64 tiles are 64 rows only (128-row FP64 tiles do not fit the registers)
  const int rt = sizeof(TA) == 8 ? 1 : c.rt;
  const int r = rt - 1;
  const int want_norm = (mode == M_SKETCH && qiter < 0) ? 1 : 0;
  hipEvent_t e1 = nullptr;
  if (timed) {
    double bytes = 0.0, flops = 0.0;
    for (const BProb& P : b->probs)
      if (qiter < 0 || qiter < P.q) {
        bytes += (double)P.m * P.n * b->es;
        flops += 2.0 * P.m * P.n * P.l;
      }
    e1 = pass_timer_begin(st, bytes, flops);
  }
  GroupFork fk(b, st, nonempty_groups(b, mode, r));
  for (int ci = 0; ci < 8; ++ci) {
    const int n = (int)b->items[mode][r][ci].size();
    if (n == 0) continue;
    const dim3 grid((unsigned)std::min(c.grid, n));
    const BItem* it = dev_items(b, ws, mode, r, ci);
    const BProb* probs = dev_table(b, ws);
    const bool tn = mode == M_ORBIT;
    const hipStream_t gs = fk.stream(ci);
    switch ((ci + 1) * 4 + (tn ? 2 : 0) + (rt - 1)) {
#define SORSVD_LP(C)                                                                                          \
  case C * 4 + 0:                                                                                             \
    hipLaunchKernelGGL((k_bpass<TA, false, 1, C>), grid, dim3(256), (tile_lds<TA, C>()), gs, probs, it, n, mode, qiter,   \
                       want_norm);                                                                            \
    break;                                                                                                    \
  case C * 4 + 1:                                                                                             \
    hipLaunchKernelGGL((k_bpass<TA, false, sizeof(TA) == 8 ? 1 : 2, C>), grid, dim3(256), (tile_lds<TA, C>()), gs, probs, \
                       it, n, mode, qiter, want_norm);                                                        \
    break;                                                                                                    \
  case C * 4 + 2:                                                                                             \
    hipLaunchKernelGGL((k_bpass<TA, true, 1, C>), grid, dim3(256), (tile_lds<TA, C>()), gs, probs, it, n, mode, qiter, 0); \
    break;                                                                                                    \
  case C * 4 + 3:                                                                                             \
    hipLaunchKernelGGL((k_bpass<TA, true, sizeof(TA) == 8 ? 1 : 2, C>), grid, dim3(256), (tile_lds<TA, C>()), gs, probs,  \
                       it, n, mode, qiter, 0);                                                                \
    break;
      SORSVD_CT_CASES(SORSVD_LP)
#undef SORSVD_LP
    }
    SORSVD_TRY(hipGetLastError());
  }
  SORSVD_TRY(fk.join());
  if (e1) SORSVD_TRY(hipEventRecord(e1, st));
  return SORSVD_OK;
}

// mode: M_GRAM1 / M_GRAM2 / M_PGRAM, M_APPLY1 / M_APPLY2, M_LIFTU / M_LIFTV.
int launch_f64(const sorsvd_batch* b, void* ws, int mode, int qiter, int step, hipStream_t st) {
  const BProb* probs = dev_table(b, ws);
  GroupFork fk(b, st, nonempty_groups(b, mode, 0));
  for (int ci = 0; ci < 8; ++ci) {
    const int n = (int)b->items[mode][0][ci].size();
    if (n == 0) continue;
    const hipStream_t gs = fk.stream(ci);
    const dim3 grid((unsigned)std::min(2048, n));
    const BItem* it = dev_items(b, ws, mode, 0, ci);
    if (mode == M_GRAM1 || mode == M_GRAM2 || mode == M_PGRAM) {
      switch (ci + 1) {
#define SORSVD_LP(C)                                                                                                \
  case C:                                                                                                           \
    hipLaunchKernelGGL(k_bgram<C>, grid, dim3(256), (tile_lds<double, C>()), gs, probs, it, n, mode, qiter, step);              \
    break;
        SORSVD_CT_CASES(SORSVD_LP)
#undef SORSVD_LP
      }
    } else if (mode == M_APPLY1 || mode == M_APPLY2) {
      const int which = mode == M_APPLY2 ? 2 : 1;
      switch (ci + 1) {
#define SORSVD_LP(C)                                                                                                \
  case C:                                                                                                           \
    hipLaunchKernelGGL(k_bapply<C>, grid, dim3(256), (tile_lds<double, C>()), gs, probs, it, n, which, qiter, step);            \
    break;
        SORSVD_CT_CASES(SORSVD_LP)
#undef SORSVD_LP
      }
    } else {
      const int which = mode == M_LIFTV ? 2 : 1;
      switch (ci + 1) {
#define SORSVD_LP(C)                                                                                                \
  case C:                                                                                                           \
    hipLaunchKernelGGL(k_blift<C>, grid, dim3(256), (tile_lds<double, C>()), gs, probs, it, n, which);                           \
    break;
        SORSVD_CT_CASES(SORSVD_LP)
#undef SORSVD_LP
      }
    }
    SORSVD_TRY(hipGetLastError());
  }
  SORSVD_TRY(fk.join());
  return SORSVD_OK;
}

template <typename TA>
int run_batch(const sorsvd_batch* b, void* ws, bool timed, hipStream_t st) {
  const BProb* probs = dev_table(b, ws);
  const int32_t* order = reinterpret_cast<const int32_t*>((char*)ws + b->off_order);
  const unsigned np = (unsigned)b->count;
  const dim3 g2((unsigned)std::max<int64_t>(1, (b->max_elems + kElemsPerBlock - 1) / kElemsPerBlock), np);
  const size_t chol_shm = chol_lds(b->max_l);
  int rc;
  SORSVD_TRY(make_fork_streams(b));

  hipLaunchKernelGGL((k_bclear<TA>), g2, dim3(256), 0, st, probs);
  SORSVD_TRY(hipGetLastError());
  // Omega (Alg. 3 / Alg. 4 step 1) of every problem, in the compute type.
  SORSVD_TRY(launch_omega_batch(reinterpret_cast<const OmegaJob*>((char*)ws + b->off_omega), b->count,
                                b->max_omega, b->a_type == SORSVD_F32 ? 1 : 0, st));

  // Cholesky QR, repeated (CholQR2 + the conditional shifted third step).
  auto tsqr = [&](int which, int qiter) -> int {
    const int gmode = which == 2 ? M_GRAM2 : M_GRAM1;
    const int amode = which == 2 ? M_APPLY2 : M_APPLY1;
    for (int it = 0; it < 3; ++it) {
      int r;
      if ((r = launch_f64(b, ws, gmode, qiter, it, st))) return r;
      hipLaunchKernelGGL(k_bchol, dim3(np), dim3(kSmallThreads), chol_shm, st, probs, order, which, it, qiter);
      SORSVD_TRY(hipGetLastError());
      if ((r = launch_f64(b, ws, amode, qiter, it, st))) return r;
    }
    return SORSVD_OK;
  };
  auto cast = [&](int which, int qiter) -> int {
    hipLaunchKernelGGL((k_bcast<TA>), g2, dim3(256), 0, st, probs, which, qiter);
    SORSVD_TRY(hipGetLastError());
    return SORSVD_OK;
  };

  // T1 = A Omega (eq. T1) with ||A||_F^2 on the way; Q1 = qr(T1);
  // T2 = A^T Q1 (eq. AT1); Q2 = qr(T2).
  if ((rc = launch_pass<TA>(b, ws, M_SKETCH, -1, b->cfg[0], timed, st))) return rc;
  if ((rc = tsqr(1, -1))) return rc;
  if ((rc = cast(1, -1))) return rc;
  if ((rc = launch_pass<TA>(b, ws, M_ORBIT, -1, b->cfg[1], timed, st))) return rc;
  if ((rc = tsqr(2, -1))) return rc;
  // power steps (Alg. 4), each problem its own q
  for (int q = 0; q < b->max_q; ++q) {
    if ((rc = cast(2, q))) return rc;
    if ((rc = launch_pass<TA>(b, ws, M_SKETCH, q, b->cfg[0], timed, st))) return rc;
    if ((rc = tsqr(1, q))) return rc;
    if ((rc = cast(1, q))) return rc;
    if ((rc = launch_pass<TA>(b, ws, M_ORBIT, q, b->cfg[1], timed, st))) return rc;
    if ((rc = tsqr(2, q))) return rc;
  }
  // M = Q1^T (A Q2) (eq. M)
  if ((rc = cast(2, -1))) return rc;
  if ((rc = launch_pass<TA>(b, ws, M_PROJ, -1, b->cfg[2], timed, st))) return rc;
  if ((rc = launch_f64(b, ws, M_PGRAM, -1, 0, st))) return rc;
  // core SVD, truncated to k (Alg. 3 step 6)
  // (the layout of each problem follows its own l. With V in LDS a smaller
  // problem may take the padded V layout, which can need more than the
  // largest problem's unpadded one: LDS is sized for the largest need)
  bool v_lds = false;
  size_t jshm = jacobi_lds(b->max_l, true, &v_lds);
  if (v_lds)
    for (const BProb& P : b->probs) {
      bool vl = false;
      jshm = std::max(jshm, jacobi_lds(P.l, true, &vl));
    }
  if (v_lds)
    hipLaunchKernelGGL(k_bjacobi<true>, dim3(np), dim3(kJacThreads), jshm, st, probs, order, b->max_sweeps);
  else
    hipLaunchKernelGGL(k_bjacobi<false>, dim3(np), dim3(kJacThreads), jshm, st, probs, order, b->max_sweeps);
  SORSVD_TRY(hipGetLastError());
  // lift (Alg. 3 step 7) and the sign convention
  if ((rc = launch_f64(b, ws, M_LIFTU, -1, 0, st))) return rc;
  if ((rc = launch_f64(b, ws, M_LIFTV, -1, 0, st))) return rc;
  hipLaunchKernelGGL(k_bcolmax, dim3((unsigned)b->max_sblocks, np), dim3(256), 0, st, probs);
  hipLaunchKernelGGL(k_bsigns, dim3((unsigned)((b->max_k + 63) / 64), np), dim3(64), 0, st, probs);
  hipLaunchKernelGGL(k_bout, g2, dim3(256), 0, st, probs);
  hipLaunchKernelGGL(k_bfinal, dim3(np), dim3(256), 0, st, probs);
  SORSVD_TRY(hipGetLastError());
  return SORSVD_OK;
}

int run_any(const sorsvd_batch* b, void* ws, bool timed, hipStream_t st) {
  return b->a_type == SORSVD_F32 ? run_batch<float>(b, ws, timed, st) : run_batch<double>(b, ws, timed, st);
}

std::string tune_key(const sorsvd_batch* b) {
  double work = 0.0;
  for (const auto& P : b->probs) work += (double)P.m * P.n * P.LP;
  char buf[128];
  std::snprintf(buf, sizeof(buf), "t%d_c%d_w%.6e", b->a_type, b->count, work);
  return buf;
}

// Tuning cache: text lines "key rt grid rt grid rt grid" (sketch, orbit,
// projection) in the file named by SORSVD_TUNE_CACHE, if set.
bool tune_cache_load(sorsvd_batch* b) {
  const char* path = std::getenv("SORSVD_TUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char key[128];
  int v[6];
  bool found = false;
  const std::string want = tune_key(b);
  while (std::fscanf(f, "%127s %d %d %d %d %d %d", key, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) == 7) {
    if (want != key) continue;
    bool ok = true;
    for (int i = 0; i < 3; ++i) ok = ok && (v[2 * i] == 1 || (v[2 * i] == 2 && b->a_type == SORSVD_F32)) && v[2 * i + 1] >= 1;
    if (!ok) continue;
    for (int i = 0; i < 3; ++i) {
      b->cfg[i].rt = v[2 * i];
      b->cfg[i].grid = v[2 * i + 1];
    }
    found = true;
  }
  std::fclose(f);
  return found;
}

void tune_cache_store(const sorsvd_batch* b) {
  const char* path = std::getenv("SORSVD_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d %d %d\n", tune_key(b).c_str(), b->cfg[0].rt, b->cfg[0].grid, b->cfg[1].rt,
               b->cfg[1].grid, b->cfg[2].rt, b->cfg[2].grid);
  std::fclose(f);
}

}  // namespace

extern "C" {

int sorsvd_batch_create(int32_t count, const sorsvd_problem* probs, int32_t a_type, const sorsvd_opts* opts,
                        sorsvd_batch** out, size_t* ws_bytes) {
  if (!out || !ws_bytes || !probs || count < 1 || count > kMaxBatch) return SORSVD_EINVAL;
  *out = nullptr;
  *ws_bytes = 0;
  if (a_type != SORSVD_F32 && a_type != SORSVD_F64 && a_type != SORSVD_DIAG) return SORSVD_EUNSUPPORTED;
  if (opts && (opts->refine || opts->residual || opts->split || opts->tile || opts->l || opts->pass_efficient ||
               opts->col_exp))
    return SORSVD_EUNSUPPORTED;
  sorsvd_batch* b = new sorsvd_batch();
  b->count = count;
  b->a_type = a_type;
  b->es = a_type == SORSVD_F32 ? 4 : 8;
  b->max_sweeps = (opts && opts->max_sweeps > 0) ? opts->max_sweeps : 40;
  b->probs.resize(count);
  b->omega.resize(count);
  b->off_prob.resize(count);
  for (int i = 0; i < count; ++i) {
    const sorsvd_problem& u = probs[i];
    const int64_t l = u.l > 0 ? u.l : u.k;
    const bool diag = a_type == SORSVD_DIAG;
    const bool bad = !u.A || !u.U || !u.S || !u.V || u.m < 1 || u.n < 1 || u.k < 1 || u.q < 0 || l < u.k ||
                     l > std::min(u.m, u.n) || (!diag && u.lda < u.n) || (diag && u.m != u.n) ||
                     u.ldu < u.k || u.ldv < u.k;
    if (bad || round_up(l, kTile) > kMaxBatchLP || u.m > INT32_MAX || u.n > INT32_MAX) {
      delete b;
      return bad ? SORSVD_EINVAL : SORSVD_EUNSUPPORTED;
    }
    BProb& P = b->probs[i];
    std::memset(&P, 0, sizeof(P));
    P.m = u.m;
    P.n = u.n;
    P.k = (int)u.k;
    P.l = (int)l;
    P.q = u.q;
    P.LP = (int)round_up(l, kTile);
    P.KP = (int)round_up(u.k, kTile);
    P.A = u.A;
    P.lda = u.lda;
    P.U = u.U;
    P.ldu = u.ldu;
    P.S = u.S;
    P.V = u.V;
    P.ldv = u.ldv;
    P.vec_ok = ((u.lda * b->es) % 16 == 0) && (((uintptr_t)u.A) % 16 == 0);
    P.gch_m = (int)ceil_div(u.m, kGramRows);
    P.gch_n = (int)ceil_div(u.n, kGramRows);
    P.ntile1 = (int)ceil_div(u.m, 64);
    P.sblocks = (int)std::min<int64_t>(64, ceil_div(u.m, 256));
    b->omega[i] = OmegaJob{u.seed, u.n, l, P.LP, nullptr};
    b->max_q = std::max(b->max_q, (int)u.q);
    b->max_l = std::max(b->max_l, P.l);
    b->max_k = std::max(b->max_k, P.k);
    b->max_sblocks = std::max(b->max_sblocks, P.sblocks);
    b->max_elems = std::max<int64_t>({b->max_elems, std::max(u.m, u.n) * P.LP, (u.m + u.n) * P.k});
    b->max_omega = std::max<int64_t>(b->max_omega, u.n * l);
  }
  build_items(b);
  b->order.resize(count);
  for (int i = 0; i < count; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int32_t x, int32_t y) { return b->probs[x].l > b->probs[y].l; });
  size_t off = 0;
  b->off_table = off;
  off += align256(sizeof(BProb) * count);
  b->off_omega = off;
  off += align256(sizeof(OmegaJob) * count);
  b->off_order = off;
  off += align256(sizeof(int32_t) * count);
  for (int mode = 0; mode < M_COUNT; ++mode)
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 8; ++c) {
        b->off_items[mode][r][c] = off;
        off += align256(sizeof(BItem) * b->items[mode][r][c].size());
      }
  for (int i = 0; i < count; ++i) {
    const BProb& P = b->probs[i];
    b->off_prob[i] = off;
    const size_t rows = (size_t)std::max(P.m, P.n), LP = P.LP, KP = P.KP;
    off += align256(rows * LP * b->es);                                 // Xc
    off += 2 * align256(P.m * LP * 8) + align256(P.m * KP * 8);         // T1, W, U64
    off += align256(P.n * LP * 8) + align256(P.n * KP * 8);             // T2, V64
    off += align256(LP * LP * 8) + align256(LP * jac_vg_ld(P.l) * 8);  // Rinv, Vg
    off += 2 * align256(LP * KP * 8);                                   // Ut, Vt
    off += align256((size_t)std::max(P.gch_m, P.gch_n) * LP * LP * 8);  // gpart
    off += align256((size_t)P.ntile1 * 8);                              // normp
    off += 2 * align256((size_t)P.sblocks * KP * 8) + align256(KP * 8); // pval, pidx, sgn
    off += 2 * 256;                                                     // skip3, info
  }
  b->total = off;
  tune_cache_load(b);
  *out = b;
  *ws_bytes = b->total;
  return SORSVD_OK;
}

int sorsvd_batch_upload(sorsvd_batch* b, void* ws, size_t ws_bytes, void* stream) {
  if (!b || !ws) return SORSVD_EINVAL;
  if (ws_bytes < b->total) return SORSVD_EWORKSPACE;
  if (((uintptr_t)ws) % 256) return SORSVD_EINVAL;
  char* base = (char*)ws;
  for (int i = 0; i < b->count; ++i) {
    BProb& P = b->probs[i];
    char* p = base + b->off_prob[i];
    auto take = [&](size_t bytes) {
      char* r = p;
      p += align256(bytes);
      return r;
    };
    const size_t rows = (size_t)std::max(P.m, P.n), LP = P.LP, KP = P.KP;
    P.Xc = take(rows * LP * b->es);
    P.T1 = (double*)take(P.m * LP * 8);
    P.W = (double*)take(P.m * LP * 8);
    P.U64 = (double*)take(P.m * KP * 8);
    P.T2 = (double*)take(P.n * LP * 8);
    P.V64 = (double*)take(P.n * KP * 8);
    P.Rinv = (double*)take(LP * LP * 8);
    P.Vg = (double*)take(LP * jac_vg_ld(P.l) * 8);
    P.Ut = (double*)take(LP * KP * 8);
    P.Vt = (double*)take(LP * KP * 8);
    P.gpart = (double*)take((size_t)std::max(P.gch_m, P.gch_n) * LP * LP * 8);
    P.normp = (double*)take((size_t)P.ntile1 * 8);
    P.pval = (double*)take((size_t)P.sblocks * KP * 8);
    P.pidx = (int64_t*)take((size_t)P.sblocks * KP * 8);
    P.sgn = (double*)take(KP * 8);
    P.skip3 = (int*)take(256);
    P.info = (DevInfo*)take(256);
    b->omega[i].out = P.Xc;
  }
  hipStream_t st = (hipStream_t)stream;
  SORSVD_TRY(hipMemcpyAsync(base + b->off_table, b->probs.data(), sizeof(BProb) * b->count,
                            hipMemcpyHostToDevice, st));
  SORSVD_TRY(hipMemcpyAsync(base + b->off_omega, b->omega.data(), sizeof(OmegaJob) * b->count,
                            hipMemcpyHostToDevice, st));
  SORSVD_TRY(hipMemcpyAsync(base + b->off_order, b->order.data(), sizeof(int32_t) * b->count,
                            hipMemcpyHostToDevice, st));
  for (int mode = 0; mode < M_COUNT; ++mode)
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 8; ++c) {
        const auto& v = b->items[mode][r][c];
        if (!v.empty())
          SORSVD_TRY(hipMemcpyAsync(base + b->off_items[mode][r][c], v.data(), sizeof(BItem) * v.size(),
                                    hipMemcpyHostToDevice, st));
      }
  SORSVD_TRY(hipStreamSynchronize(st));
  b->uploaded = true;
  return SORSVD_OK;
}

int sorsvd_batch_run(const sorsvd_batch* b, void* ws, void* stream) {
  if (!b || !ws || !b->uploaded) return SORSVD_EINVAL;
  return run_any(b, ws, true, (hipStream_t)stream);
}

int sorsvd_batch_get_config(const sorsvd_batch* b, int32_t* config) {
  if (!b || !config) return SORSVD_EINVAL;
  for (int i = 0; i < 3; ++i) {
    config[2 * i] = b->cfg[i].rt;
    config[2 * i + 1] = b->cfg[i].grid;
  }
  return SORSVD_OK;
}

int sorsvd_batch_set_config(sorsvd_batch* b, const int32_t* config) {
  if (!b || !config) return SORSVD_EINVAL;
  const int max_rt = b->a_type == SORSVD_F32 ? 2 : 1;
  for (int i = 0; i < 3; ++i)
    if (config[2 * i] < 1 || config[2 * i] > max_rt || config[2 * i + 1] < 1) return SORSVD_EINVAL;
  for (int i = 0; i < 3; ++i) {
    b->cfg[i].rt = config[2 * i];
    b->cfg[i].grid = config[2 * i + 1];
  }
  return SORSVD_OK;
}

int sorsvd_batch_autotune(sorsvd_batch* b, void* ws, void* stream, int32_t* config_out) {
  if (!b || !ws || !b->uploaded) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  int rc = run_any(b, ws, false, st);  // leaves valid skinny operands behind
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return SORSVD_EHIP;
  }
  const int modes[3] = {M_SKETCH, M_ORBIT, M_PROJ};
  for (int mi = 0; mi < 3 && rc == SORSVD_OK; ++mi) {
    float best = 1e30f;
    Cfg bestc = b->cfg[mi];
    for (int rt = 1; rt <= (b->a_type == SORSVD_F32 ? 2 : 1); ++rt)
      for (int grid : {256, 512, 1024, 2048, 4096}) {
        const Cfg c{rt, grid};
        float tot = 0.f;
        for (int rep = 0; rep < 4 && rc == SORSVD_OK; ++rep) {
          if (hipEventRecord(e0, st) != hipSuccess) { rc = SORSVD_EHIP; break; }
          rc = b->a_type == SORSVD_F32 ? launch_pass<float>(b, ws, modes[mi], -1, c, false, st)
                                       : launch_pass<double>(b, ws, modes[mi], -1, c, false, st);
          if (rc) break;
          float ms = 0.f;
          if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
              hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = SORSVD_EHIP;
            break;
          }
          if (rep > 0) tot += ms;  // the first repetition warms caches and code
        }
        if (rc) break;
        if (tot < best) {
          best = tot;
          bestc = c;
        }
      }
    b->cfg[mi] = bestc;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  tune_cache_store(b);
  if (config_out) sorsvd_batch_get_config(b, config_out);
  // the timing launches overwrote intermediate results: leave a complete run behind
  return run_any(b, ws, false, st);
}

int sorsvd_batch_read_info(const sorsvd_batch* b, sorsvd_info* out, void* stream) {
  if (!b || !out || !b->uploaded) return SORSVD_EINVAL;
  SORSVD_TRY(hipStreamSynchronize((hipStream_t)stream));
  for (int i = 0; i < b->count; ++i)
    SORSVD_TRY(hipMemcpy(&out[i], b->probs[i].info, sizeof(sorsvd_info), hipMemcpyDeviceToHost));
  return SORSVD_OK;
}

int sorsvd_batch_graph(const sorsvd_batch* b, void* ws, void** graph_exec) {
  if (!b || !ws || !graph_exec || !b->uploaded) return SORSVD_EINVAL;
  *graph_exec = nullptr;
  hipStream_t cs;
  SORSVD_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    hipStreamDestroy(cs);
    return SORSVD_EHIP;
  }
  hipGraph_t graph = nullptr;
  const int rc = run_any(b, ws, false, cs);  // no timing events inside a graph
  const hipError_t e = hipStreamEndCapture(cs, &graph);
  hipStreamDestroy(cs);
  if (rc || e != hipSuccess) {
    if (graph) hipGraphDestroy(graph);
    return rc ? rc : SORSVD_EHIP;
  }
  hipGraphExec_t exec;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (ei != hipSuccess) return SORSVD_EHIP;
  *graph_exec = (void*)exec;
  return SORSVD_OK;
}

int sorsvd_graph_launch(void* graph_exec, void* stream) {
  if (!graph_exec) return SORSVD_EINVAL;
  SORSVD_TRY(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
  return SORSVD_OK;
}

int sorsvd_graph_destroy(void* graph_exec) {
  if (!graph_exec) return SORSVD_EINVAL;
  SORSVD_TRY(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
  return SORSVD_OK;
}

int32_t sorsvd_batch_count(const sorsvd_batch* b) { return b ? b->count : 0; }

void sorsvd_batch_destroy(sorsvd_batch* b) { delete b; }

}  // extern "C"
