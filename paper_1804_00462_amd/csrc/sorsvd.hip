// Host orchestration and C ABI of the SOR-SVD library (see include/sorsvd.h).
//
// One call enqueues, on the caller's stream, the sequence of Sec. III:
//   Omega (Philox) -> T1 = A Omega -> QR -> T2 = A^T Q1 -> QR
//   -> q x {T1 = A Q2 -> QR -> T2 = A^T Q1 -> QR}
//   -> M = Q1^T (A Q2) -> core SVD -> U = Q1 U~_k, V = Q2 V~_k -> signs, error.
// Nothing is allocated and nothing waits for the device; argument checks come
// first and fail before any launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/sorsvd.h"
#include "half16.hpp"

namespace sor {

// gemm.hip
hipError_t launch_skinny_f64(bool trans, const double* A, int64_t lda, int64_t OUT, int64_t K,
                             const double* X, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                             double* P, double* normp, const int* skipflag, hipStream_t st,
                             double* Tout = nullptr, int tri = 0, int ncb = 1);
hipError_t launch_skinny_f32(bool trans, const float* A, int64_t lda, int64_t OUT, int64_t K,
                             const float* X, int64_t ldx, int LP, int64_t kchunk, int nsplit,
                             float* P, double* normp, const int* skipflag, hipStream_t st,
                             double* Tout = nullptr, int ncb = 1);
hipError_t launch_apply_tri_blocks(double* T, int64_t rows, int LP, const double* Z, int ncb,
                                   const int* skipflag, hipStream_t st);
hipError_t launch_reduce_f64(const double* P, int64_t OUT, int LP, int nsplit, double* out,
                             int64_t ldo, int ncols, hipStream_t st, const int* skipflag = nullptr);
hipError_t launch_reduce_f32(const float* P, int64_t OUT, int LP, int nsplit, double* out,
                             int64_t ldo, int ncols, hipStream_t st);
hipError_t launch_pack_f64(const double* src, int64_t rows, int cols, int64_t lds, double* dst,
                           int LP, hipStream_t st);
hipError_t launch_pack_f32(const double* src, int64_t rows, int cols, int64_t lds, float* dst,
                           int LP, hipStream_t st);
hipError_t launch_cast_f32(const double* Q, int64_t n_elem, float* Xc, hipStream_t st);
hipError_t launch_zero_lower(double* R, int l, hipStream_t st);
hipError_t launch_diag_pass(const double* sigma, int64_t n, int LP, const double* X, double* T, double* normp,
                            int nparts, hipStream_t st);
int skinny_rows_per_block(int a_type, int64_t OUT);
int skinny_slots(int a_type, bool trans, int LP);
// rpca.hip
int rpca_stat_blocks(int64_t m, int64_t n);
int64_t rpca_step_blocks(int64_t m, int64_t n);
hipError_t launch_rpca_stats(const double* X, int64_t ldx, int64_t m, int64_t n, double* psq, double* pmax,
                             hipStream_t st);
hipError_t launch_rpca_init(const double* X, int64_t ldx, int64_t m, int64_t n, double inv_j, double inv_mu,
                            double* S, int64_t lds, double* Y, double* W, hipStream_t st);
hipError_t launch_rpca_step(const double* X, int64_t ldx, int64_t m, int64_t n, const double* U, const double* V,
                            const double* z, int l, double inv_mu, double thr_s, double mu, double inv_mu_next,
                            double* L, double* S, int64_t ld, double* Y, double* W, double* rpart,
                            hipStream_t st);
hipError_t launch_rpca_nnz(const double* S, int64_t ld, int64_t m, int64_t n, double* pcount, hipStream_t st);
int skinny_step(int a_type);
// gemm_bf16.hip (16-bit passes; FP16 instantiations in gemm_f16.hip)
hipError_t launch_h16_pass(int fmt, bool trans, const uint16_t* A, int64_t lda, int64_t OUT, int64_t K,
                           const uint16_t* XT, int64_t ldx, int LP, int64_t kchunk, int nsplit, int ncb, float* P,
                           double* normp, double* Tout, int fold, int rt, const H16Scale* sc, const int* cexp,
                           hipStream_t st);
int h16_slots(int fmt, bool trans, int rt, int LP);
int bf16_step(bool trans, int rt, int LP);
hipError_t launch_cast_h16_t(int fmt, const double* Q, int64_t rows, int LP, int ncb, int64_t ldt, int permute,
                             int with_lo, uint16_t* QT, const H16Scale* sc, const int* cexp, hipStream_t st);
hipError_t launch_reduce_fold(const float* P, int64_t OUT, int LP2, int nsplit, double* out,
                              int64_t ldo, int ncols, int cbw, hipStream_t st);
hipError_t launch_reduce_h16(bool trans, const float* P, int64_t OUT, int LP2, int nsplit, double* out, int64_t ldo,
                             int ncols, int fold, int cbw, const H16Scale* sc, const int* cexp, hipStream_t st);
hipError_t launch_h16_scale(const int* cexp, int64_t n, int shift, H16Scale* sc, int* flags, hipStream_t st);
// philox.hip
hipError_t launch_omega_bf16_t(uint64_t seed, int64_t rows, int64_t cols, bf16_t* out,
                               int64_t ldx, hipStream_t st);
hipError_t launch_omega_f16_t(uint64_t seed, int64_t rows, int64_t cols, uint16_t* out, int64_t ldx,
                              const H16Scale* sc, const int* cexp, hipStream_t st);
hipError_t launch_omega_f64_colmajor(uint64_t seed, uint64_t stream_id, uint64_t word2,
                                     int64_t rows, int64_t cols, double* out, hipStream_t st);
hipError_t launch_omega_rowmajor_f64(uint64_t seed, int64_t rows, int64_t cols, double* out,
                                     int64_t ldx, hipStream_t st);
hipError_t launch_omega_rowmajor_f32(uint64_t seed, int64_t rows, int64_t cols, float* out,
                                     int64_t ldx, hipStream_t st);
// small.hip
hipError_t launch_chol_inv(const double* G, int LP, int l, int64_t rows, int mode, double* Rinv,
                           int* skip3, void* info, hipStream_t st);
hipError_t launch_jacobi(const double* M, int LP, int l, int k, int max_sweeps, double* Ut,
                         double* sv, double* Vt, int ldk, double* Vg, void* info, hipStream_t st,
                         bool want_v = true, double tol = 0.0, void* rlog = nullptr);
size_t jacobi_log_bytes(int l, int max_sweeps);
bool jacobi_uses_log(int l);
hipError_t launch_signfix(const double* U64, int64_t m, const double* V64, int64_t n, int ld, int k,
                          double* pval, int64_t* pidx, int nblocks_max, double* sgn, void* U,
                          int64_t ldu, void* V, int64_t ldv, hipStream_t st, int out_f32);
hipError_t launch_finalize(const double* normp, int nparts, const double* sv, int k, void* info,
                           hipStream_t st);
hipError_t launch_info_init(void* info, hipStream_t st);
// mlp.hip
int mlp_param_count();
size_t mlp_work_floats(int B);
hipError_t launch_mlp_forward(const float* P, const float* X, int B, float* Y, float* work, hipStream_t st);
hipError_t launch_mlp_backward(const float* P, const float* X, const float* T, int B, float* G, float* loss,
                               float* work, hipStream_t st);
hipError_t launch_mlp_adam(float* P, const float* G, float* M, float* V, int64_t step, float lr, float beta1,
                           float beta2, float eps, hipStream_t st);
hipError_t launch_features(const double* sv, int l, float* feat, hipStream_t st);
// residual.hip
int64_t residual_parts(int64_t m, int64_t n);
size_t residual_ws_bytes(int a_type, int64_t m, int64_t n, int KP);
hipError_t launch_residual(int a_type, const void* A, int64_t lda, int64_t m, int64_t n, const double* U,
                           int64_t ldu, const double* S, const double* V, int64_t ldv, int k, int KP, double* part,
                           void* info, hipStream_t st, const int* cexp);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t st);
hipError_t launch_sub_f64(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t rows, int cols,
                          double* C, int64_t ldc, hipStream_t st);
hipError_t launch_transpose_f64(const double* src, int64_t lds, int64_t rows, int cols, double* dst, int64_t ldd,
                                hipStream_t st);
// wide.hip (l > 128)
size_t chol_wide_bytes(int LP);
hipError_t launch_chol_wide(double* G, int LP, int l, int64_t rows, int mode, double* Z, int* skip3, void* info,
                            void* scratch, hipStream_t st);
size_t jacobi_wide_bytes(int l);
hipError_t launch_jacobi_wide(const double* M, int LPm, int l, int k, int max_sweeps, double* Ut, double* sv,
                              double* Vt, int ldk, void* scratch, void* info, hipStream_t st, double tol,
                              bool trans = false);

namespace {

constexpr int kMaxLP = 1024;       // widest sketch
constexpr int kNarrowLP = 128;     // widest sketch of the one-workgroup QR factor and core SVD
constexpr int kBlk = 128;          // widest column block of the pass kernels
constexpr int kProbeL = 128;       // sketch width of the (k, q) predictor's probe
constexpr int kWideSweeps = 16;    // default sweep cap of the core SVD of the method for l > 128
constexpr int kWideMaxSweeps = 64; // largest sweep cap for l > 128
constexpr int kSignBlocks = 1024;  // max row blocks of the sign search
constexpr size_t kAlign = 256;

// Padded width of a skinny operand of w columns and its column blocks: up to
// 128 columns one block (w rounded up to 16); wider operands ncb blocks of
// equal width, a multiple of 16 up to 128 (the padding columns are zero).
void width_blocks(int64_t w, int64_t* WP, int* ncb) {
  const int64_t w16 = round_up(w, kTile);
  if (w16 <= kBlk) {
    *WP = w16;
    *ncb = 1;
    return;
  }
  const int64_t nb = ceil_div(w16, kBlk);
  const int64_t ct = ceil_div(w16 / kTile, nb);
  *WP = nb * ct * kTile;
  *ncb = (int)nb;
}

struct Split {
  int64_t kchunk = 0;
  int nsplit = 1;
};

// Split of a contraction of length K for OUT output rows: about `target`
// workgroups (enough to fill 256 CUs several times over by default), each
// split at least `min_steps` steps long, and partial sums no larger than
// 1/`part_div` of the bytes of the streamed operand. slots > 0 (workgroups the device holds at once): among
// the splits from half of that count up to it, the one whose workgroups fill
// whole waves of `slots` best (a last, mostly empty wave of workgroups costs
// as much as a full one); never more splits than without it, so a workspace
// sized without a device also fits.
Split choose_split(int64_t OUT, int64_t K, int rows_per_block, int KS, int LP, int es_a,
                   int acc_bytes, int forced, int min_steps = 8, int part_div = 8, int slots = 0,
                   int64_t target = 2048, int ncb = 1) {
  Split sp;
  if (K <= 0) { sp.kchunk = KS; sp.nsplit = 1; return sp; }
  // (ncb column blocks: workgroups per split = row tiles x ncb)
  const int64_t tiles = std::max<int64_t>(1, ceil_div(OUT, rows_per_block)) * ncb;
  int64_t s = std::max<int64_t>(1, ceil_div(target, tiles));
  s = std::min<int64_t>(s, std::max<int64_t>(1, K / ((int64_t)min_steps * KS)));
  s = std::min<int64_t>(s, std::max<int64_t>(1, (K * es_a) / ((int64_t)part_div * LP * acc_bytes)));
  if (forced > 0) s = forced;
  sp.kchunk = round_up(ceil_div(K, s), KS);
  sp.nsplit = (int)ceil_div(K, sp.kchunk);
  if (forced <= 0 && slots > 0 && sp.nsplit > 1) {
    double best = -1.0;
    Split pick = sp;
    for (int64_t c = sp.nsplit; c >= std::max<int64_t>(1, sp.nsplit / 2); --c) {
      Split t;
      t.kchunk = round_up(ceil_div(K, c), KS);
      t.nsplit = (int)ceil_div(K, t.kchunk);
      const int64_t W = tiles * t.nsplit;
      const double fill = (double)W / (double)(ceil_div(W, slots) * slots);
      if (fill > best + 1e-9) {
        best = fill;
        pick = t;
      }
    }
    sp = pick;
  }
  return sp;
}

struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    const size_t off = total;
    total += round_up((int64_t)bytes, kAlign);
    return off;
  }
};

struct Plan {
  int a_type;
  int64_t m, n, k, l, LP, KP;
  int ncb, ncbk;  // column blocks of the LP-wide and KP-wide operands (1 up to 128 columns)
  int64_t CB;     // width of one LP column block
  bool wide;      // l > 128: blocked QR factor and core SVD (wide.hip)
  int q;
  int es;
  int max_sweeps;
  int fmt;        // 16-bit A: kFmtBF16 / kFmtF16; -1 otherwise
  const int* cexp;  // FP16 A: column exponents (A = A_stored diag(2^-e_j)), or null
  int refine;     // 16-bit A: projection pass with Q2 = hi + lo
  int residual;   // explicit residual pass after the lift
  int pass_eff;   // M from the last orbit product (no projection pass)
  int literal;    // Alg. 4 as printed: no QR between the products
  int out_f32;    // U and V written as FP32
  int64_t ldt;    // 16-bit A: leading dimension of the transposed skinny operands
  int rt_nn, rt_tn, rt_proj;  // 16-bit A: rows (NN) / columns (TN) of A per workgroup = 64 rt
  Split projb;    // 16-bit A: split of the refinement projection pass
  int rt_tnb;     // 16-bit A, pass_eff with refine: the last orbit product with Q1 = hi + lo
  Split tnb;      // ... and its split
  Split nn, tn, gram_m, gram_n, proj;
  int nn_blocks;
  size_t off_info, off_xc, off_t1, off_t2, off_w, off_u64, off_v64, off_p, off_normp;
  size_t off_g, off_rinv, off_m, off_ut, off_vt, off_vg, off_pval, off_pidx, off_sgn, off_skip, off_res;
  size_t off_t2p;  // pass_eff: the last orbit product before its QR (n x LP FP64)
  size_t off_hsc;  // FP16 A: the operand scale record (H16Scale)
  size_t off_rlog; // core SVD: rotation log from which V is rebuilt (0: V kept in the Jacobi kernel)
  size_t off_wchol, off_wjac;  // wide: scratch of the blocked factor and of the blocked Jacobi
  size_t total;
};

int elem_size(int t) { return (t == SORSVD_F64 || t == SORSVD_DIAG) ? 8 : (t == SORSVD_F32 ? 4 : 2); }

// FP16 skinny operands are lifted by 2^12 (orthonormal entries |q| <= 1 and
// Gaussian draws below 7 stay under 2^15), which keeps all but entries below
// 2^-26 out of the FP16 subnormal range.
constexpr int kF16Shift = 12;

size_t partial_bytes(int64_t OUT, int64_t LP, const Split& s, int acc) {
  return (size_t)s.nsplit * OUT * LP * acc;
}

int make_plan(int64_t m, int64_t n, int64_t k, int32_t q, int32_t a_type, const sorsvd_opts* o,
              Plan* p) {
  if (a_type != SORSVD_F64 && a_type != SORSVD_F32 && a_type != SORSVD_BF16 && a_type != SORSVD_DIAG &&
      a_type != SORSVD_F16)
    return SORSVD_EINVAL;
  const bool h16 = a_type == SORSVD_BF16 || a_type == SORSVD_F16;
  if (o && o->col_exp && a_type != SORSVD_F16) return SORSVD_EUNSUPPORTED;
  if (m < 1 || n < 1 || k < 1 || q < 0) return SORSVD_EINVAL;
  if (a_type == SORSVD_DIAG && m != n) return SORSVD_EINVAL;
  if (a_type == SORSVD_DIAG && o && o->residual) return SORSVD_EUNSUPPORTED;
  const int64_t l = (o && o->l > 0) ? o->l : k;
  if (k > l || l > std::min(m, n)) return SORSVD_EINVAL;
  if (l > kMaxLP) return SORSVD_EUNSUPPORTED;
  int64_t LP, KP;
  int ncb, ncbk;
  width_blocks(l, &LP, &ncb);
  width_blocks(k, &KP, &ncbk);
  p->a_type = a_type; p->m = m; p->n = n; p->k = k; p->l = l; p->LP = LP; p->KP = KP; p->q = q;
  p->ncb = ncb; p->ncbk = ncbk; p->CB = LP / ncb;
  p->wide = l > kNarrowLP;
  p->es = elem_size(a_type);
  p->max_sweeps = (o && o->max_sweeps > 0) ? o->max_sweeps : (p->wide ? kWideSweeps : 40);
  if (p->wide && p->max_sweeps > kWideMaxSweeps) return SORSVD_EINVAL;
  const int CB = (int)p->CB;
  p->fmt = a_type == SORSVD_BF16 ? kFmtBF16 : (a_type == SORSVD_F16 ? kFmtF16 : -1);
  p->cexp = (o && a_type == SORSVD_F16) ? (const int*)o->col_exp : nullptr;
  p->refine = (h16 && o && o->refine) ? 1 : 0;
  p->residual = (o && o->residual) ? 1 : 0;
  p->pass_eff = (o && o->pass_efficient) ? 1 : 0;
  p->literal = (o && o->literal) ? 1 : 0;
  p->out_f32 = (o && o->out_f32) ? 1 : 0;
  if (p->literal && (p->pass_eff || a_type == SORSVD_DIAG)) return SORSVD_EUNSUPPORTED;
  p->ldt = round_up(std::max(m, n), 128) + 128;  // room for the last step's over-read
  const int forced = o ? o->split : 0;
  const int ks = skinny_step(a_type == SORSVD_DIAG ? SORSVD_F64 : a_type);
  const int acc = (a_type == SORSVD_F64 || a_type == SORSVD_DIAG) ? 8 : 4;
  // 16-bit tiles (an opts override serves tuning sweeps). A X: 128 rows per
  // workgroup balances the row run each load reads against the re-read of
  // the skinny block (measured at 200000 x 4000: 4.1 TB/s at 128 rows, 3.8 at
  // 256, and the same order for the 2l-column refinement pass). A^T Y: 256
  // columns when l <= 64.
  const int tile_opt = o ? o->tile : 0;
  p->rt_nn = tile_opt ? tile_opt : 2;
  p->rt_tn = tile_opt ? tile_opt : (CB <= 64 ? 4 : 2);
  p->rt_proj = tile_opt ? std::min(tile_opt, p->refine && CB > 32 ? 2 : 4) : 2;
  const int t64 = a_type == SORSVD_DIAG ? SORSVD_F64 : a_type;
  const int rpb_m = h16 ? 64 * p->rt_nn : skinny_rows_per_block(t64, m);
  const int rpb_n = h16 ? 64 * p->rt_tn : skinny_rows_per_block(t64, n);
  const int ks_nn = h16 ? bf16_step(false, p->rt_nn, CB) : ks;
  const int ks_tn = h16 ? bf16_step(true, p->rt_tn, CB) : ks;
  const bool skinny_pass = a_type == SORSVD_F32 || a_type == SORSVD_F64;
  const int tcode = a_type == SORSVD_F32 ? 1 : 0;
  // 16-bit passes aim at one wave of resident workgroups (see A^T Y below)
  const int nn_slots = skinny_pass ? skinny_slots(tcode, false, CB)
                                   : (h16 ? h16_slots(p->fmt, false, p->rt_nn, CB) : 0);
  p->nn = choose_split(m, n, rpb_m, ks_nn, (int)LP, p->es, acc, forced, 8, 8, nn_slots,
                       (h16 && nn_slots > 0) ? nn_slots : 2048, ncb);
  // 16-bit A^T Y: a workgroup streams 64 rt whole columns of A with its
  // contraction rows staged through LDS, so one wave of resident workgroups
  // already keeps HBM busy; more splits only add partial sums to write and
  // reduce (measured at 200000 x 4000, l = 64: 6.2 TB/s at 512 workgroups,
  // 5.0 TB/s at 2000)
  const int tn_slots = skinny_pass ? skinny_slots(tcode, true, CB)
                                   : (h16 ? h16_slots(p->fmt, true, p->rt_tn, CB) : 0);
  p->tn = choose_split(n, m, rpb_n, ks_tn, (int)LP, p->es, acc, forced, 8, 8, tn_slots,
                       (h16 && tn_slots > 0) ? tn_slots : 2048, ncb);
  // pass-efficient core matrix on 16-bit A with refinement: the last orbit
  // product takes [Q1 hi | Q1 lo] (2 LP columns), so that T2 = A^T Q1, from
  // which M is formed, carries Q1 to ~2^-17 as the projection pass would
  p->rt_tnb = tile_opt ? tile_opt : 2;
  if (h16 && p->pass_eff && p->refine) {
    const int tnb_slots = h16_slots(p->fmt, true, p->rt_tnb, 2 * CB);
    p->tnb = choose_split(n, m, 64 * p->rt_tnb, bf16_step(true, p->rt_tnb, 2 * CB), 2 * (int)LP, p->es, acc,
                          forced, 8, 8, tnb_slots, tnb_slots > 0 ? tnb_slots : 2048, ncb);
  }
  const int LPproj = (int)LP * (p->refine ? 2 : 1);
  const int CBproj = CB * (p->refine ? 2 : 1);
  const int proj_slots = h16 ? h16_slots(p->fmt, false, p->rt_proj, CBproj) : 0;
  p->projb = choose_split(m, n, 64 * p->rt_proj, h16 ? bf16_step(false, p->rt_proj, CBproj) : 128, LPproj, p->es,
                          acc, forced, 8, 8, proj_slots, proj_slots > 0 ? proj_slots : 2048, ncb);
  // l x l products over a tall FP64 operand: many short splits, with partial
  // sums up to the size of the operand (at 20000 x 100 the Gram product then
  // runs 250 workgroups instead of 158: 26 -> 21 us)
  const int ks64 = skinny_step(SORSVD_F64);
  const int rpbg = skinny_rows_per_block(SORSVD_F64, LP);
  // one wave of resident workgroups: more splits only add partial sums
  // (l x l FP64 each) to write and reduce
  const int gslots = skinny_slots(SORSVD_F64, true, CB);
  const int64_t gtarget = gslots > 0 ? gslots : 2048;
  p->gram_m = choose_split(LP, m, rpbg, ks64, (int)LP, 8, 8, 0, 4, 1, gslots, gtarget, ncb);
  p->gram_n = choose_split(LP, n, rpbg, ks64, (int)LP, 8, 8, 0, 4, 1, gslots, gtarget, ncb);
  p->proj = p->gram_m;
  p->nn_blocks = (int)(ceil_div(m, rpb_m) * p->nn.nsplit);
  if (h16 && p->rt_nn != 1 && p->rt_nn != 2 && p->rt_nn != 4) return SORSVD_EINVAL;

  Layout L;
  p->off_info = L.take(256);
  const int64_t rows = std::max(m, n);
  p->off_xc = h16 ? L.take((size_t)2 * LP * p->ldt * 2) : L.take((size_t)rows * LP * p->es);
  p->off_t1 = L.take((size_t)m * LP * 8);
  p->off_t2 = L.take((size_t)n * LP * 8);
  p->off_w = L.take((size_t)m * LP * 8);
  p->off_u64 = L.take((size_t)m * KP * 8);
  p->off_v64 = L.take((size_t)n * KP * 8);
  size_t pb = 0;
  pb = std::max(pb, partial_bytes(m, LP, p->nn, acc));
  pb = std::max(pb, partial_bytes(m, (p->refine ? 2 : 1) * LP, p->projb, acc));
  pb = std::max(pb, partial_bytes(n, LP, p->tn, acc));
  if (h16 && p->pass_eff && p->refine) pb = std::max(pb, partial_bytes(n, 2 * LP, p->tnb, acc));
  pb = std::max(pb, partial_bytes(LP, LP, p->gram_m, 8));
  pb = std::max(pb, partial_bytes(LP, LP, p->gram_n, 8));
  p->off_p = L.take(pb);
  p->off_normp = L.take((size_t)std::max(p->nn_blocks, 1) * 8);
  p->off_g = L.take((size_t)LP * LP * 8);
  p->off_rinv = L.take((size_t)LP * LP * 8);
  p->off_m = L.take((size_t)LP * LP * 8);
  p->off_ut = L.take((size_t)LP * KP * 8);
  p->off_vt = L.take((size_t)LP * KP * 8);
  p->off_vg = L.take(p->wide ? 0 : (size_t)LP * kNarrowLP * 8);  // Jacobi's V: l columns of up to 128 padded rows
  p->off_pval = L.take((size_t)kSignBlocks * KP * 8);
  p->off_pidx = L.take((size_t)kSignBlocks * KP * 8);
  p->off_sgn = L.take((size_t)KP * 8);
  p->off_skip = L.take(64);
  p->off_res = p->residual ? L.take(residual_ws_bytes(a_type == SORSVD_F64 ? 0 : (a_type == SORSVD_F32 ? 1 : (a_type == SORSVD_F16 ? 4 : 2)), m, n, (int)KP)) : 0;
  p->off_t2p = p->pass_eff ? L.take((size_t)n * LP * 8) : 0;
  p->off_hsc = a_type == SORSVD_F16 ? L.take(sizeof(H16Scale)) : 0;
  p->off_rlog = (!p->wide && jacobi_uses_log((int)l)) ? L.take(jacobi_log_bytes((int)l, p->max_sweeps)) : 0;
  p->off_wchol = p->wide ? L.take(chol_wide_bytes((int)LP)) : 0;
  p->off_wjac = p->wide ? L.take(jacobi_wide_bytes((int)l)) : 0;
  p->total = L.total;
  return SORSVD_OK;
}

#define SORSVD_TRY(expr)                          \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return SORSVD_EHIP;     \
  } while (0)

template <typename T> T* at(void* ws, size_t off) { return reinterpret_cast<T*>((char*)ws + off); }

// Cholesky QR of T (rows x LP, FP64, padding columns zero) in place: two
// steps T <- T R^{-1}, the first shifted when T is ill-conditioned, and then
// a third step whose kernels return at once unless the first was shifted.
// A basis that only feeds the next product (final = false: the Q1 and Q2 of
// every power step but the last) takes one step when that step needed no
// shift: its columns are then orthonormal to ~cond(T)^2 u, which is a
// well-conditioned basis of the same span, and only the span enters the next
// product. The bases that form M and the lifted factors take both steps.
// For l > 128 the factor is the blocked one of wide.hip and T R^{-1} is formed
// column block by column block (launch_apply_tri_blocks); the steps are the same.
int tsqr_inplace(const Plan& p, double* T, int64_t rows, const Split& gram, void* ws, hipStream_t st,
                 bool final = true) {
  double* P = at<double>(ws, p.off_p);
  double* G = at<double>(ws, p.off_g);
  double* Rinv = at<double>(ws, p.off_rinv);
  int* skip3 = at<int>(ws, p.off_skip);
  void* info = at<void>(ws, p.off_info);
  const int LP = (int)p.LP;
  for (int it = 0; it < 3; ++it) {
    if (!final && it == 1) continue;
    const int* skip = it == 2 ? skip3 : nullptr;
    SORSVD_TRY(launch_skinny_f64(true, T, LP, LP, rows, T, LP, LP, gram.kchunk, gram.nsplit, P,
                                 nullptr, skip, st, nullptr, 2, p.ncb));  // upper triangle of T^T T
    SORSVD_TRY(launch_reduce_f64(P, LP, LP, gram.nsplit, G, LP, LP, st, skip));
    if (p.wide) {
      SORSVD_TRY(launch_chol_wide(G, LP, (int)p.l, rows, it, Rinv, skip3, info, at<void>(ws, p.off_wchol), st));
      SORSVD_TRY(launch_apply_tri_blocks(T, rows, LP, Rinv, p.ncb, skip, st));
    } else {
      SORSVD_TRY(launch_chol_inv(G, LP, (int)p.l, rows, it, Rinv, skip3, info, st));
      SORSVD_TRY(launch_skinny_f64(false, T, LP, rows, LP, Rinv, LP, LP, LP, 1, T, nullptr, skip, st, nullptr,
                                   true));
    }
  }
  return SORSVD_OK;
}

// Core SVD of M (l x l in an LP-wide buffer) into Ut, S, Vt (l x k, ld KP).
int core_svd(const Plan& p, const double* M, double* Ut, double* S, double* Vt, void* ws, hipStream_t st) {
  void* info = at<void>(ws, p.off_info);
  if (p.wide) {
    SORSVD_TRY(launch_jacobi_wide(M, (int)p.LP, (int)p.l, (int)p.k, p.max_sweeps, Ut, S, Vt, (int)p.KP,
                                  at<void>(ws, p.off_wjac), info, st, 0.0));
  } else {
    SORSVD_TRY(launch_jacobi(M, (int)p.LP, (int)p.l, (int)p.k, p.max_sweeps, Ut, S, Vt, (int)p.KP,
                             at<double>(ws, p.off_vg), info, st, true, 0.0,
                             p.off_rlog ? at<void>(ws, p.off_rlog) : nullptr));
  }
  return SORSVD_OK;
}

// Optional per-launch timing of the pass kernel over A (profiling aid):
// a pair of HIP events is recorded around each launch on the call's stream.
struct PassTimer {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  double bytes = 0.0, flops = 0.0;
};
PassTimer& timer() {
  static PassTimer t;
  return t;
}

// T (OUT x LP, FP64) = A X   (trans = false, X in compute type, K = n)
//                    = A^T Y (trans = true,  Y in compute type, K = m)
int pass(const Plan& p, bool trans, const void* A, int64_t lda, const void* Xc, double* T,
         double* normp, void* ws, hipStream_t st, bool fold = false, bool proj = false) {
  // (trans with fold: the last orbit product of the pass-efficient form, with
  // [Q1 hi | Q1 lo]; its halves are always added by the reduction)
  const int LP = (int)p.LP;
  const int64_t OUT = trans ? p.n : p.m;
  const int64_t K = trans ? p.m : p.n;
  const Split& sp = trans ? p.tn : p.nn;
  PassTimer& tm = timer();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (tm.on) {
    std::lock_guard<std::mutex> g(tm.mu);
    if (tm.used + 2 <= tm.ev.size()) {
      e0 = tm.ev[tm.used];
      e1 = tm.ev[tm.used + 1];
      tm.used += 2;
      tm.bytes += (double)p.m * p.n * p.es;
      tm.flops += 2.0 * p.m * p.n * p.l;
    }
  }
  if (e0) SORSVD_TRY(hipEventRecord(e0, st));
  if (p.a_type == SORSVD_DIAG) {
    SORSVD_TRY(launch_diag_pass((const double*)A, p.n, LP, (const double*)Xc, T, normp, p.nn_blocks, st));
    if (e1) SORSVD_TRY(hipEventRecord(e1, st));
  } else if (p.a_type == SORSVD_F64) {
    double* P = at<double>(ws, p.off_p);
    SORSVD_TRY(launch_skinny_f64(trans, (const double*)A, lda, OUT, K, (const double*)Xc, LP, LP,
                                 sp.kchunk, sp.nsplit, P, normp, nullptr, st, T, false, p.ncb));
    if (e1) SORSVD_TRY(hipEventRecord(e1, st));
    if (sp.nsplit > 1) SORSVD_TRY(launch_reduce_f64(P, OUT, LP, sp.nsplit, T, LP, LP, st));
  } else if (p.a_type == SORSVD_F32) {
    float* P = at<float>(ws, p.off_p);
    SORSVD_TRY(launch_skinny_f32(trans, (const float*)A, lda, OUT, K, (const float*)Xc, LP, LP,
                                 sp.kchunk, sp.nsplit, P, normp, nullptr, st, T, p.ncb));
    if (e1) SORSVD_TRY(hipEventRecord(e1, st));
    if (sp.nsplit > 1) SORSVD_TRY(launch_reduce_f32(P, OUT, LP, sp.nsplit, T, LP, LP, st));
  } else {
    // 16-bit A: Xc is the transposed operand; `fold` = the refinement pass
    // with [Q2 hi | Q2 lo] (2 LP columns) whose two halves are summed. FP16
    // operands carry the scaling of the scale record, undone on T.
    float* P = at<float>(ws, p.off_p);
    const int LPw = fold ? 2 * LP : LP;
    const bool tfold = trans && fold;
    const Split& spb = proj ? p.projb : (tfold ? p.tnb : sp);
    const int rt = proj ? p.rt_proj : (tfold ? p.rt_tnb : (trans ? p.rt_tn : p.rt_nn));
    const H16Scale* sc = p.fmt == kFmtF16 ? at<H16Scale>(ws, p.off_hsc) : nullptr;
    SORSVD_TRY(launch_h16_pass(p.fmt, trans, (const uint16_t*)A, lda, OUT, K, (const uint16_t*)Xc, p.ldt, LPw,
                               spb.kchunk, spb.nsplit, p.ncb, P, normp, tfold ? nullptr : T, fold ? 1 : 0, rt, sc,
                               p.cexp, st));
    if (e1) SORSVD_TRY(hipEventRecord(e1, st));
    if (spb.nsplit > 1 || tfold) {  // with one split the kernel wrote T itself (not the A^T Y kernel with fold)
      if (sc)
        SORSVD_TRY(launch_reduce_h16(trans, P, OUT, LPw, spb.nsplit, T, LP, LP, fold ? 1 : 0, (int)p.CB, sc, p.cexp,
                                     st));
      else if (fold)
        SORSVD_TRY(launch_reduce_fold(P, OUT, LPw, spb.nsplit, T, LP, LP, (int)p.CB, st));
      else
        SORSVD_TRY(launch_reduce_f32(P, OUT, LP, spb.nsplit, T, LP, LP, st));
    }
  }
  return SORSVD_OK;
}

// Skinny operand of the next pass: Q (rows x LP, FP64) in A's compute type.
// 16-bit: transposed, with the contraction permutation for the orbit (TN)
// pass, and with the low part appended for the refinement pass; FP16 also
// scaled (H16Scale).
const void* as_operand(const Plan& p, const double* Q, int64_t rows, void* ws, hipStream_t st, int* rc,
                       bool for_tn = false, bool with_lo = false) {
  *rc = SORSVD_OK;
  if (p.a_type == SORSVD_F64 || p.a_type == SORSVD_DIAG) return Q;
  if (p.fmt >= 0) {
    uint16_t* XT = at<uint16_t>(ws, p.off_xc);
    const H16Scale* sc = p.fmt == kFmtF16 ? at<H16Scale>(ws, p.off_hsc) : nullptr;
    if (launch_cast_h16_t(p.fmt, Q, rows, (int)p.CB, p.ncb, p.ldt, for_tn ? 1 : 0, with_lo ? 1 : 0, XT, sc,
                          for_tn ? nullptr : p.cexp, st) != hipSuccess)
      *rc = SORSVD_EHIP;
    return XT;
  }
  float* Xc = at<float>(ws, p.off_xc);
  if (launch_cast_f32(Q, rows * p.LP, Xc, st) != hipSuccess) *rc = SORSVD_EHIP;
  return Xc;
}

// FP16 A: the operand scale record of this run (min of the column exponents;
// flags bit 3 of the result record when one lies outside +-kMaxColExp).
int h16_setup(const Plan& p, void* ws, hipStream_t st) {
  if (p.fmt != kFmtF16) return SORSVD_OK;
  int* flags = reinterpret_cast<int*>(at<char>(ws, p.off_info) + offsetof(sorsvd_info, flags));
  SORSVD_TRY(launch_h16_scale(p.cexp, p.n, kF16Shift, at<H16Scale>(ws, p.off_hsc), flags, st));
  return SORSVD_OK;
}

// q1 != null: Q1 of the first sketch is given (q1, leading dimension ldq1, at
// least l columns: the leading l columns of an orthonormal basis of a wider
// sketch A Omega' with Omega nested in Omega'), together with the sums of
// squares of A (normp_ext, nparts_ext slots); the first pass and its QR are
// skipped.
int run(const Plan& p, const void* A, int64_t lda, uint64_t seed, void* U, int64_t ldu, double* S,
        void* V, int64_t ldv, void* ws, hipStream_t st, const double* q1 = nullptr, int64_t ldq1 = 0,
        const double* normp_ext = nullptr, int nparts_ext = 0) {
  const int LP = (int)p.LP, KP = (int)p.KP;
  void* info = at<void>(ws, p.off_info);
  double* T1 = at<double>(ws, p.off_t1);
  double* T2 = at<double>(ws, p.off_t2);
  double* W = at<double>(ws, p.off_w);
  double* T2P = p.pass_eff ? at<double>(ws, p.off_t2p) : nullptr;
  double* normp = at<double>(ws, p.off_normp);
  int rc;
  SORSVD_TRY(launch_info_init(info, st));
  if ((rc = h16_setup(p, ws, st))) return rc;

  // Omega, n x l (Alg. 3 / Alg. 4 step 1), straight into the compute-type operand.
  void* Xc = at<void>(ws, p.off_xc);
  if (q1) {
    // nothing to draw
  } else if (p.a_type == SORSVD_F64 || p.a_type == SORSVD_DIAG) {
    SORSVD_TRY(launch_fill((double*)Xc, p.n * LP, 0.0, st));
    SORSVD_TRY(launch_omega_rowmajor_f64(seed, p.n, p.l, (double*)Xc, LP, st));
  } else if (p.a_type == SORSVD_F32) {
    SORSVD_TRY(launch_fill((double*)Xc, (p.n * LP * 4 + 7) / 8, 0.0, st));
    SORSVD_TRY(launch_omega_rowmajor_f32(seed, p.n, p.l, (float*)Xc, LP, st));
  } else {
    SORSVD_TRY(launch_fill((double*)Xc, LP * p.ldt * 2 / 8, 0.0, st));
    if (p.fmt == kFmtF16)
      SORSVD_TRY(launch_omega_f16_t(seed, p.n, p.l, (uint16_t*)Xc, p.ldt, at<H16Scale>(ws, p.off_hsc), p.cexp, st));
    else
      SORSVD_TRY(launch_omega_bf16_t(seed, p.n, p.l, (bf16_t*)Xc, p.ldt, st));
  }

  if (p.literal) {
    // Alg. 4 as printed: T2 <- Omega; q + 1 times {T1 = A T2; T2 = A^T T1};
    // the QRs only at the end
    if ((rc = pass(p, false, A, lda, Xc, T1, normp, ws, st))) return rc;
    for (int it = 0; it <= p.q; ++it) {
      const void* Y = as_operand(p, T1, p.m, ws, st, &rc, true);
      if (rc) return rc;
      if ((rc = pass(p, true, A, lda, Y, T2, nullptr, ws, st))) return rc;
      if (it == p.q) break;
      const void* X = as_operand(p, T2, p.n, ws, st, &rc);
      if (rc) return rc;
      if ((rc = pass(p, false, A, lda, X, T1, nullptr, ws, st))) return rc;
    }
    if ((rc = tsqr_inplace(p, T1, p.m, p.gram_m, ws, st))) return rc;
    if ((rc = tsqr_inplace(p, T2, p.n, p.gram_n, ws, st))) return rc;
  }
  // T1 = A Omega (eq. T1), with ||A||_F^2 accumulated on the way; Q1 = qr(T1).
  if (p.literal) {
    // (done above)
  } else if (q1) {
    SORSVD_TRY(launch_pack_f64(q1, p.m, (int)p.l, ldq1, T1, LP, st));
  } else {
    if ((rc = pass(p, false, A, lda, Xc, T1, normp, ws, st))) return rc;
    if ((rc = tsqr_inplace(p, T1, p.m, p.gram_m, ws, st, p.q == 0))) return rc;
  }
  // T2 = A^T Q1 (eq. AT1; the span of A^T T1 by Lemma 1); Q2 = qr(T2).
  // (the pass-efficient form with refinement splits Q1 into hi + lo for the
  // orbit product that M is formed from)
  const bool pe_lo = p.pass_eff && p.refine;
  if (!p.literal) {
    const void* Y = as_operand(p, T1, p.m, ws, st, &rc, true, pe_lo && p.q == 0);
    if (rc) return rc;
    if ((rc = pass(p, true, A, lda, Y, T2, nullptr, ws, st, pe_lo && p.q == 0))) return rc;
    if (p.pass_eff && p.q == 0) SORSVD_TRY(launch_pack_f64(T2, p.n, LP, LP, T2P, LP, st));
    if ((rc = tsqr_inplace(p, T2, p.n, p.gram_n, ws, st, p.q == 0))) return rc;
  }
  // Power method (Alg. 4 loop), orthonormalising after each product.
  for (int it = 0; !p.literal && it < p.q; ++it) {
    const bool last = it == p.q - 1;
    const void* X = as_operand(p, T2, p.n, ws, st, &rc);
    if (rc) return rc;
    if ((rc = pass(p, false, A, lda, X, T1, nullptr, ws, st))) return rc;
    if ((rc = tsqr_inplace(p, T1, p.m, p.gram_m, ws, st, last))) return rc;
    const void* Y = as_operand(p, T1, p.m, ws, st, &rc, true, pe_lo && last);
    if (rc) return rc;
    if ((rc = pass(p, true, A, lda, Y, T2, nullptr, ws, st, pe_lo && last))) return rc;
    if (p.pass_eff && last) SORSVD_TRY(launch_pack_f64(T2, p.n, LP, LP, T2P, LP, st));
    if ((rc = tsqr_inplace(p, T2, p.n, p.gram_n, ws, st, last))) return rc;
  }
  double* P = at<double>(ws, p.off_p);
  double* M = at<double>(ws, p.off_m);
  if (p.pass_eff) {
    // pass-efficient core matrix (eq. M_approx): Q1^T A = T2^T for the kept
    // T2 = A^T Q1, so Q1^T A Q2 = T2^T Q2 (an FP64 l x l product over n rows)
    SORSVD_TRY(launch_skinny_f64(true, T2P, LP, LP, p.n, T2, LP, LP, p.gram_n.kchunk, p.gram_n.nsplit, P,
                                 nullptr, nullptr, st, nullptr, false, p.ncb));
    SORSVD_TRY(launch_reduce_f64(P, LP, LP, p.gram_n.nsplit, M, LP, LP, st));
  } else {
    // M = Q1^T (A Q2) (eq. M): W = A Q2 in the pass kernel, then the FP64 Q1^T W.
    const void* X = as_operand(p, T2, p.n, ws, st, &rc, false, p.refine != 0);
    if (rc) return rc;
    if ((rc = pass(p, false, A, lda, X, W, nullptr, ws, st, p.refine != 0, true))) return rc;
    SORSVD_TRY(launch_skinny_f64(true, T1, LP, LP, p.m, W, LP, LP, p.proj.kchunk, p.proj.nsplit, P,
                                 nullptr, nullptr, st, nullptr, false, p.ncb));
    SORSVD_TRY(launch_reduce_f64(P, LP, LP, p.proj.nsplit, M, LP, LP, st));
  }

  // Core SVD M = U~ S~ V~^T, truncated to k (Alg. 3 step 6).
  double* Ut = at<double>(ws, p.off_ut);
  double* Vt = at<double>(ws, p.off_vt);
  SORSVD_TRY(launch_fill(Ut, (int64_t)LP * KP, 0.0, st));
  SORSVD_TRY(launch_fill(Vt, (int64_t)LP * KP, 0.0, st));
  if ((rc = core_svd(p, M, Ut, S, Vt, ws, st))) return rc;

  // Lift: U = Q1 U~_k, V = Q2 V~_k (Alg. 3 step 7), then the sign convention.
  double* U64 = at<double>(ws, p.off_u64);
  double* V64 = at<double>(ws, p.off_v64);
  SORSVD_TRY(launch_skinny_f64(false, T1, LP, p.m, LP, Ut, KP, KP, LP, 1, U64, nullptr, nullptr, st, nullptr, false,
                               p.ncbk));
  SORSVD_TRY(launch_skinny_f64(false, T2, LP, p.n, LP, Vt, KP, KP, LP, 1, V64, nullptr, nullptr, st, nullptr, false,
                               p.ncbk));
  SORSVD_TRY(launch_signfix(U64, p.m, V64, p.n, KP, (int)p.k, at<double>(ws, p.off_pval),
                            at<int64_t>(ws, p.off_pidx), kSignBlocks, at<double>(ws, p.off_sgn), U, ldu,
                            V, ldv, st, p.out_f32));
  SORSVD_TRY(launch_finalize(normp_ext ? normp_ext : normp, normp_ext ? nparts_ext : p.nn_blocks, S, (int)p.k,
                             info, st));
  // Error check as one more pass (the identity above is free; this one is
  // exact up to the pass arithmetic, and for BF16 A also measures the
  // rounding of A to BF16).
  // (on the lifted factors before the sign convention: the flips of u_j and
  // v_j cancel in U S V^T, and these stay FP64 whatever the output type)
  if (p.residual)
    SORSVD_TRY(launch_residual(p.a_type, A, lda, p.m, p.n, U64, KP, S, V64, KP, (int)p.k, (int)KP,
                               at<double>(ws, p.off_res), info, st, p.cexp));
  return SORSVD_OK;
}

// Probe of the (k, q) predictor: Y0 = A Omega[:, :l], l = min(128, m, n), the
// same draw as a SOR-SVD with that seed (Omega is nested in its width); the
// singular values of Y0 are those of R in Y0 = Q R; features as in
// launch_features. p: plan with k = l, q = 0.
int probe(const Plan& p, const void* A, int64_t lda, uint64_t seed, float* feat, void* ws, hipStream_t st) {
  const int LP = (int)p.LP, KP = (int)p.KP;
  void* info = at<void>(ws, p.off_info);
  double* T1 = at<double>(ws, p.off_t1);
  double* Wc = at<double>(ws, p.off_w);
  double* normp = at<double>(ws, p.off_normp);
  int rc;
  SORSVD_TRY(launch_info_init(info, st));
  void* Xc = at<void>(ws, p.off_xc);
  if (p.a_type == SORSVD_F64 || p.a_type == SORSVD_DIAG) {
    SORSVD_TRY(launch_fill((double*)Xc, p.n * LP, 0.0, st));
    SORSVD_TRY(launch_omega_rowmajor_f64(seed, p.n, p.l, (double*)Xc, LP, st));
  } else if (p.a_type == SORSVD_F32) {
    SORSVD_TRY(launch_fill((double*)Xc, (p.n * LP * 4 + 7) / 8, 0.0, st));
    SORSVD_TRY(launch_omega_rowmajor_f32(seed, p.n, p.l, (float*)Xc, LP, st));
  } else {
    SORSVD_TRY(launch_fill((double*)Xc, LP * p.ldt * 2 / 8, 0.0, st));
    SORSVD_TRY(launch_omega_bf16_t(seed, p.n, p.l, (bf16_t*)Xc, p.ldt, st));
  }
  if ((rc = pass(p, false, A, lda, Xc, T1, normp, ws, st))) return rc;
  SORSVD_TRY(launch_pack_f64(T1, p.m, LP, LP, Wc, LP, st));
  if ((rc = tsqr_inplace(p, T1, p.m, p.gram_m, ws, st))) return rc;
  // R^T = Y0^T Q: its rows are the columns of R, whose norms fall with the
  // singular values, and one-sided Jacobi on that graded form takes a few
  // sweeps fewer than on R. Only singular values are needed: no V, and the
  // pairs stop at an orthogonality of 1e-8 (values to ~1e-14 relative).
  double* P = at<double>(ws, p.off_p);
  double* G = at<double>(ws, p.off_g);
  SORSVD_TRY(launch_skinny_f64(true, Wc, LP, LP, p.m, T1, LP, LP, p.gram_m.kchunk, p.gram_m.nsplit, P, nullptr,
                               nullptr, st));
  SORSVD_TRY(launch_reduce_f64(P, LP, LP, p.gram_m.nsplit, G, LP, LP, st));
  double* Ut = at<double>(ws, p.off_ut);
  double* sv = at<double>(ws, p.off_sgn);
  SORSVD_TRY(launch_jacobi(G, LP, (int)p.l, (int)p.l, p.max_sweeps, Ut, sv, nullptr, KP, at<double>(ws, p.off_vg),
                           info, st, false, 1e-8));
  SORSVD_TRY(launch_features(sv, (int)p.l, feat, st));
  return SORSVD_OK;
}

}  // namespace

// Timing hook for launches of pass kernels outside this file (the batched
// engine): records the start event and returns the end event to record after
// the launch, or null when timing is off or its capacity is used up.
hipEvent_t pass_timer_begin(hipStream_t st, double bytes, double flops) {
  PassTimer& tm = timer();
  std::lock_guard<std::mutex> g(tm.mu);
  if (!tm.on || tm.used + 2 > tm.ev.size()) return nullptr;
  hipEvent_t e0 = tm.ev[tm.used], e1 = tm.ev[tm.used + 1];
  tm.used += 2;
  tm.bytes += bytes;
  tm.flops += flops;
  if (hipEventRecord(e0, st) != hipSuccess) return nullptr;
  return e1;
}

struct BoundsLayout {
  int64_t LP = 0, RP = 0;
  int ncb = 1;
  Split sp;
  size_t off_om = 0, off_o1 = 0, off_o1t = 0, off_g = 0, off_h1 = 0, off_h = 0, off_p = 0, off_ut = 0, off_vt = 0,
         off_s = 0, off_q = 0, off_r = 0, off_sub = 0, sub_bytes = 0, total = 0;
};

int bounds_layout(int64_t n, int64_t l, int64_t p, BoundsLayout* b) {
  const int64_t r = l - p;
  if (n < 1 || l < 1 || p < 0 || r < 1 || l > n || l > kMaxLP) return SORSVD_EINVAL;
  width_blocks(l, &b->LP, &b->ncb);
  int ncbr;
  width_blocks(r, &b->RP, &ncbr);
  const int64_t LP = b->LP;
  const int ks = skinny_step(SORSVD_F64);
  b->sp = choose_split(LP, n, skinny_rows_per_block(SORSVD_F64, LP), ks, (int)LP, 8, 8, 0, 8, 1, 0, 2048, b->ncb);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up((int64_t)bytes, kAlign);
    return o;
  };
  b->off_om = take((size_t)n * LP * 8);   // Omega, n x LP (zero padding columns)
  b->off_o1 = take((size_t)LP * LP * 8);  // Omega1, r x LP (rows r.. zero)
  b->off_o1t = take((size_t)l * r * 8);   // Omega1^T, l x r
  b->off_g = take((size_t)LP * LP * 8);   // Omega^T Omega
  b->off_h1 = take((size_t)LP * LP * 8);  // Omega1^T Omega1
  b->off_h = take((size_t)l * l * 8);     // Omega2^T Omega2, l x l
  b->off_p = take(partial_bytes(LP, LP, b->sp, 8));
  b->off_ut = take((size_t)l * l * 8);
  b->off_vt = take((size_t)l * l * 8);
  b->off_s = take((size_t)l * 8);
  b->off_q = take((size_t)l * r * 8);
  b->off_r = take((size_t)r * r * 8);
  b->sub_bytes = std::max({sorsvd_step_workspace_bytes(l, r, r, SORSVD_F64),
                           sorsvd_step_workspace_bytes(r, r, r, SORSVD_F64),
                           sorsvd_step_workspace_bytes(l, l, l, SORSVD_F64)});
  if (b->sub_bytes == 0) return SORSVD_EINVAL;
  b->off_sub = take(b->sub_bytes);
  b->total = off;
  return SORSVD_OK;
}

// nu of Th. 6 / Th. 7
double bounds_nu(int64_t n, int64_t l, int64_t p) {
  const double nu1 = std::sqrt((double)(n - l + p)) + std::sqrt((double)l) + 7.0;
  const double nu2 = 4.0 * std::exp(1.0) * std::sqrt((double)l) / (double)(p + 1);
  return nu1 * nu2;
}

}  // namespace sor

using namespace sor;

extern "C" {

size_t sorsvd_workspace_bytes(int64_t m, int64_t n, int64_t k, int32_t q, int32_t a_type,
                              const sorsvd_opts* opts) {
  Plan p;
  if (make_plan(m, n, k, q, a_type, opts, &p) != SORSVD_OK) return 0;
  return p.total;
}

int sorsvd(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, int64_t k, int32_t q,
           uint64_t seed, void* U, int64_t ldu, double* S, void* V, int64_t ldv, void* workspace,
           size_t ws_bytes, void* stream, const sorsvd_opts* opts) {
  Plan p;
  const int rc = make_plan(m, n, k, q, a_type, opts, &p);
  if (rc != SORSVD_OK) return rc;
  if (!A || !U || !S || !V || !workspace) return SORSVD_EINVAL;
  if ((lda < n && a_type != SORSVD_DIAG) || ldu < k || ldv < k) return SORSVD_EINVAL;
  if (ws_bytes < p.total) return SORSVD_EWORKSPACE;
  if (((uintptr_t)workspace) % kAlign) return SORSVD_EINVAL;
  return run(p, A, lda, seed, U, ldu, S, V, ldv, workspace, (hipStream_t)stream);
}

int sorsvd_read_info(const void* workspace, sorsvd_info* out, void* stream) {
  if (!workspace || !out) return SORSVD_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SORSVD_EHIP;
  if (hipMemcpy(out, workspace, sizeof(sorsvd_info), hipMemcpyDeviceToHost) != hipSuccess) return SORSVD_EHIP;
  return SORSVD_OK;
}

int sorsvd_philox_normal(uint64_t seed, uint64_t stream_id, uint64_t word2, int64_t rows,
                         int64_t cols, double* out, void* stream) {
  if (rows < 0 || cols < 0 || (!out && rows * cols > 0)) return SORSVD_EINVAL;
  if (launch_omega_f64_colmajor(seed, stream_id, word2, rows, cols, out, (hipStream_t)stream) != hipSuccess)
    return SORSVD_EHIP;
  return SORSVD_OK;
}

// ------------------------------------------------------------- single steps

size_t sorsvd_step_workspace_bytes(int64_t m, int64_t n, int64_t l, int32_t a_type) {
  sorsvd_opts o;
  std::memset(&o, 0, sizeof(o));
  o.l = l;
  o.refine = (a_type == SORSVD_BF16 || a_type == SORSVD_F16) ? 1 : 0;
  Plan p;
  if (make_plan(m, n, l, 0, a_type, &o, &p) != SORSVD_OK) return 0;
  // room for packed FP64 copies of two skinny operands (QR input copy, projection)
  return p.total + 2 * round_up((int64_t)std::max(m, n) * p.LP * 8, kAlign);
}

static int step_plan(int64_t m, int64_t n, int64_t l, int32_t a_type, size_t ws_bytes, Plan* p) {
  sorsvd_opts o;
  std::memset(&o, 0, sizeof(o));
  o.l = l;
  o.refine = (a_type == SORSVD_BF16 || a_type == SORSVD_F16) ? 1 : 0;  // 16-bit projection: hi + lo split
  const int rc = make_plan(m, n, l, 0, a_type, &o, p);
  if (rc != SORSVD_OK) return rc;
  if (ws_bytes < sorsvd_step_workspace_bytes(m, n, l, a_type)) return SORSVD_EWORKSPACE;
  return SORSVD_OK;
}

static int pack_operand(const Plan& p, const double* src, int64_t rows, int64_t l, void* ws,
                        hipStream_t st, const void** out, bool for_tn = false, bool with_lo = false) {
  if (p.fmt >= 0) {
    double* tmp = at<double>(ws, p.total + round_up(std::max(p.m, p.n) * p.LP * 8, kAlign));
    SORSVD_TRY(launch_pack_f64(src, rows, (int)l, l, tmp, (int)p.LP, st));
    int rc;
    *out = as_operand(p, tmp, rows, ws, st, &rc, for_tn, with_lo);
    return rc;
  }
  if (p.a_type == SORSVD_F64 || p.a_type == SORSVD_DIAG) {
    double* d = at<double>(ws, p.off_xc);
    SORSVD_TRY(launch_pack_f64(src, rows, (int)l, l, d, (int)p.LP, st));
    *out = d;
  } else {
    float* d = at<float>(ws, p.off_xc);
    SORSVD_TRY(launch_pack_f32(src, rows, (int)l, l, d, (int)p.LP, st));
    *out = d;
  }
  return SORSVD_OK;
}

int sorsvd_step_sketch(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n,
                       const double* X, int64_t l, double* T, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int rc = step_plan(m, n, l, a_type, ws_bytes, &p);
  if (rc) return rc;
  if (!A || !X || !T || lda < n) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = h16_setup(p, ws, st))) return rc;
  const void* Xc;
  if ((rc = pack_operand(p, X, n, l, ws, st, &Xc))) return rc;
  double* Tp = at<double>(ws, p.off_t1);
  if ((rc = pass(p, false, A, lda, Xc, Tp, nullptr, ws, st))) return rc;
  SORSVD_TRY(launch_pack_f64(Tp, m, (int)l, p.LP, T, (int)l, st));
  return SORSVD_OK;
}

int sorsvd_step_orbit(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n,
                      const double* Y, int64_t l, double* T, void* ws, size_t ws_bytes, void* stream) {
  Plan p;
  int rc = step_plan(m, n, l, a_type, ws_bytes, &p);
  if (rc) return rc;
  if (!A || !Y || !T || lda < n) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = h16_setup(p, ws, st))) return rc;
  const void* Yc;
  if ((rc = pack_operand(p, Y, m, l, ws, st, &Yc, true))) return rc;
  double* Tp = at<double>(ws, p.off_t2);
  if ((rc = pass(p, true, A, lda, Yc, Tp, nullptr, ws, st))) return rc;
  SORSVD_TRY(launch_pack_f64(Tp, n, (int)l, p.LP, T, (int)l, st));
  return SORSVD_OK;
}

int sorsvd_step_qr(const double* T, int64_t rows, int64_t l, double* Q, double* R, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!T || !Q || !R || l < 1 || rows < l) return SORSVD_EINVAL;
  Plan p;
  int rc = step_plan(rows, l, l, SORSVD_F64, ws_bytes, &p);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const int LP = (int)p.LP;
  double* Tq = at<double>(ws, p.off_t1);
  double* Tc = at<double>(ws, p.total);  // packed copy of the input
  SORSVD_TRY(launch_info_init(at<void>(ws, p.off_info), st));
  SORSVD_TRY(launch_pack_f64(T, rows, (int)l, l, Tq, LP, st));
  SORSVD_TRY(launch_pack_f64(T, rows, (int)l, l, Tc, LP, st));
  if ((rc = tsqr_inplace(p, Tq, rows, p.gram_m, ws, st))) return rc;
  // R = Q^T T (upper triangular up to rounding; the strict lower part is cleared)
  double* P = at<double>(ws, p.off_p);
  double* G = at<double>(ws, p.off_g);
  SORSVD_TRY(launch_skinny_f64(true, Tq, LP, LP, rows, Tc, LP, LP, p.gram_m.kchunk, p.gram_m.nsplit,
                                   P, nullptr, nullptr, st, nullptr, false, p.ncb));
  SORSVD_TRY(launch_reduce_f64(P, LP, LP, p.gram_m.nsplit, G, LP, LP, st));
  SORSVD_TRY(launch_pack_f64(Tq, rows, (int)l, LP, Q, (int)l, st));
  SORSVD_TRY(launch_pack_f64(G, l, (int)l, LP, R, (int)l, st));
  SORSVD_TRY(launch_zero_lower(R, (int)l, st));
  return SORSVD_OK;
}

int sorsvd_step_project(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n,
                        const double* Q1, const double* Q2, int64_t l, double* M, void* ws,
                        size_t ws_bytes, void* stream) {
  Plan p;
  int rc = step_plan(m, n, l, a_type, ws_bytes, &p);
  if (rc) return rc;
  if (!A || !Q1 || !Q2 || !M || lda < n) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int LP = (int)p.LP;
  if ((rc = h16_setup(p, ws, st))) return rc;
  const void* Xc;
  const bool fold = p.fmt >= 0;
  if ((rc = pack_operand(p, Q2, n, l, ws, st, &Xc, false, fold))) return rc;
  double* W = at<double>(ws, p.off_w);
  if ((rc = pass(p, false, A, lda, Xc, W, nullptr, ws, st, fold, true))) return rc;
  double* Q1p = at<double>(ws, p.total);
  SORSVD_TRY(launch_pack_f64(Q1, m, (int)l, l, Q1p, LP, st));
  double* P = at<double>(ws, p.off_p);
  double* Mp = at<double>(ws, p.off_m);
  SORSVD_TRY(launch_skinny_f64(true, Q1p, LP, LP, m, W, LP, LP, p.proj.kchunk, p.proj.nsplit, P,
                                   nullptr, nullptr, st, nullptr, false, p.ncb));
  SORSVD_TRY(launch_reduce_f64(P, LP, LP, p.proj.nsplit, Mp, LP, LP, st));
  SORSVD_TRY(launch_pack_f64(Mp, l, (int)l, LP, M, (int)l, st));
  return SORSVD_OK;
}

int sorsvd_step_core_svd(const double* M, int64_t l, int64_t k, double* Ut, double* s, double* Vt,
                         int32_t max_sweeps, void* ws, size_t ws_bytes, void* stream) {
  if (!M || !Ut || !s || !Vt || l < 1 || k < 1 || k > l) return SORSVD_EINVAL;
  Plan p;
  int rc = step_plan(l, l, l, SORSVD_F64, ws_bytes, &p);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  SORSVD_TRY(launch_info_init(at<void>(ws, p.off_info), st));
  SORSVD_TRY(launch_fill(Ut, l * k, 0.0, st));
  SORSVD_TRY(launch_fill(Vt, l * k, 0.0, st));
  if (p.wide) {
    // A general M (unlike the core matrix of the method, which is R2^T of
    // the last QR step up to rounding) is first factored M = Q R (Cholesky
    // QR); one-sided Jacobi on R^T then needs far fewer sweeps (the QR
    // preconditioning of Drmac and Veselic). With R^T = U' S V'^T,
    // M = (Q V') S U'^T.
    if (max_sweeps > kWideMaxSweeps) return SORSVD_EINVAL;
    const int ms = max_sweeps > 0 ? max_sweeps : 40;
    const int LP = (int)p.LP, KP = (int)p.KP;
    double* Tq = at<double>(ws, p.off_t1);  // M, then Q (l x LP)
    double* Mp = at<double>(ws, p.total);   // M (l x LP)
    double* P = at<double>(ws, p.off_p);
    double* R = at<double>(ws, p.off_m);
    double* Ua = at<double>(ws, p.off_ut);  // U' (l x KP)
    double* Va = at<double>(ws, p.off_vt);  // V' (l x KP)
    double* QV = at<double>(ws, p.off_u64);
    SORSVD_TRY(launch_pack_f64(M, l, (int)l, l, Tq, LP, st));
    SORSVD_TRY(launch_pack_f64(M, l, (int)l, l, Mp, LP, st));
    if ((rc = tsqr_inplace(p, Tq, l, p.gram_m, ws, st))) return rc;
    SORSVD_TRY(launch_skinny_f64(true, Tq, LP, LP, l, Mp, LP, LP, p.gram_m.kchunk, p.gram_m.nsplit, P, nullptr,
                                 nullptr, st, nullptr, false, p.ncb));
    SORSVD_TRY(launch_reduce_f64(P, LP, LP, p.gram_m.nsplit, R, LP, LP, st));
    SORSVD_TRY(launch_fill(Ua, (int64_t)LP * KP, 0.0, st));
    SORSVD_TRY(launch_fill(Va, (int64_t)LP * KP, 0.0, st));
    SORSVD_TRY(launch_jacobi_wide(R, LP, (int)l, (int)k, ms, Ua, s, Va, KP, at<void>(ws, p.off_wjac),
                                  at<void>(ws, p.off_info), st, 0.0, true));
    SORSVD_TRY(launch_skinny_f64(false, Tq, LP, l, LP, Va, KP, KP, LP, 1, QV, nullptr, nullptr, st, nullptr, false,
                                 p.ncbk));
    SORSVD_TRY(launch_pack_f64(QV, l, (int)k, KP, Ut, (int)k, st));
    SORSVD_TRY(launch_pack_f64(Ua, l, (int)k, KP, Vt, (int)k, st));
    return SORSVD_OK;
  }
  const int ms = max_sweeps > 0 ? max_sweeps : 40;
  // the log in the workspace holds p.max_sweeps sweeps
  void* rlog = (p.off_rlog && ms <= p.max_sweeps) ? at<void>(ws, p.off_rlog) : nullptr;
  SORSVD_TRY(launch_jacobi(M, (int)l, (int)l, (int)k, ms, Ut, s, Vt, (int)k, at<double>(ws, p.off_vg),
                           at<void>(ws, p.off_info), st, true, 0.0, rlog));
  return SORSVD_OK;
}

// ------------------------------------------------------------ theorem bounds
//
// Th. 4 - Th. 7 for one draw of Omega (the FP64 draw of the run with the same
// seed). With V = [V1 V2] the right singular vectors of A, V1 its first
// r = l - p columns, Omega1 = V1^T Omega (r x l) and Omega2 = V2^T Omega
// (Sec. IV-A). Omega2 is never formed: V is orthogonal, so
// Omega2^T Omega2 = Omega^T Omega - Omega1^T Omega1, and ||Omega2||_2 is the
// square root of that l x l matrix's largest eigenvalue (its largest
// singular value, from the core SVD). ||Omega1^+||_2 = 1 / sigma_min(Omega1):
// the QR Omega1^T = Q R (l x r) leaves the singular values in R (r x r),
// whose core SVD gives sigma_min. The bounds themselves are scalar formulas
// of those two norms and of the singular values of A.

size_t sorsvd_bounds_workspace_bytes(int64_t n, int64_t l, int64_t p) {
  BoundsLayout b;
  return bounds_layout(n, l, p, &b) == SORSVD_OK ? b.total : 0;
}

int sorsvd_bounds(const double* V1, int64_t ldv, int64_t n, int64_t l, int64_t p, int64_t k, int32_t q,
                  uint64_t seed, const double* sigma, int64_t nsig, double* th4, double* th6,
                  sorsvd_bounds_info* out, void* ws, size_t ws_bytes, void* stream) {
  BoundsLayout b;
  int rc = bounds_layout(n, l, p, &b);
  if (rc) return rc;
  const int64_t r = l - p;
  if (!V1 || !sigma || !out || !ws || ldv < r || q < 0 || k < 1 || p + k > l || p + k < 2 || nsig < r + 1 ||
      nsig < k + 1)
    return SORSVD_EINVAL;
  for (int64_t j = 0; j < nsig; ++j)
    if (!(sigma[j] >= 0.0) || (j > 0 && sigma[j] > sigma[j - 1])) return SORSVD_EINVAL;
  if (!(sigma[k - 1] > 0.0)) return SORSVD_EINVAL;
  if (ws_bytes < b.total) return SORSVD_EWORKSPACE;
  if (((uintptr_t)ws) % kAlign) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int64_t LP = b.LP;
  double* Om = at<double>(ws, b.off_om);
  double* O1 = at<double>(ws, b.off_o1);
  double* O1t = at<double>(ws, b.off_o1t);
  double* G = at<double>(ws, b.off_g);
  double* H1 = at<double>(ws, b.off_h1);
  double* H = at<double>(ws, b.off_h);
  double* P = at<double>(ws, b.off_p);
  double* Ut = at<double>(ws, b.off_ut);
  double* Vt = at<double>(ws, b.off_vt);
  double* sv = at<double>(ws, b.off_s);
  double* Q = at<double>(ws, b.off_q);
  double* R = at<double>(ws, b.off_r);
  void* sub = at<void>(ws, b.off_sub);
  SORSVD_TRY(launch_fill(Om, n * LP, 0.0, st));
  SORSVD_TRY(launch_omega_rowmajor_f64(seed, n, l, Om, LP, st));
  // Omega1 = V1^T Omega (r x LP), Omega^T Omega (LP x LP)
  SORSVD_TRY(launch_fill(O1, LP * LP, 0.0, st));
  SORSVD_TRY(launch_skinny_f64(true, V1, ldv, r, n, Om, LP, (int)LP, b.sp.kchunk, b.sp.nsplit, P, nullptr, nullptr,
                               st, nullptr, false, b.ncb));
  SORSVD_TRY(launch_reduce_f64(P, r, (int)LP, b.sp.nsplit, O1, LP, (int)LP, st));
  SORSVD_TRY(launch_skinny_f64(true, Om, LP, LP, n, Om, LP, (int)LP, b.sp.kchunk, b.sp.nsplit, P, nullptr, nullptr,
                               st, nullptr, false, b.ncb));
  SORSVD_TRY(launch_reduce_f64(P, LP, (int)LP, b.sp.nsplit, G, LP, (int)LP, st));
  // Omega1^T Omega1 over the r rows of Omega1 (one split)
  const int ks = skinny_step(SORSVD_F64);
  SORSVD_TRY(launch_skinny_f64(true, O1, LP, LP, r, O1, LP, (int)LP, round_up(r, ks), 1, P, nullptr, nullptr, st,
                               H1, false, b.ncb));
  // Omega2^T Omega2 = Omega^T Omega - Omega1^T Omega1 (l x l): its largest singular value
  SORSVD_TRY(launch_sub_f64(G, LP, H1, LP, l, (int)l, H, l, st));
  if ((rc = sorsvd_step_core_svd(H, l, 1, Ut, sv, Vt, 0, sub, b.sub_bytes, stream))) return rc;
  double lam = 0.0;
  SORSVD_TRY(hipMemcpyAsync(&lam, sv, sizeof(double), hipMemcpyDeviceToHost, st));
  // sigma_min(Omega1) from R of Omega1^T = Q R
  SORSVD_TRY(launch_transpose_f64(O1, LP, r, (int)l, O1t, r, st));
  if ((rc = sorsvd_step_qr(O1t, l, r, Q, R, sub, b.sub_bytes, stream))) return rc;
  if ((rc = sorsvd_step_core_svd(R, r, r, Ut, sv, Vt, 0, sub, b.sub_bytes, stream))) return rc;
  double smin = 0.0;
  SORSVD_TRY(hipMemcpyAsync(&smin, sv + (r - 1), sizeof(double), hipMemcpyDeviceToHost, st));
  SORSVD_TRY(hipStreamSynchronize(st));
  std::memset(out, 0, sizeof(*out));
  out->omega2_norm = std::sqrt(std::max(lam, 0.0));
  out->omega1_pinv_norm = smin > 0.0 ? 1.0 / smin : INFINITY;
  // Th. 1 floors
  double tail = 0.0;
  for (int64_t j = nsig - 1; j >= k; --j) tail += sigma[j] * sigma[j];
  const double a0f = std::sqrt(tail), a02 = sigma[k];
  const double s1 = sigma[0], sk = sigma[k - 1], slp = sigma[r];
  const double gprod = out->omega2_norm * out->omega1_pinv_norm;
  const double g = gprod * gprod;
  // Th. 4: per-j lower bounds
  if (th4)
    for (int64_t j = 0; j < k; ++j)
      th4[j] = sigma[j] > 0.0 ? sigma[j] / std::sqrt(1.0 + g * std::pow(slp / sigma[j], 4.0 * q + 4.0)) : 0.0;
  // Th. 5, with the power-method factors (slp / sk)^(2q) and the reading of
  // tau = (sk / slp) beta, as for eta = (sk / slp) alpha
  const double decay = std::pow(slp / sk, 2.0 * q);
  const double alpha = std::sqrt((double)k) * slp * slp / sk * decay;
  const double beta = slp * slp / (s1 * sk) * decay;
  const double eta = slp > 0.0 ? (sk / slp) * alpha : 0.0;
  const double tau = slp > 0.0 ? (sk / slp) * beta : 0.0;
  const double extra = std::sqrt(alpha * alpha * g / (1.0 + beta * beta * g)) +
                       std::sqrt(eta * eta * g / (1.0 + tau * tau * g));
  out->th5_fro = a0f + extra;
  out->th5_2 = a02 + extra;
  // Th. 6 / Th. 7 (expectations over Omega; need p >= 2)
  if (p >= 2) {
    const double nu = bounds_nu(n, l, p);
    if (th6)
      for (int64_t j = 0; j < k; ++j)
        th6[j] = sigma[j] > 0.0 ? sigma[j] / std::sqrt(1.0 + nu * nu * std::pow(slp / sigma[j], 4.0 * q + 4.0)) : 0.0;
    const double gk = slp / sk;
    const double t7 = (1.0 + gk) * std::sqrt((double)k) * nu * slp * std::pow(gk, 2.0 * q);
    out->th7_fro = a0f + t7;
    out->th7_2 = a02 + t7;
  } else {
    if (th6)
      for (int64_t j = 0; j < k; ++j) th6[j] = NAN;
    out->th7_fro = out->th7_2 = NAN;
  }
  return SORSVD_OK;
}

int sorsvd_pass_timing(int32_t enable, int32_t capacity) {
  PassTimer& tm = timer();
  std::lock_guard<std::mutex> g(tm.mu);
  if (enable && capacity < 1) return SORSVD_EINVAL;
  for (hipEvent_t e : tm.ev) hipEventDestroy(e);
  tm.ev.clear();
  tm.used = 0;
  tm.bytes = tm.flops = 0.0;
  tm.on = false;
  if (!enable) return SORSVD_OK;
  tm.ev.resize(2 * (size_t)capacity, nullptr);
  for (auto& e : tm.ev)
    if (hipEventCreate(&e) != hipSuccess) return SORSVD_EHIP;
  tm.on = true;
  return SORSVD_OK;
}

int sorsvd_pass_timing_read(double* total_ms, int64_t* launches, double* bytes, double* flops) {
  if (!total_ms || !launches || !bytes || !flops) return SORSVD_EINVAL;
  PassTimer& tm = timer();
  std::lock_guard<std::mutex> g(tm.mu);
  double ms = 0.0;
  for (size_t i = 0; i + 1 < tm.used; i += 2) {
    if (hipEventSynchronize(tm.ev[i + 1]) != hipSuccess) return SORSVD_EHIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, tm.ev[i], tm.ev[i + 1]) != hipSuccess) return SORSVD_EHIP;
    ms += t;
  }
  *total_ms = ms;
  *launches = (int64_t)(tm.used / 2);
  *bytes = tm.bytes;
  *flops = tm.flops;
  tm.used = 0;
  tm.bytes = tm.flops = 0.0;
  return SORSVD_OK;
}

// ------------------------------------------------------------------ learned (k, q)

static int probe_plan(int64_t m, int64_t n, int32_t a_type, Plan* p) {
  if (a_type == SORSVD_F16) return SORSVD_EUNSUPPORTED;
  const int64_t l = std::min<int64_t>(kProbeL, std::min(m, n));
  sorsvd_opts o;
  std::memset(&o, 0, sizeof(o));
  o.l = l;
  return make_plan(m, n, l, 0, a_type, &o, p);
}

size_t sorsvd_probe_workspace_bytes(int64_t m, int64_t n, int32_t a_type) {
  Plan p;
  return probe_plan(m, n, a_type, &p) == SORSVD_OK ? p.total : 0;
}

int sorsvd_probe_features(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, uint64_t seed,
                          float* features, void* workspace, size_t ws_bytes, void* stream) {
  Plan p;
  const int rc = probe_plan(m, n, a_type, &p);
  if (rc) return rc;
  if (!A || !features || !workspace || (lda < n && a_type != SORSVD_DIAG)) return SORSVD_EINVAL;
  if (ws_bytes < p.total) return SORSVD_EWORKSPACE;
  if (((uintptr_t)workspace) % kAlign) return SORSVD_EINVAL;
  return probe(p, A, lda, seed, features, workspace, (hipStream_t)stream);
}

int32_t sorsvd_mlp_param_count(void) { return mlp_param_count(); }

size_t sorsvd_mlp_work_floats(int32_t batch) { return batch < 1 ? 0 : mlp_work_floats(batch); }

int sorsvd_mlp_forward(const float* params, const float* X, int32_t batch, float* Y, float* work, void* stream) {
  if (!params || !X || !Y || !work || batch < 1) return SORSVD_EINVAL;
  SORSVD_TRY(launch_mlp_forward(params, X, batch, Y, work, (hipStream_t)stream));
  return SORSVD_OK;
}

int sorsvd_mlp_backward(const float* params, const float* X, const float* T, int32_t batch, float* grad,
                        float* loss, float* work, void* stream) {
  if (!params || !X || !T || !grad || !loss || !work || batch < 1) return SORSVD_EINVAL;
  SORSVD_TRY(launch_mlp_backward(params, X, T, batch, grad, loss, work, (hipStream_t)stream));
  return SORSVD_OK;
}

int sorsvd_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                    float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return SORSVD_EINVAL;
  SORSVD_TRY(launch_mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream));
  return SORSVD_OK;
}

int sorsvd_mlp_train_step(float* params, float* m, float* v, const float* X, const float* T, int32_t batch,
                          int64_t step, float lr, float* grad, float* loss, float* work, void* stream) {
  int rc = sorsvd_mlp_backward(params, X, T, batch, grad, loss, work, stream);
  if (rc) return rc;
  return sorsvd_mlp_adam(params, grad, m, v, step, lr, 0.9f, 0.999f, 1e-8f, stream);
}

static constexpr double kAutoMargin = 1.25;      // head-room on the predicted width
// BF16: more head-room, since the judge certifies a BF16 result only below the
// tolerance minus its rounding-noise allowance (the labels are the widths at
// which the true error reaches the tolerance)
static constexpr double kAutoMarginBF16 = 1.6;
static constexpr int64_t kAutoFallbackK = 256;  // first rung of the fixed ladder
static constexpr int kAutoFallbackQ = 2;
static constexpr double kNoiseShare = 2.5;   // BF16 judge: captured rounding-noise allowance / i.i.d. share

// Options of every run sorsvd_auto may start, and so of its workspace: BF16
// A with refinement and the pass-efficient core matrix (2q + 2 passes, the
// last orbit product with Q1 split hi + lo); the explicit residual is added
// by the caller where the judge needs it.
static void auto_opts(int32_t a_type, sorsvd_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->refine = a_type == SORSVD_BF16 ? 1 : 0;
  o->pass_efficient = a_type == SORSVD_BF16 ? 1 : 0;
}

static int auto_plan(int64_t m, int64_t n, int32_t a_type, Plan* p) {
  if (a_type == SORSVD_F16) return SORSVD_EUNSUPPORTED;
  const int64_t kcap = std::min<int64_t>(kMaxLP, std::min(m, n));
  sorsvd_opts o;
  auto_opts(a_type, &o);
  o.residual = a_type == SORSVD_DIAG ? 0 : 1;  // (diagonal stand-ins take no residual pass)
  return make_plan(m, n, kcap, 3, a_type, &o, p);
}

// Tail of the sorsvd_auto workspace: features and network outputs, network
// scratch, and the probe's Q (m x its padded width) and norm slots, kept for
// the runs that start from them.
static size_t auto_tail_bytes(int64_t m, int64_t n, int32_t a_type) {
  Plan pp;
  size_t keep = 0;
  if (probe_plan(m, n, a_type, &pp) == SORSVD_OK)
    keep = round_up((int64_t)m * pp.LP * 8, kAlign) + round_up((int64_t)std::max(pp.nn_blocks, 1) * 8, kAlign);
  return 256 + 4096 + round_up((int64_t)mlp_work_floats(1) * 4, 256) + keep;
}

// Largest workspace of any run sorsvd_auto may start (k a multiple of 8 or the
// cap, any q <= 3) and of the probe; the tail (features, outputs, network
// scratch) follows it.
static size_t auto_main_bytes(int64_t m, int64_t n, int32_t a_type) {
  Plan p;
  if (auto_plan(m, n, a_type, &p) != SORSVD_OK) return 0;
  size_t mx = p.total;
  const int64_t kcap = p.k;
  sorsvd_opts o;
  auto_opts(a_type, &o);
  o.residual = a_type == SORSVD_DIAG ? 0 : 1;
  for (int64_t k = 8; k < kcap; k += 8) {
    Plan pk;
    if (make_plan(m, n, k, 3, a_type, &o, &pk) == SORSVD_OK) mx = std::max(mx, pk.total);
  }
  Plan pp;
  if (probe_plan(m, n, a_type, &pp) == SORSVD_OK) mx = std::max(mx, pp.total);
  return round_up((int64_t)mx, kAlign);
}

size_t sorsvd_auto_workspace_bytes(int64_t m, int64_t n, int32_t a_type) {
  const size_t mb = auto_main_bytes(m, n, a_type);
  return mb ? mb + auto_tail_bytes(m, n, a_type) : 0;
}

// The (k, q) of a run from the network's outputs y_q = log2 of the width
// that meets the trained tolerance with q power steps: each width gets
// kAutoMargin head-room (kAutoMarginBF16 for BF16 A; rounded up to a
// multiple of 8) and is capped at kcap; a width predicted beyond kcap is
// dropped (the network then says kcap is short for that q; its label for
// "more than the widest sketch" is 2 kcap), and among the rest the q of the
// least modelled time is taken. k_pred[q] = 2^y_q. Returns whether any
// width is left.
static bool choose_kq(int32_t a_type, int64_t m, int64_t n, int64_t kcap, const float yh[4], double k_pred[4],
                      int64_t* k, int* q) {
  // Modelled time of a run of width k with q power steps (seconds), to pick
  // q among the predicted widths: the passes over A (bytes at ~5 TB/s or
  // flops at the MFMA rate reached, whichever is larger), the FP64 Cholesky
  // QRs of the two sketches (a Gram and an apply per step, ~2 steps per QR)
  // and the core SVD (~1e-11 k^3 s for the blocked one-sided Jacobi).
  const double es = a_type == SORSVD_BF16 ? 2.0 : (a_type == SORSVD_F32 ? 4.0 : 8.0);
  const double rate = a_type == SORSVD_BF16 ? 1.2e15 : (a_type == SORSVD_F32 ? 9e13 : 4e13);
  auto model_s = [&](double kk, int qq) {
    const double passes = 2.0 * qq + (a_type == SORSVD_BF16 ? 2.0 : 3.0);  // see auto_opts
    const double t_pass = std::max((double)m * n * es / 5e12, 2.0 * m * n * kk / rate);
    const double t_qr = (2.0 * qq + 2.0) * 2.0 * 3.0 * (double)(m + n) / 2.0 * kk * kk / 4e13;
    return passes * t_pass + t_qr + 1e-11 * kk * kk * kk;
  };
  double best = 1e300;
  bool predicted = false;
  // BF16 passes round the skinny operand: without a power step the subspace
  // error of that rounding stays near 1e-3, so BF16 runs take q >= 1
  const int qmin = a_type == SORSVD_BF16 ? 1 : 0;
  for (int qq = 0; qq < 4; ++qq) {
    k_pred[qq] = yh[qq] == yh[qq] ? std::exp2((double)yh[qq]) : 1e30;
    if (qq < qmin) continue;
    if (!(k_pred[qq] <= (double)kcap)) continue;  // the network says even kcap is short
    const double margin = a_type == SORSVD_BF16 ? kAutoMarginBF16 : kAutoMargin;
    const double kk = std::min((double)kcap, std::ceil(margin * k_pred[qq] / 8.0) * 8.0);
    const int64_t ki = std::max<int64_t>(1, (int64_t)kk);
    const double cost = model_s((double)ki, qq);
    if (cost < best) {
      best = cost;
      *k = ki;
      *q = qq;
      predicted = true;
    }
  }
  return predicted;
}

int sorsvd_auto(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, uint64_t seed, double tol,
                const float* params, double* U, int64_t ldu, double* S, double* V, int64_t ldv, void* workspace,
                size_t ws_bytes, void* stream, sorsvd_auto_info* out) {
  Plan big;
  int rc = auto_plan(m, n, a_type, &big);
  if (rc) return rc;
  const int64_t kcap = big.k;
  if (!A || !U || !S || !V || !workspace || !out || lda < n || ldu < kcap || ldv < kcap || !(tol > 0.0))
    return SORSVD_EINVAL;
  const size_t main_bytes = auto_main_bytes(m, n, a_type);
  if (ws_bytes < main_bytes + auto_tail_bytes(m, n, a_type)) return SORSVD_EWORKSPACE;
  if (((uintptr_t)workspace) % kAlign) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  std::memset(out, 0, sizeof(*out));
  char* tail = (char*)workspace + main_bytes;
  float* feat = (float*)(tail + 256);
  float* y = feat + 128;
  float* work = (float*)(tail + 256 + 4096);
  double* keep_q = (double*)(tail + 256 + 4096 + round_up((int64_t)mlp_work_floats(1) * 4, 256));
  double* keep_n = nullptr;
  int64_t keep_ld = 0;
  int keep_parts = 0;

  int64_t k = std::min(kAutoFallbackK, kcap);
  int q = kAutoFallbackQ;
  bool predicted = false;
  if (params) {
    Plan pp;
    if ((rc = probe_plan(m, n, a_type, &pp))) return rc;
    if ((rc = probe(pp, A, lda, seed, feat, workspace, st))) return rc;
    // keep the probe's Q and norm slots: Omega is nested in its width and
    // Cholesky QR keeps column prefixes, so the leading k columns of that Q
    // are Q1 of the run's first sketch
    keep_ld = pp.LP;
    keep_n = keep_q + round_up((int64_t)m * pp.LP * 8, kAlign) / 8;
    keep_parts = pp.nn_blocks;
    SORSVD_TRY(launch_pack_f64(at<double>(workspace, pp.off_t1), m, (int)pp.LP, pp.LP, keep_q, (int)pp.LP, st));
    SORSVD_TRY(launch_pack_f64(at<double>(workspace, pp.off_normp), pp.nn_blocks, 1, 1, keep_n, 1, st));
    SORSVD_TRY(launch_mlp_forward(params, feat, 1, y, work, st));
    float yh[4];
    SORSVD_TRY(hipMemcpyAsync(yh, y, sizeof(yh), hipMemcpyDeviceToHost, st));
    SORSVD_TRY(hipStreamSynchronize(st));
    predicted = choose_kq(a_type, m, n, kcap, yh, out->k_pred, &k, &q);
  }
  // the predicted (k, q), then the fixed ladder: (256, 2), (512, 2), ... up
  // to the cap, until the judge accepts
  std::vector<std::pair<int64_t, int>> runs;
  if (predicted) runs.emplace_back(k, q);
  for (int64_t kf = std::min(kAutoFallbackK, kcap);; kf = std::min(2 * kf, kcap)) {
    if (!(predicted && kf == k && q == kAutoFallbackQ)) runs.emplace_back(kf, kAutoFallbackQ);
    if (kf == kcap) break;
  }
  for (size_t attempt = 0; attempt < runs.size(); ++attempt) {
    k = runs[attempt].first;
    q = runs[attempt].second;
    sorsvd_opts o;
    auto_opts(a_type, &o);
    o.residual = a_type == SORSVD_BF16 ? 1 : 0;  // BF16: the identity cannot resolve 1e-3
    Plan p;
    if ((rc = make_plan(m, n, k, q, a_type, &o, &p))) return rc;
    const bool reuse = keep_n && p.l <= keep_ld;
    if ((rc = run(p, A, lda, seed, U, ldu, S, V, ldv, workspace, st, reuse ? keep_q : nullptr, keep_ld,
                  reuse ? keep_n : nullptr, keep_parts)))
      return rc;
    sorsvd_info info;
    SORSVD_TRY(hipMemcpyAsync(&info, workspace, sizeof(info), hipMemcpyDeviceToHost, st));
    SORSVD_TRY(hipStreamSynchronize(st));
    double e = info.err_fro;
    out->err_stored = o.residual ? info.err_fro_explicit : e;
    if (o.residual) {
      // error against A before rounding: e^2 = e_stored^2 - (1 - 2 c) noise^2,
      // c the share of the rounding noise E (expected size a_noise_rel) that
      // the rank-k fit absorbs. For i.i.d. noise c is at most
      // k (m^-1/2 + n^-1/2)^2 (the top-k singular values of an m x n noise
      // matrix); BF16 rounding noise follows |a_ij| (heteroscedastic), and
      // measured shares near the tolerance reach 1.9 times that, so the
      // allowance is 2.5 times it (overestimating c only makes e larger)
      const double es = info.err_fro_explicit, nz = info.a_noise_rel;
      const double rho = std::min(1.0, kNoiseShare * (double)k *
                                           std::pow(1.0 / std::sqrt((double)m) + 1.0 / std::sqrt((double)n), 2.0));
      e = std::sqrt(std::max(es * es - (1.0 - 2.0 * rho) * nz * nz, 0.0));
    }
    out->runs += 1;
    out->k_used = (int32_t)k;
    out->q_used = q;
    out->err = e;
    out->used_fallback = (attempt > 0 || !predicted) ? 1 : 0;
    out->flags = info.flags;
    if (e <= tol) return SORSVD_OK;
  }
  return SORSVD_ETOL;
}

int sorsvd_predict_kq(const void* A, int64_t lda, int32_t a_type, int64_t m, int64_t n, uint64_t seed,
                      const float* params, double tol, int64_t* k_out, int32_t* q_out, double* k_pred,
                      void* workspace, size_t ws_bytes, void* stream) {
  Plan big;
  int rc = auto_plan(m, n, a_type, &big);
  if (rc) return rc;
  if (!A || !params || !k_out || !q_out || !workspace || (lda < n && a_type != SORSVD_DIAG) || !(tol > 0.0))
    return SORSVD_EINVAL;
  const size_t main_bytes = auto_main_bytes(m, n, a_type);
  if (ws_bytes < main_bytes + auto_tail_bytes(m, n, a_type)) return SORSVD_EWORKSPACE;
  if (((uintptr_t)workspace) % kAlign) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char* tail = (char*)workspace + main_bytes;
  float* feat = (float*)(tail + 256);
  float* y = feat + 128;
  float* work = (float*)(tail + 256 + 4096);
  Plan pp;
  if ((rc = probe_plan(m, n, a_type, &pp))) return rc;
  if ((rc = probe(pp, A, lda, seed, feat, workspace, st))) return rc;
  SORSVD_TRY(launch_mlp_forward(params, feat, 1, y, work, st));
  float yh[4];
  SORSVD_TRY(hipMemcpyAsync(yh, y, sizeof(yh), hipMemcpyDeviceToHost, st));
  SORSVD_TRY(hipStreamSynchronize(st));
  double kp[4];
  int64_t k = std::min(kAutoFallbackK, big.k);
  int q = kAutoFallbackQ;
  const bool predicted = choose_kq(a_type, m, n, big.k, yh, kp, &k, &q);
  if (k_pred)
    for (int i = 0; i < 4; ++i) k_pred[i] = kp[i];
  *k_out = k;
  *q_out = q;
  return predicted ? SORSVD_OK : SORSVD_ETOL;
}

// ------------------------------------------------------------------ robust PCA (ALM-SOR-SVD)

static constexpr int kRpcaNormWidth = 32;  // sketch width of the ||X||_2 estimate
static constexpr int kRpcaNormQ = 8;

static int rpca_plans(int64_t m, int64_t n, int64_t l, int32_t q, Plan* p, Plan* pn) {
  if (m < 1 || n < 1 || l < 1 || l > std::min<int64_t>(kMaxLP, std::min(m, n)) || q < 0) return SORSVD_EINVAL;
  int rc = make_plan(m, n, l, q, SORSVD_F64, nullptr, p);
  if (rc) return rc;
  return make_plan(m, n, std::min<int64_t>(kRpcaNormWidth, std::min(m, n)), kRpcaNormQ, SORSVD_F64, nullptr, pn);
}

// Layout after the SOR-SVD workspace: Y, W (m x n), U (m x l), V (n x l), z (l),
// the norm sketch's factors, and the per-block partial sums.
struct RpcaLayout {
  size_t y, w, u, v, z, un, vn, zn, part, total;
};
static RpcaLayout rpca_layout(const Plan& p, const Plan& pn, int64_t m, int64_t n, int64_t l) {
  Layout L;
  L.take(std::max(p.total, pn.total));
  RpcaLayout r;
  r.y = L.take((size_t)m * n * 8);
  r.w = L.take((size_t)m * n * 8);
  r.u = L.take((size_t)m * l * 8);
  r.v = L.take((size_t)n * l * 8);
  r.z = L.take((size_t)l * 8);
  r.un = L.take((size_t)m * pn.k * 8);
  r.vn = L.take((size_t)n * pn.k * 8);
  r.zn = L.take((size_t)pn.k * 8);
  const int64_t parts = std::max<int64_t>(rpca_step_blocks(m, n), 2 * (int64_t)rpca_stat_blocks(m, n));
  r.part = L.take((size_t)parts * 8);
  r.total = L.total;
  return r;
}

size_t sorsvd_rpca_workspace_bytes(int64_t m, int64_t n, int64_t l, int32_t q) {
  Plan p, pn;
  if (rpca_plans(m, n, l, q, &p, &pn)) return 0;
  return rpca_layout(p, pn, m, n, l).total;
}

int sorsvd_rpca(const double* X, int64_t ldx, int64_t m, int64_t n, int64_t l, int32_t q, uint64_t seed,
                double tol, int32_t max_iter, double* L, double* S, int64_t ld, void* workspace, size_t ws_bytes,
                void* stream, sorsvd_rpca_info* out) {
  Plan p, pn;
  int rc = rpca_plans(m, n, l, q, &p, &pn);
  if (rc) return rc;
  if (!X || !L || !S || !workspace || !out || ldx < n || ld < n || !(tol > 0.0) || max_iter < 1)
    return SORSVD_EINVAL;
  const RpcaLayout R = rpca_layout(p, pn, m, n, l);
  if (ws_bytes < R.total) return SORSVD_EWORKSPACE;
  if (((uintptr_t)workspace) % kAlign) return SORSVD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  std::memset(out, 0, sizeof(*out));
  double* Y = at<double>(workspace, R.y);
  double* W = at<double>(workspace, R.w);
  double* U = at<double>(workspace, R.u);
  double* V = at<double>(workspace, R.v);
  double* z = at<double>(workspace, R.z);
  double* part = at<double>(workspace, R.part);
  const int kn = (int)pn.k;

  // ||X||_F, ||X||_max (fixed-order sums on the host of per-block partials)
  const int sb = rpca_stat_blocks(m, n);
  SORSVD_TRY(launch_rpca_stats(X, ldx, m, n, part, part + sb, st));
  std::vector<double> hp(2 * (size_t)sb);
  SORSVD_TRY(hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, st));
  SORSVD_TRY(hipStreamSynchronize(st));
  double fro2 = 0.0, xmax = 0.0;
  for (int i = 0; i < sb; ++i) {
    fro2 += hp[i];
    xmax = std::max(xmax, hp[sb + i]);
  }
  const double xfro = std::sqrt(fro2);
  // ||X||_2: the leading value of a narrow SOR-SVD of X with power steps
  if ((rc = run(pn, X, ldx, seed ^ 0x9E3779B97F4A7C15ull, at<double>(workspace, R.un), kn,
                at<double>(workspace, R.zn), at<double>(workspace, R.vn), kn, workspace, st)))
    return rc;
  double norm2 = 0.0;
  SORSVD_TRY(hipMemcpyAsync(&norm2, at<double>(workspace, R.zn), 8, hipMemcpyDeviceToHost, st));
  SORSVD_TRY(hipStreamSynchronize(st));
  out->norm2 = norm2;
  if (!(xfro > 0.0) || !(norm2 > 0.0) || !std::isfinite(fro2)) return SORSVD_EINVAL;
  const double lambda = 1.0 / std::sqrt((double)std::max(m, n));
  out->lambda = lambda;
  double mu = 1.25 / norm2;
  const double mu_bar = 1e7 * mu, rho = 1.5;
  const double J = std::max(norm2, xmax / lambda);
  SORSVD_TRY(launch_rpca_init(X, ldx, m, n, 1.0 / J, 1.0 / mu, S, ld, Y, W, st));

  const int64_t nb = rpca_step_blocks(m, n);
  std::vector<double> rp((size_t)nb);
  double mu_used = mu;
  int it = 0;
  double xi = 0.0;
  while (it < max_iter) {
    if ((rc = run(p, W, n, seed + (uint64_t)it, U, l, z, V, l, workspace, st))) return rc;
    const double mu_next = std::min(rho * mu, mu_bar);
    SORSVD_TRY(launch_rpca_step(X, ldx, m, n, U, V, z, (int)l, 1.0 / mu, lambda / mu, mu, 1.0 / mu_next, L, S, ld,
                                Y, W, part, st));
    SORSVD_TRY(hipMemcpyAsync(rp.data(), part, (size_t)nb * 8, hipMemcpyDeviceToHost, st));
    SORSVD_TRY(hipStreamSynchronize(st));
    double r2 = 0.0;
    for (int64_t i = 0; i < nb; ++i) r2 += rp[i];
    mu_used = mu;
    mu = mu_next;
    ++it;
    xi = std::sqrt(r2) / xfro;
    if (!std::isfinite(xi) || xi < tol) break;
  }
  out->iters = it;
  out->xi = xi;
  // singular values kept by the last thresholding; nonzeros of S
  std::vector<double> hz((size_t)l);
  SORSVD_TRY(hipMemcpyAsync(hz.data(), z, (size_t)l * 8, hipMemcpyDeviceToHost, st));
  SORSVD_TRY(launch_rpca_nnz(S, ld, m, n, part, st));
  std::vector<double> hc((size_t)sb);
  SORSVD_TRY(hipMemcpyAsync(hc.data(), part, (size_t)sb * 8, hipMemcpyDeviceToHost, st));
  SORSVD_TRY(hipStreamSynchronize(st));
  int kept = 0;
  for (int64_t t = 0; t < l; ++t) kept += hz[t] - 1.0 / mu_used > 0.0 ? 1 : 0;
  out->rank = kept;
  double nnz = 0.0;
  for (int i = 0; i < sb; ++i) nnz += hc[i];
  out->nnz_s = (int64_t)nnz;
  return xi < tol ? SORSVD_OK : SORSVD_ETOL;
}

const char* sorsvd_status_string(int status) {
  switch (status) {
    case SORSVD_OK: return "ok";
    case SORSVD_EINVAL: return "invalid argument";
    case SORSVD_EWORKSPACE: return "workspace too small";
    case SORSVD_EHIP: return "HIP runtime error";
    case SORSVD_ENOCONV: return "Jacobi sweep cap reached";
    case SORSVD_ENONFINITE: return "non-finite input";
    case SORSVD_ETOL: return "tolerance not met";
    case SORSVD_EUNSUPPORTED: return "unsupported by the library";
    default: return "unknown status";
  }
}

const char* sorsvd_version(void) { return "sorsvd-gfx950 0.1"; }

}  // extern "C"
