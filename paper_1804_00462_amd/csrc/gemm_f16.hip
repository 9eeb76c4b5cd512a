// 16-bit passes over A: the FP16 instantiations of the pass kernels
// (h16_body.hpp; v_mfma_f32_16x16x32_f16, operands scaled by powers of two).
#include "h16_body.hpp"

namespace sor {

hipError_t launch_h16_f16(bool trans, const uint16_t* A, int64_t lda, int64_t OUT, int64_t K, const uint16_t* XT,
                          int64_t ldx, int LP, int64_t kchunk, int nsplit, int ncb, float* P, double* normp,
                          double* Tout, int fold, int rt, const H16Scale* sc, const int* cexp, hipStream_t st) {
  return launch_h16_fmt<kFmtF16>(trans, A, lda, OUT, K, XT, ldx, LP, kchunk, nsplit, ncb, P, normp, Tout, fold, rt,
                                 sc, cexp, st);
}

int h16_blocks_f16(bool trans, int rt, int CT) { return h16_blocks<kFmtF16>(trans, rt, CT); }

}  // namespace sor
