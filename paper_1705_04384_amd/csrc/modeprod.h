// Reduced-precision fast-diagonalization apply (FP32, or BF16 inputs with FP32
// accumulation), used inside flexible GMRES whose outer iteration stays FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdg {

// s = P~^{-1} b for a batch of same-shape problems.  b, s: FP64 device vectors.
// ta, tb: FP32 device scratch of batch * n^d elements each.  Wv[l] / Wu[l]: the ldw x ldw
// zero-padded factors V_l^T and U_l in FP32 (prec = FP32) or BF16 bits (prec = BF16);
// lam[l]: FP32 eigenvalues padded with 1.  Returns an fdg_status.
int fd_apply_lowp(hipStream_t s, int prec, int d, int n, int64_t batch, const double *b, double *out,
                  void *ta, void *tb, const void *const *Wv, const void *const *Wu, float *const *lam,
                  int ldw);

}  // namespace fdg
