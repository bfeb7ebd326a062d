// Fused FP64 fast-diagonalization passes (see fd_apply.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_addr.h"

namespace fdg {

// Fused passes exist for 1 <= n <= 256 (factors zero-padded to ldw = roundup(n, 64)).
bool fd_fused_supported(int n);

// For each of nentries batch entries (spe contiguous n x n slabs each, entry e at X.at(e)):
// Y[s] = W2 . X[s] . W1^T per slab; with divide, Y[s][k2][k1] /= lam2[k2] + lam1[k1].
// W1, W2: ldw x ldw, row = output index.  aligned32: every entry pointer is 32-byte aligned.
// ev0, ev1 (optional): events the kernel's dispatch records at its start and end.
void launch_slab_f64(hipStream_t s, CBatch X, MBatch Y, const double *W1, const double *W2, int ldw,
                     int n, int64_t nentries, int spe, bool divide, const double *lam1, const double *lam2,
                     bool aligned32, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// For each batch entry b (at X.at(b)) and column c of the n x n^2 matrix X[b]:
//   Y[b][:, c] = Wb . ((Wa . X[b][:, c]) / (lam3 + lam2[c / n] + lam1[c % n])).
// lam3 padded with 1 to ldw entries.
void launch_fibre_f64(hipStream_t s, CBatch X, MBatch Y, const double *Wa, const double *Wb, int ldw,
                      int n, int64_t batch, const double *lam1, const double *lam2, const double *lam3,
                      hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// Fused FP32 solve of batch contiguous entries (FP64 b in, FP64 out): FP32 factors
// Wv[l] = V_l^T, Wu[l] = U_l (ldw x ldw, zero-padded) and eigenvalues lam[l] (padded
// with 1), FP32 intermediates t1, t2 of batch * N floats.  n <= 256.
void launch_fd_apply_f32(hipStream_t s, int d, int n, int64_t batch, const double *b, double *out, float *t1,
                         float *t2, const float *const *Wv, const float *const *Wu, const float *const *lam, int ldw);

// The same with BF16 products (inputs rounded to BF16 on entry to each MFMA, FP32
// accumulation and FP32 intermediates): Wv, Wu are the BF16 factor copies (ldw x ldw,
// zero-padded), lam the FP32 eigenvalues (padded with 1).  n <= 256.
void launch_fd_apply_bf16(hipStream_t s, int d, int n, int64_t batch, const double *b, double *out, float *t1,
                          float *t2, const void *const *Wv, const void *const *Wu, const float *const *lam, int ldw);

}  // namespace fdg
