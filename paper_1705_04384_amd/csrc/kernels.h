// Launch wrappers of the device kernels (host-callable, stream-ordered, no allocation).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fdg {

// Number of partial-sum blocks of a reduction over vectors of length N.  Depends on N
// only, so a reduction gives the same bits for a problem alone or inside a batch.
int reduction_blocks(int64_t N);

// ---- FD mode products --------------------------------------------------------------
// Mode product over a tensor stored as [nbatch][n][ncols] with general strides:
//   Y[o*sO + k*sJ + c*sC] = sum_j W[k*ldw + j] X[o*sO + j*sJ + c*sC],
// k, j < n, c < ncols, o < nbatch.  W is zero-padded to ldw >= roundup(n, 64) rows and
// columns.  X and Y must not alias.
void launch_modeprod_f64(hipStream_t s, const double *X, double *Y, const double *W, int ldw,
                         int n, int64_t ncols, int64_t sO, int64_t sJ, int64_t sC, int64_t nbatch);

// t[b][i_d]..[i_1] /= sum_l lam_l[i_l]; lam3 may be NULL for d = 2.
void launch_divide_f64(hipStream_t s, double *t, int d, int n, int64_t nbatch, const double *lam1,
                       const double *lam2, const double *lam3);

// ---- operator ------------------------------------------------------------------------
// Banded univariate factors of the unit-domain operator: row i of factor F holds
// F[i][lo[i] + t] at band[i*w + t], t < w, with lo[i] + w <= n.
struct KronBands {
  const double *M[3];
  const double *K[3];
  const int32_t *lo[3];
  int w[3];
};
// Requires non-decreasing band starts lo[] and w <= kron_window_max().
void launch_kron_matvec_f64(hipStream_t s, const double *x, double *y, int d, int n, int64_t nbatch,
                            const KronBands &bands);
int kron_window_max();

// Slot-major ELL: entry (row, slot) at col[slot*ld + row], val[slot*ld + row].
void launch_ell_matvec_f64(hipStream_t s, const double *x, double *y, int64_t nrows, int64_t ld,
                           int width, const int32_t *col, const double *val, int64_t nbatch);

// ---- Krylov vector kernels --------------------------------------------------------------
// Vectors of a basis are stored q-major: element (q, b, i) at V[q*ldv + b*N + i].
// Partial sums of batch entry b, block g, component q at P[(b*G + g)*nv + q].
void launch_dots(hipStream_t s, const double *V, int64_t ldv, int nv, const double *w, int64_t N,
                 int64_t nbatch, int G, double *P);
// out[b*ostride + q] = sum_g P (sqrt of it if do_sqrt), q < ncomp; with add != NULL also
// out2[b*o2stride + q] = sum + add[b*astride + q].
void launch_reduce(hipStream_t s, const double *P, int G, int ncomp, int64_t nbatch, double *out,
                   int ostride, bool do_sqrt, const double *add, int astride, double *out2, int o2stride);
// w -= sum_q V_q h[b*hstride + q]; with Pnorm != NULL also the partial sums of |w|^2.
void launch_update(hipStream_t s, const double *V, int64_t ldv, int nv, const double *h, int hstride,
                   double *w, int64_t N, int64_t nbatch, int G, double *Pnorm);
// v = w / nrm[b*nstride] (0 where nrm is 0).
void launch_scale(hipStream_t s, const double *w, double *v, const double *nrm, int nstride,
                  int64_t N, int64_t nbatch);
// x += sum_q Z_q y[b*ystride + q], q < k.
void launch_lincomb(hipStream_t s, double *x, const double *Z, int64_t ldz, int k, const double *y,
                    int ystride, int64_t N, int64_t nbatch);
// r = b - Ax and partial sums of |r|^2.
void launch_residual(hipStream_t s, const double *b, const double *Ax, double *r, int64_t N,
                     int64_t nbatch, int G, double *P);

}  // namespace fdg
