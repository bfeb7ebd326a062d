// Launch wrappers of the device kernels (host-callable, stream-ordered, no allocation).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_addr.h"

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

// Univariate D_l with 2 x 2 blocks: lam (n), mu (n; +b / -b on a pair's two indices),
// role (n; 0 single, 1 first of a pair, 2 second) and the first index of each of the nb
// blocks (start, nb entries).  Device pointers.
struct BlockEig {
  const double *lam = nullptr;
  const double *mu = nullptr;
  const int8_t *role = nullptr;
  const int32_t *start = nullptr;
  int nb = 0;
};
// y[b] = (sum_l I x D_l x I)^{-1} t[b] for block-diagonal D_l (e3 unused for d = 2), out
// of place; one thread per cell (block combination), the entries of a cell never straddle
// batch entries (a pair never straddles n).
void launch_blockdiv_f64(hipStream_t s, const double *t, double *y, int d, int n, int64_t nbatch,
                         const BlockEig &e1, const BlockEig &e2, const BlockEig &e3);

// ---- operator ------------------------------------------------------------------------
// Banded univariate factors of the unit-domain operator: row i of factor F holds
// F[i][lo[i] + t] at band[i*w + t], t < w, with lo[i] + w <= n.
struct KronBands {
  const double *M[3];
  const double *K[3];
  const int32_t *lo[3];
  int w[3];
  int rows4;   // max over i of lo2[min(i+3, n-1)] + w2 - lo2[i]: rows j2 that 4 rows i2 need
  int rows16;  // the same for 16 rows i2 (aligned tiles)
  int step3;   // max over i of lo3[i+1] - lo3[i]
  int step[3];  // max over i of lo_l[i+1] - lo_l[i], per direction
};
// Requires non-decreasing band starts lo[] and w <= kron_window_max().  tmp_a, tmp_c:
// per-entry scratch of n^3 doubles each for the two-pass 3D form (invalid: one pass).
// Returns false (nothing launched) for a gathered batch the two-pass form cannot take.
bool launch_kron_matvec_f64(hipStream_t s, CBatch x, MBatch y, int d, int n, int64_t nbatch,
                            const KronBands &bands, MBatch tmp_a, MBatch tmp_c);
int kron_window_max();
// The 3D matvec of nbatch entries can take the two-pass form (which accepts gathered
// batches); always true in 2D.
bool kron_two_pass_ok(int d, int n, int64_t nbatch, const KronBands &bands);
// r = b - A x with the one-pass 3D form, and one partial sum of |r|^2 per workgroup at
// part.at(e)[g], g < kron_residual_partials(d, n, bands) (block order).  Returns false
// (nothing launched) when that form does not apply.
bool launch_kron_residual_f64(hipStream_t s, CBatch x, CBatch rhs, MBatch r, int d, int n, int64_t nbatch,
                              const KronBands &bands, MBatch part);
// Number of partials launch_kron_residual_f64 writes per entry, 0 if it does not apply.
int kron_residual_partials(int d, int n, const KronBands &bands);
// The one-pass 3D form applies (band width <= 8, band starts growing by <= 1 per row in
// directions 1 and 2); it needs no scratch and accepts gathered batches.
bool kron_fused_ok(int n, int64_t nbatch, const KronBands &bands);

// Slot-major ELL: entry (row, slot) at col[slot*ld + row], val[slot*ld + row].
void launch_ell_matvec_f64(hipStream_t s, CBatch x, MBatch y, int64_t nrows, int64_t ld, int width,
                           const int32_t *col, const double *val, int64_t nbatch);

// Slot-major ELL with implicit columns, for a matrix on the n^d tensor grid whose row
// (i1, i2, i3) couples exactly the columns (lo1[i1] + t1, lo2[i2] + t2, lo3[i3] + t3),
// t_l < w[l] (lo_l[i] + w[l] <= n): slot t = (t3 w2 + t2) w1 + t1 of row r at
// val[t * nrows + r].  For d = 2, w[2] = 1 and lo3 is all zero.
void launch_ell_tensor_f64(hipStream_t s, CBatch x, MBatch y, int n, int d, const int w[3],
                           const int32_t *lo, const double *val, int64_t nbatch);

// ---- Krylov vector kernels --------------------------------------------------------------
// Vectors of a basis are stored q-major: element (q, b, i) at V[q*ldv + b*N + i].
// Partial sums of batch entry b, block g, component q at P[(b*G + g)*nv + q]
// (G = reduction_blocks(N) <= 256); the consuming kernel reduces them in a fixed order.
// "host" pointers are device addresses of host-mapped pinned memory (may be NULL).

// Coefficients passed by value (kernel argument), at most 256.
struct Coeffs {
  double v[256];
};

// Batch entry e of a Krylov kernel: basis (q = 0) at V.at(e), vector q at + q*ldv;
// nv.at(e) basis vectors; partial g of component q at P.at(e)[g*ldp + q] (one partial per
// block for norms: P.at(e)[g]).  aligned16_all: every pointer involved is 16-byte aligned
// (enables 2-wide accesses, which changes the summation order).

// P = partial sums of V_q . w, q < nv.
void launch_dots(hipStream_t s, CBatch V, int64_t ldv, IBatch nv, CBatch w, int64_t N, int64_t nbatch,
                 int G, int ldp, MBatch P, bool aligned16_all);
// h1 = sum(Pin) (block 0 stores it to hout.at(e)); w -= V h1; Pout = partials of V^T w.
void launch_update_dots(hipStream_t s, CBatch V, int64_t ldv, IBatch nv, CBatch Pin, int G, int ldp,
                        MBatch w, int64_t N, int64_t nbatch, MBatch Pout, MBatch hout, bool aligned16_all);
// h2 = sum(Pin); Hcol = h1 + h2 (and host copy); w -= V h2; Pnorm = partials of |w|^2
// (and, when valid, the same partials to Pdev, device memory a later kernel reduces).
void launch_update_norm(hipStream_t s, CBatch V, int64_t ldv, IBatch nv, CBatch Pin, int G, int ldp,
                        MBatch w, int64_t N, int64_t nbatch, MBatch Pnorm, CBatch h1, MBatch Hcol,
                        MBatch host, bool aligned16_all, MBatch Pdev = MBatch{});
// d = sqrt(sum of Pn.at(e)[g], g < G); v = w / d (0 if d = 0; v may equal w); d to
// out.at(e)[0] and host.at(e)[0] (either may be invalid).
void launch_scale_reduce(hipStream_t s, CBatch w, MBatch v, CBatch Pn, int G, int64_t N, int64_t nbatch,
                         MBatch out, MBatch host, bool aligned16_all);
// v = w / d (0 if d = 0; v may equal w), d = dtab[e] when dtab is given, else dval.
void launch_scale_by(hipStream_t s, CBatch w, MBatch v, const double *dtab, double dval, int64_t N,
                     int64_t nbatch, bool aligned16_all);
// d = sqrt(sum of Pn.at(e)[g]) to out and host.
void launch_norm_reduce(hipStream_t s, CBatch Pn, int G, int64_t nbatch, MBatch out, MBatch host);
// x = (overwrite ? 0 : x) + sum_q Z_q y_q, q < k.at(e) <= 256; coefficients from ytab[e*256 + q]
// when ytab is given, else y (shared by every entry).
void launch_lincomb(hipStream_t s, MBatch x, CBatch Z, int64_t ldz, IBatch k, const Coeffs &y,
                    const double *ytab, int64_t N, int64_t nbatch, IBatch overwrite, bool aligned16_all);
// r = b - Ax and the partials P.at(e)[g] of |r|^2 (2-wide accesses, and so a different
// summation order, when every pointer is 16-byte aligned and N is even).
void launch_residual(hipStream_t s, CBatch b, CBatch Ax, MBatch r, int64_t N, int64_t nbatch, int G,
                     MBatch P, bool aligned16_all);

}  // namespace fdg
