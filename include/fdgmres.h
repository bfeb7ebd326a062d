/*
 * fdgmres.h -- C ABI of the MI355X (gfx950) FD-preconditioned flexible GMRES library.
 *
 * Problem (M. Tani, arXiv 1705.04384): the nonsymmetric system A u = f of eq. 3.1
 * from B-spline collocation of the Poisson problem (eq. 2.1 with K = I, Sec. 2.2),
 * solved by GMRES (Sec. 3) preconditioned with P, the same discretization on the
 * unit domain: P is the Kronecker sum of eq. 2.7 (d = 2) or eq. 2.9 (d = 3), and
 * P s = b (eq. 4.1) is solved exactly by the nonsymmetric fast diagonalization of
 * eq. 4.7 / 4.9 from the pencil factors of eq. 4.6.
 *
 * Conventions used by every entry point:
 *  - Unknowns are numbered with i_1 fastest (Sec. 2.1, after eq. 2.3): a vector of
 *    length N = n_1 n_2 (n_3) is the row-major array X[i_d]...[i_2][i_1].
 *    Direction index l is 0-based here: l = 0 is i_1.
 *  - Dense matrices are row-major: F[i*n + j] = (F)_{ij}.
 *  - Every function returns an int status (fdg_status); nothing else crosses the ABI
 *    as an error.  A negative value is an error and leaves outputs unspecified.
 *    fdg_last_error() gives a message for the most recent error in the calling thread.
 *  - "host" pointers are ordinary CPU memory, read during the call and never kept.
 *    "device" pointers are HIP device memory (e.g. a torch tensor's data_ptr()),
 *    owned by the caller; calls on a context are ordered on the context's HIP stream
 *    and device inputs must not alias device outputs.
 *  - A context is not thread-safe; use one context per thread/stream.
 */
#ifndef FDGMRES_H
#define FDGMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FDG_OK = 0,
  FDG_NOT_CONVERGED = 1,  /* solve ran out of iterations; x holds the last iterate        */
  FDG_EINVAL = -1,        /* bad argument (size, pointer, malformed CSR, non-finite data)   */
  FDG_ENOMEM = -2,        /* device allocation failed                                      */
  FDG_EHIP = -3,          /* a HIP runtime call failed                                     */
  FDG_ECOMPLEX = -4,      /* pencil eigenvalues not real and positive (Remark 1 violated)  */
  FDG_ENOTREADY = -5,     /* factors or operator missing for the requested call            */
  FDG_ENOCONV = -6,       /* host eigen-iteration did not converge                         */
  FDG_EFULL = -7          /* server: no free slot or arena space for the request right now  */
} fdg_status;

typedef enum {
  FDG_PREC_FP64 = 0,      /* P^{-1} in FP64 (exact up to rounding)                          */
  FDG_PREC_FP32 = 1,      /* factors and mode products in FP32                              */
  FDG_PREC_BF16 = 2       /* BF16 factors and inputs, FP32 accumulation and intermediates   */
} fdg_prec;

enum {
  FDG_SOLVE_USE_X0 = 1,       /* start from the x passed in instead of 0                     */
  FDG_SOLVE_FIXED_ITERS = 2,  /* run exactly maxit inner iterations, ignore rtol in a cycle  */
  FDG_SOLVE_NO_AHEAD = 4,     /* fdg_solve: do not queue Arnoldi steps ahead (same results)  */
  FDG_SOLVE_TIME_SPLIT = 8    /* fdg_solve: fill the device time split in the info, from the kernel
                                 timers (it reads and resets them; each timed launch leaves the
                                 queue idle for a few microseconds, so the solve is slower) */
};

typedef struct {
  int iterations;        /* inner (Arnoldi) iterations performed                           */
  int restarts;          /* completed cycles                                               */
  int converged;         /* 1 iff ||b - A x|| <= rtol ||b||                                 */
  int breakdown;         /* 1 if the last cycle ended on h_{j+1,j} <= 1e-14 ||A z_j||       */
  double rel_res_est;    /* |g_{j+1}| / ||b|| after the last iteration                      */
  double rel_res_true;   /* ||b - A x||_2 / ||b||_2, recomputed in FP64 at the end          */
  double ms_total;       /* wall time of the call, host clock                               */
  int half_steps;        /* BiCGStab: half steps done (the paper's count is half_steps / 2,
                            "k + 0.5" when the last iteration stopped after its BiCG half);
                            0 for flexible GMRES                                           */
  double t_apply_ms;     /* fdg_solve with FDG_SOLVE_TIME_SPLIT: device time of the P^{-1}
                            applies (HIP events around their kernels); 0 otherwise         */
  double t_matvec_ms;    /* the same for the operator matvecs (true residuals included)    */
  double t_orth_ms;      /* the same for the Gram-Schmidt and other vector kernels         */
  double t_host_ms;      /* fdg_solve: host time spent on the Givens least-squares update,
                            the choice of the next phase and its launches (always set)    */
} fdg_info;

/* ------------------------------------------------------------------------------------
 * Host-only setup.  These touch no GPU and may be called without one.
 * ---------------------------------------------------------------------------------- */

/* Univariate collocation factors of eq. 2.8 for degree p >= 1 and n >= max(p-1, 1)
 * interior unknowns: open uniform knot vector with E = n + 2 - p spans (Sec. 2.1),
 * Greville points of the interior functions (eq. 2.4).
 *   M[i*n+j]  = B_j(tau_i),  K[i*n+j] = -B_j''(tau_i),  D1[i*n+j] = B_j'(tau_i)  (host, n*n)
 *   tau[i]    = tau_i                                                             (host, n)
 * Any output pointer may be NULL.  Errors: FDG_EINVAL for bad p, n. */
int fdg_colloc_factors(int p, int n, double *M, double *K, double *D1, double *tau);

/* Nonsymmetric FD factors of one pencil (eq. 4.6 and the definition of V after it):
 * K U = M U diag(lambda), V = (M U)^{-T}.  Eigenvalues ascending, columns of U of unit
 * 2-norm.  K, M: host n*n input; U, V: host n*n output; lambda: host n output.
 * cond_u (may be NULL) receives the 1-norm condition number of U.
 * Errors: FDG_EINVAL (bad n, singular M or M U), FDG_ECOMPLEX (an eigenvalue with a
 * relative imaginary part above 1e-10 or a non-positive real part), FDG_ENOCONV. */
int fdg_factor_pencil(int n, const double *K, const double *M,
                      double *U, double *V, double *lambda, double *cond_u);

/* The same factorization for a pencil whose eigenvalues may include complex-conjugate
 * pairs (Sec. 4, the remark after eq. 4.7: D then has 2 x 2 real blocks).  A pair
 * a +- ib occupies two adjacent columns c, c+1 of U, holding the real and imaginary parts
 * of the eigenvector of a + ib (z = u + i v, phase chosen so u and v are orthogonal,
 * |u|^2 + |v|^2 = 1); lambda[c] = lambda[c+1] = a, mu[c] = b > 0, mu[c+1] = -b, so that
 * K U = M U D with D's block [[a, b], [-b, a]] at (c, c+1).  Real eigenvalues have
 * mu = 0.  Units (a real eigenvalue or a pair) in ascending order of real part.  V, U,
 * lambda, mu: host n*n, n*n, n, n outputs.  Errors as fdg_factor_pencil, with FDG_ECOMPLEX
 * only for a non-positive real part. */
int fdg_factor_pencil_blocks(int n, const double *K, const double *M, double *U, double *V,
                             double *lambda, double *mu, double *cond_u);

/* Symmetric FD factors (Sec. 4, after eq. 4.6) of a pencil with K symmetric and M
 * symmetric positive definite (e.g. the Galerkin factors of eq. 3.8): K U = M U
 * diag(lambda) with U^T M U = I, so that V = (M U)^{-T} = U.  Eigenvalues ascending.
 * K, M: host n*n input (symmetric to 1e-12 relative); U: host n*n output; lambda: host n.
 * Errors: FDG_EINVAL (bad n, not symmetric, M not positive definite), FDG_ECOMPLEX (an
 * eigenvalue <= 0), FDG_ENOCONV. */
int fdg_factor_pencil_sym(int n, const double *K, const double *M, double *U, double *lambda);

/* Univariate Galerkin factors of Sec. 3.2 (eq. 3.8 and the convection factor after
 * eq. 3.9) for degree p and n interior functions on the open uniform knot vector with
 * E = n + 2 - p spans, by (p+1)-point Gauss quadrature on every span:
 *   M[i*n+j] = int B_i B_j,  K[i*n+j] = int B_i' B_j',  H[i*n+j] = int w(z) B_i B_j'
 * with the affine univariate wind w(z) = w0 + w1 z (exact for this rule).  Host n*n
 * outputs, any may be NULL.  Errors: FDG_EINVAL. */
int fdg_galerkin_factors(int p, int n, double w0, double w1, double *M, double *K, double *H);

/* Galerkin matrix (Sec. 3.2) of -Lap u + w . grad u, homogeneous Dirichlet, on the
 * deformed cube of fdg_deformed_csr (amp = 0: the unit cube), pulled back to the
 * parametric cube and integrated with the tensor (p+1)^3-point Gauss rule of every
 * element:  A_ij = sum_q omega_q [grad B_i^T Q grad B_j + B_i b^T grad B_j](xi_q),
 * Q = det(J) J^{-1} J^{-T} (eq. 2.10, K = I), b = det(J) J^{-1} w(F(xi)), with
 *   w_a(x) = c_a (1 + x_a) (1 + beta cos(2 pi x_{a+1}) cos(2 pi x_{a+2}))  (cyclic a),
 * c = wind[0..2] (NULL: no convection).  Rows = test functions, i_1 fastest; the pattern
 * is every column with |j_l - i_l| <= p (the (2p+1)^3 stencil, clipped at the boundary),
 * columns ascending.  Call with rowptr/col/val NULL to get *nnz; then pass arrays of
 * n^3+1, *nnz, *nnz.  Uses up to 16 host threads. */
int fdg_galerkin_csr(int p, int n, double amp, const double *wind, double beta, int64_t *nnz,
                     int64_t *rowptr, int32_t *col, double *val);

/* Collocation matrix of -Laplace on the deformed cube F([0,1]^3) with
 * F_a(xi) = xi_a + amp sin(2 pi xi_{a+1}) sin(2 pi xi_{a+2}) (cyclic a), degree p,
 * n unknowns per direction, in CSR (rows = collocation points, i_1 fastest).
 * The general-geometry matrix of Sec. 2.2 is built from the chain rule
 *   -Lap u = -sum_kl C_kl d_k d_l u^ - sum_k g_k d_k u^,  C = J^{-1}J^{-T},
 *   g = -J^{-1} sum_lm (d_l d_m F) C_lm.
 * band = 0 stores the true pattern (B-splines whose support holds the point);
 * band = 1 stores every column with |j_l - i_l| <= p in each direction (explicit zeros
 * included: the (2p+1)^3 stencil).
 * Call with rowptr/col/val NULL to get *nnz; then pass arrays of n^3+1, *nnz, *nnz. */
int fdg_deformed_csr(int p, int n, double amp, int band, int64_t *nnz,
                     int64_t *rowptr, int32_t *col, double *val);

/* f = d pi^2 prod_l sin(pi tau_{i_l}) on the unit domain (u = prod sin(pi x_l)),
 * i_1 fastest.  tau: host n; f: host n^d. */
int fdg_manufactured_rhs(int d, int n, const double *tau, double *f);

/* ------------------------------------------------------------------------------------
 * Device context.
 * ---------------------------------------------------------------------------------- */
typedef struct fdg_ctx fdg_ctx;

/* d in {2, 3}; n[l] the unknowns in direction l (all equal, 1 <= n <= 1024);
 * batch >= 1 independent same-shape problems stored back to back (vector length
 * batch * N); hip_stream a hipStream_t (NULL = default stream) on which all work of
 * the context is ordered.  Uses the current HIP device. */
int fdg_create(fdg_ctx **ctx, int d, const int32_t *n, int batch, void *hip_stream);
int fdg_destroy(fdg_ctx *ctx);

/* Preconditioner factors of direction l (eq. 4.6): U, V host n*n row-major, lambda host
 * n, all real.  Copied to the device (FP64, plus FP32/BF16 copies, rounded to nearest
 * even).  Errors: FDG_EINVAL (bad l, non-finite), FDG_ECOMPLEX (some sum of eigenvalues
 * over the directions could be <= 0 -- checked once all directions are set). */
int fdg_set_prec_factors(fdg_ctx *ctx, int l, const double *U, const double *V,
                         const double *lambda);

/* FD factors of direction l from fdg_factor_pencil_blocks: as fdg_set_prec_factors, plus
 * mu (host n; NULL or all zero: real eigenvalues) marking complex pairs: mu[c] = b > 0,
 * mu[c+1] = -b, lambda[c] = lambda[c+1] = a for the block [[a, b], [-b, a]] of a +- ib.
 * The middle solve of eq. 4.9 then couples the two indices of every pair (a block solve
 * instead of a divide); such a context needs FDG_PREC_FP64 and is not batched by the
 * server.  Errors: FDG_EINVAL (malformed pairs), as fdg_set_prec_factors otherwise. */
int fdg_set_prec_factors_blocks(fdg_ctx *ctx, int l, const double *U, const double *V,
                                const double *lambda, const double *mu);

/* Symmetric FD factors of direction l (U from fdg_factor_pencil_sym): V = U. */
int fdg_set_prec_factors_sym(fdg_ctx *ctx, int l, const double *U, const double *lambda);

/* Arithmetic of the P^{-1} mode products (default FDG_PREC_FP64). */
int fdg_set_precision(fdg_ctx *ctx, int prec);

/* Operator A = unit-domain Kronecker sum (eq. 2.7 / 2.9) with factors M_l, K_l of
 * direction l: host n*n row-major, banded (stored by their row bands). */
int fdg_set_operator_kron(fdg_ctx *ctx, int l, const double *M, const double *K);

/* Operator A as a host CSR matrix of N rows (the same for every batch entry):
 * rowptr[N+1] (int64, rowptr[0] = 0, non-decreasing), col[nnz] (int32 in [0, N)),
 * val[nnz] (finite).  Copied to the device as a slot-major ELL matrix. */
int fdg_set_operator_csr(fdg_ctx *ctx, int64_t nrows, int64_t nnz, const int64_t *rowptr,
                         const int32_t *col, const double *val);

/* Operator A of a mapped 3D domain applied matrix-free (the collocation matrix of
 * Sec. 2.2 on F([0,1]^3), K = I, never assembled):
 *   (A x)_i = -sum_k C_kk (d_k^2 u)(tau_i) - sum_{k<l} 2 C_kl (d_k d_l u)(tau_i)
 *             - sum_k g_k (d_k u)(tau_i),       u = sum_j x_j B_j,
 * with C = J^{-1} J^{-T}, g = -J^{-1} sum_lm (d_l d_m F) C_lm at the collocation points.
 * The derivatives come from the univariate factors by sum factorization:
 * fdg_set_operator_mapped gives direction l's M_l (values), D_l (first derivatives) and
 * K_l (minus second derivatives) at the collocation points (host n*n row-major, banded,
 * band width <= 8); fdg_set_operator_fields gives the 9 coefficient fields, host
 * coef[f*N + i], f = 0..8: C_11, C_22, C_33, 2 C_12, 2 C_13, 2 C_23, g_1, g_2, g_3.
 * Both are copied to the device; the context then reads 9 N + 2 N doubles per matvec
 * instead of an assembled matrix. */
int fdg_set_operator_mapped(fdg_ctx *ctx, int l, const double *M, const double *D, const double *K);
int fdg_set_operator_fields(fdg_ctx *ctx, const double *coef);

/* The 9 coefficient fields above for the deformed cube of fdg_deformed_csr (degree p,
 * n unknowns per direction, amplitude amp): host coef[9 * n^3]. */
int fdg_deformed_coefficients(int p, int n, double amp, double *coef);

/* s = P^{-1} b (eq. 4.7 / 4.9) for every batch entry.  b, s: device, batch*N FP64. */
int fdg_apply_prec(fdg_ctx *ctx, const double *b, double *s);

/* Device bytes of the scratch array fdg_apply_prec_noalloc uses on each device. */
#define FDG_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): s = P^{-1} b exactly as
 * fdg_apply_prec (same kernels, same bits), with the intermediates between the FD
 * passes held in a file-scope device array of FDG_NOALLOC_SCRATCH_BYTES that every
 * device holds until the process ends, instead of the context's own workspace.  The
 * call allocates nothing (no hipMalloc, no events) and records no kernel timers.
 * Limit: two intermediates of batch*N doubles (FDG_PREC_FP64, or pencils with complex
 * pairs) or floats (FP32, BF16), each rounded up to 256 bytes plus 256 bytes of slack,
 * must fit in the array: batch*N <= 8388576 in FP64, <= 16777152 otherwise; larger
 * shapes fail with FDG_EINVAL and launch nothing.  All calls on one device share that
 * device's array: calls that overlap in time on one device (different streams, or
 * different host threads) race and must be serialized by the caller.  b, s: device,
 * batch*N FP64.  Errors as fdg_apply_prec, and FDG_EHIP if the array could not be
 * located on the device when the context was created. */
int fdg_apply_prec_noalloc(fdg_ctx *ctx, const double *b, double *s);

/* y = A x for every batch entry.  x, y: device, batch*N FP64. */
int fdg_matvec(fdg_ctx *ctx, const double *x, double *y);

/* Right-preconditioned flexible GMRES(restart) for A x = b, batch must be 1.
 * b, x: device, N FP64.  x0 = 0 unless flags has FDG_SOLVE_USE_X0.  Each cycle runs
 * classical Gram-Schmidt with one reorthogonalisation, Givens rotations in FP64 on the
 * host, x += Z y at its end and a true FP64 residual; converged iff
 * ||b - A x|| <= rtol ||b||.  With FDG_SOLVE_FIXED_ITERS exactly maxit iterations run.
 * While the residual estimate is well above the target, the next Arnoldi step is queued
 * before the host has read the current one (FDG_SOLVE_NO_AHEAD turns this off; the
 * results are the same bits either way).
 * Blocks until done.  Returns FDG_OK, FDG_NOT_CONVERGED, or an error.
 * info may be NULL. */
int fdg_solve(fdg_ctx *ctx, const double *b, double *x, double rtol, int restart,
              int maxit, int flags, fdg_info *info);

/* Right-preconditioned BiCGStab for A x = b (Sec. 5: the Krylov method of the paper's
 * experiments; van der Vorst's method: per iteration one BiCG half step with
 * p^ = P^{-1} p, then one GMRES(1) half step with s^ = P^{-1} s), batch must be 1.
 * b, x: device, N FP64.  x0 = 0 unless flags has FDG_SOLVE_USE_X0; shadow residual
 * r~ = r_0.  After each half step the recursively updated residual is compared with
 * rtol ||b||, and a pass is confirmed by the true FP64 residual ||b - A x||; converged
 * iff that holds.  info->iterations counts full iterations, info->half_steps half steps.
 * maxit bounds full iterations; with FDG_SOLVE_FIXED_ITERS exactly maxit run (no
 * convergence test).  A breakdown (r~.r = 0, r~.v = 0 or omega = 0) stops with the
 * current iterate, info->breakdown = 1 and FDG_NOT_CONVERGED.  Device memory: 8 N
 * doubles per context, allocated on first use.  Blocks until done. */
int fdg_bicgstab(fdg_ctx *ctx, const double *b, double *x, double rtol, int maxit, int flags,
                 fdg_info *info);

/* Bytes of operator data one matvec of the context reads (stored matrix slots, implicit
 * or explicit column indices, coefficient fields or factor bands; not x and y), 0 when
 * no operator is set.  An assembled operator whose pattern is the product of
 * per-direction windows on the tensor grid is stored without column indices (8 bytes
 * per slot); any other pattern as ELL (12 bytes per slot). */
size_t fdg_operator_bytes(const fdg_ctx *ctx);

/* Device bytes a context of this shape needs for a solve with the given restart
 * (factors, operator excluded for CSR, Krylov bases, scratch). */
size_t fdg_footprint_bytes(int d, int n, int batch, int prec, int restart);

/* Device memory the context owns now, as allocated: *held = everything (factors in
 * three precisions, operator data, solve and apply workspace); *workspace = the part
 * fdg_release_workspace would return (apply buffers, Krylov bases V and Z, reduction
 * partials, BiCGStab vectors; 0 while a caller's buffer is attached).  Either pointer may be NULL.  FDG_EINVAL for a NULL
 * context, FDG_EHIP if the runtime cannot size an allocation. */
int fdg_ctx_bytes(const fdg_ctx *ctx, size_t *held, size_t *workspace);

/* Waits for the context's stream, then frees its solve and apply workspace (device
 * buffers and the host-mapped scalar slots; an attached buffer is detached, not freed);
 * factors and operator stay.  The next apply, matvec or solve allocates them again, so a
 * cache of many contexts can bound the memory its idle ones hold.  Requests of the context already admitted to a server are not
 * affected (they use the server's arena).  FDG_EINVAL for a NULL context. */
int fdg_release_workspace(fdg_ctx *ctx);

/* Bytes of a buffer that fdg_attach_workspace accepts for contexts of this shape and
 * solves with restart <= the given one (apply buffers in FP64 and FP32, the flexible
 * GMRES bases V and Z sharing one region with the BiCGStab vectors, reduction partials),
 * 0 for an invalid shape. */
size_t fdg_workspace_bytes(int d, int n, int batch, int restart);

/* Makes the context carve its solve and apply workspace from a caller's device buffer of
 * `bytes` bytes (256-byte aligned, at least fdg_workspace_bytes(d, n, batch, restart))
 * instead of allocating its own, after waiting for its stream and freeing what it owned;
 * dev = NULL detaches (own allocations again on next use).  The buffer stays the
 * caller's: it must outlive the attachment and must not be written by anything else while
 * a call of the context runs.  Several contexts may share one buffer provided their calls
 * never overlap in time (fdg_solve and fdg_bicgstab return with the stream drained;
 * fdg_apply_prec and fdg_matvec do not, so order them on one stream or synchronize).
 * A solve with a restart above the attached one fails with FDG_EINVAL.  FDG_EINVAL for a
 * NULL context, a misaligned or too small buffer, or restart outside [1, 10000]. */
int fdg_attach_workspace(fdg_ctx *ctx, void *dev, size_t bytes, int restart);

/* Per-kernel timing with HIP events on the context stream for every launch of the named
 * kernel class while enabled (FD passes: events recorded by the kernel dispatch itself;
 * other classes: events around the launch).  kernel: 0 = FD slab passes (modes 1 and 2 of
 * eq. 4.9, or the whole 2D solve in two passes; for n > 256 every unfused mode product),
 * 1 = operator matvec, 2 = Krylov vector kernels, 3 = FD fibre pass (mode 3 with V_3^T,
 * the eigenvalue divide and mode 3 with U_3), 4 = the residual form of the unit-domain
 * matvec (r = b - A x with its squared-norm partials, used for true residuals).
 * fdg_timer_read returns the number of timed launches and their summed duration in
 * milliseconds, and resets the timer. */
int fdg_timer_enable(fdg_ctx *ctx, int kernel, int enable);
int fdg_timer_read(fdg_ctx *ctx, int kernel, int64_t *launches, double *total_ms);

/* ---- Request server: continuous batching of many solves on one device ------------------
 *
 * A server owns a device arena (one allocation at creation), a pool of host-mapped
 * pinned memory and `lanes` HIP streams (default priority, non-blocking).  A request is
 * an fdg_solve on a ready context (factors and operator set, batch 1, any d and n):
 * admission takes a free slot and run_bytes(ctx, restart) of the arena for its Krylov
 * bases and scratch, or fails with FDG_EFULL and changes nothing.  fdg_server_step
 * advances every lane whose previous work has completed: it reads each request's
 * host-mapped scalars, performs its FP64 Givens update (the same host arithmetic as
 * fdg_solve) and launches its next phase.  Requests on one lane that share a context
 * and are at the same kind of phase (even at different Arnoldi indices) go into ONE
 * launch per kernel through device pointer tables; requests of different shapes run
 * concurrently on different lanes.  Every request gives bit-for-bit the fdg_solve
 * result for the same (ctx, b, restart, rtol, maxit, flags): the per-entry arithmetic
 * and reduction order of every kernel do not depend on the other entries.
 * The caller keeps b, x and the context alive and unmodified until the request's
 * completion is returned.  Not thread-safe: one thread drives a server. */
typedef struct fdg_server fdg_server;

typedef struct {
  int64_t tag;       /* caller's tag given at admission                                   */
  int status;        /* FDG_OK, FDG_NOT_CONVERGED or an error of that request             */
  fdg_info info;     /* as from fdg_solve; ms_total runs from admission to completion     */
} fdg_done;

/* max_slots in [1, 4096] requests in flight, restart in [1, 255] for every request,
 * lanes in [1, 16] streams, arena_bytes of device memory. */
int fdg_server_create(fdg_server **srv, int max_slots, int restart, int lanes, size_t arena_bytes);
int fdg_server_destroy(fdg_server *srv);
/* Arena bytes one request on this context takes (0 for a NULL context). */
size_t fdg_server_run_bytes(const fdg_ctx *ctx, int restart);
/* Admit a request: b, x device N-vectors of ctx; rtol, maxit, flags as fdg_solve.  Its
 * first phase is launched by the next fdg_server_step. */
int fdg_server_admit(fdg_server *srv, fdg_ctx *ctx, const double *b, double *x, double rtol, int maxit,
                     int flags, int64_t tag);
/* Advance the lanes that are ready; wait up to wait_us microseconds (polling) for one to
 * become ready if none is.  Writes up to cap completed requests to done (completions
 * beyond cap are returned by later calls) and their count to *ndone. */
int fdg_server_step(fdg_server *srv, int wait_us, fdg_done *done, int cap, int *ndone);
/* Requests admitted and not yet returned as completed. */
int fdg_server_pending(const fdg_server *srv);
/* Counters since creation: lane services, phase groups launched, requests in those
 * groups, and the largest group. */
int fdg_server_stats(const fdg_server *srv, int64_t *services, int64_t *groups, int64_t *grouped_runs,
                     int64_t *max_group);

const char *fdg_status_str(int status);
const char *fdg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FDGMRES_H */
