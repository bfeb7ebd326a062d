// Device context of the C ABI: factor and operator upload, the preconditioner apply
// (eq. 4.7 / 4.9), the operator matvec, and the flexible GMRES driver (Sec. 3) whose
// Givens least-squares update runs in FP64 on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "bf16_round.h"
#include "common.h"
#include "context.h"
#include "fd_apply.h"
#include "mapped.h"
#include "kernels.h"
#include "modeprod.h"
#include "reduce.h"
#include "solve_run.h"

using namespace fdg;

namespace {

bool finite_all(const double *a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

int ensure_workspace(fdg_ctx *c) {
  const size_t tot = (size_t)c->N * c->batch;
  int st;
  if ((st = dalloc(&c->t1, tot)) != FDG_OK) return st;
  if ((st = dalloc(&c->t2, tot)) != FDG_OK) return st;
  return FDG_OK;
}

int ensure_lowp_workspace(fdg_ctx *c) {
  const size_t tot = (size_t)c->N * c->batch;
  int st;
  if ((st = dalloc((float **)&c->t32a, tot)) != FDG_OK) return st;
  if ((st = dalloc((float **)&c->t32b, tot)) != FDG_OK) return st;
  return FDG_OK;
}

int check_ready_prec(fdg_ctx *c) {
  for (int l = 0; l < c->d; ++l)
    if (!c->have_factor[l]) return set_error(FDG_ENOTREADY, "preconditioner factors of direction %d not set", l);
  return FDG_OK;
}

int check_ready_op(fdg_ctx *c) {
  if (c->op_kind == 1) {
    for (int l = 0; l < c->d; ++l)
      if (!c->have_op[l]) return set_error(FDG_ENOTREADY, "operator factors of direction %d not set", l);
    return FDG_OK;
  }
  if (c->op_kind == 2) return FDG_OK;
  if (c->op_kind == 3) {
    for (int l = 0; l < 3; ++l)
      if (!c->have_op[l]) return set_error(FDG_ENOTREADY, "mapped operator factors of direction %d not set", l);
    if (!c->have_fields) return set_error(FDG_ENOTREADY, "mapped operator coefficient fields not set");
    return FDG_OK;
  }
  return set_error(FDG_ENOTREADY, "operator not set");
}

inline bool al(const void *p, int bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; }

}  // namespace

namespace fdg {

int ctx_ready(fdg_ctx *c) {
  int st = check_ready_prec(c);
  if (st == FDG_OK) st = check_ready_op(c);
  return st;
}

int ctx_ready_prec(fdg_ctx *c) { return check_ready_prec(c); }

int ensure_solve_workspace(fdg_ctx *c) {
  int st = ensure_workspace(c);
  if (st == FDG_OK && c->prec != FDG_PREC_FP64) st = ensure_lowp_workspace(c);
  return st;
}

namespace {
KronBands ctx_bands(const fdg_ctx *c) {
  KronBands bd;
  for (int l = 0; l < 3; ++l) {
    const int q = l < c->d ? l : 0;
    bd.M[l] = c->bandM[q];
    bd.K[l] = c->bandK[q];
    bd.lo[l] = c->bandlo[q];
    bd.w[l] = c->bandw[q];
  }
  bd.rows4 = c->bandrows4[c->d == 3 ? 1 : 0];
  bd.rows16 = c->bandrows16[c->d == 3 ? 1 : 0];
  bd.step3 = c->bandstep[c->d == 3 ? 2 : 0];
  for (int l = 0; l < 3; ++l) bd.step[l] = c->bandstep[l < c->d ? l : 0];
  return bd;
}
}  // namespace

namespace {
MappedOp ctx_mapped(const fdg_ctx *c) {
  MappedOp op;
  for (int l = 0; l < 3; ++l) {
    op.M[l] = c->bandM[l];
    op.D[l] = c->bandD[l];
    op.K[l] = c->bandK[l];
    op.lo[l] = c->bandlo[l];
    op.w[l] = c->bandw[l];
    op.step[l] = c->bandstep[l];
  }
  op.coef = c->fields;
  op.N = c->N;
  return op;
}
}  // namespace

bool ctx_has_pairs(const fdg_ctx *c) {
  for (int l = 0; l < c->d; ++l)
    if (c->pairs[l]) return true;
  return false;
}

bool groupable(const fdg_ctx *c) {
  if (c->prec != FDG_PREC_FP64 || !fd_fused_supported(c->n) || ctx_has_pairs(c)) return false;
  if (c->op_kind == 2 || c->d == 2) return true;
  if (c->op_kind == 3) return mapped_matvec_ok(c->n, kMaxGroupEntries, ctx_mapped(c));
  int w = 0;
  for (int l = 0; l < c->d; ++l) w = std::max(w, c->bandw[l]);
  KronBands bd = ctx_bands(c);
  return kron_fused_ok(c->n, kMaxGroupEntries, bd) || kron_two_pass_ok(c->d, c->n, kMaxGroupEntries, bd);
}

namespace {

// P^{-1} when some D_l has 2 x 2 blocks (complex pairs, Sec. 4 after eq. 4.7): the mode
// products are those of the real case; the middle solve couples the two indices of a
// pair, across slabs and columns, so it runs as its own pass between the V^T and the U
// products (3D: fused slab pass for modes 1-2, mode-3 product, block solve, mode-3
// product, fused slab pass; 2D: slab pass, block solve, slab pass; n > 256: unfused).
int apply_blocks(fdg_ctx *c, const Exec &ex, CBatch in, MBatch out, int64_t nent, MBatch t1, MBatch t2,
                 bool gathered) {
  if (c->prec != FDG_PREC_FP64)
    return set_error(FDG_EINVAL, "apply: pencils with complex eigenvalue pairs need the FP64 preconditioner");
  if (gathered) return set_error(FDG_EINVAL, "apply: gathered batches need pencils with real eigenvalues");
  const int n = c->n;
  const int64_t n2 = (int64_t)n * n, B = nent;
  const double *b = in.base;
  double *s = out.base, *T1 = t1.base, *T2 = t2.base;
  BlockEig e[3];
  for (int l = 0; l < c->d; ++l) e[l] = BlockEig{c->lam[l], c->mu[l], c->role[l], c->bstart[l], c->nblocks[l]};
  TimedLaunch tl(c, 0, ex.stream, ex.timed);
  auto mode = [&](const double *X, double *Y, const double *W, int l) {
    if (l == 0)
      launch_modeprod_f64(ex.stream, X, Y, W, c->ldw, n, B * (c->d == 3 ? n2 : n), 0, 1, n, 1);
    else if (l == 1)
      launch_modeprod_f64(ex.stream, X, Y, W, c->ldw, n, n, n2, n, 1, B * (c->d == 3 ? n : 1));
    else
      launch_modeprod_f64(ex.stream, X, Y, W, c->ldw, n, n2, n2 * n, n2, 1, B);
  };
  const bool a32 = al(b, 32) && al(s, 32) && (nent == 1 || (in.stride % 4 == 0 && out.stride % 4 == 0));
  if (fd_fused_supported(n)) {
    if (c->d == 3) {
      launch_slab_f64(ex.stream, in, t1, c->Wv[0], c->Wv[1], c->ldw, n, nent, n, false, nullptr, nullptr, a32,
                      nullptr, nullptr);
      mode(T1, T2, c->Wv[2], 2);
      launch_blockdiv_f64(ex.stream, T2, T1, 3, n, B, e[0], e[1], e[2]);
      mode(T1, T2, c->Wu[2], 2);
      launch_slab_f64(ex.stream, as_const(t2), out, c->Wu[0], c->Wu[1], c->ldw, n, nent, n, false, nullptr,
                      nullptr, a32, nullptr, nullptr);
    } else {
      launch_slab_f64(ex.stream, in, t1, c->Wv[0], c->Wv[1], c->ldw, n, nent, 1, false, nullptr, nullptr, a32,
                      nullptr, nullptr);
      launch_blockdiv_f64(ex.stream, T1, T2, 2, n, B, e[0], e[1], e[1]);
      launch_slab_f64(ex.stream, as_const(t2), out, c->Wu[0], c->Wu[1], c->ldw, n, nent, 1, false, nullptr,
                      nullptr, a32, nullptr, nullptr);
    }
  } else if (c->d == 3) {
    mode(b, T1, c->Wv[0], 0);
    mode(T1, T2, c->Wv[1], 1);
    mode(T2, T1, c->Wv[2], 2);
    launch_blockdiv_f64(ex.stream, T1, T2, 3, n, B, e[0], e[1], e[2]);
    mode(T2, T1, c->Wu[0], 0);
    mode(T1, T2, c->Wu[1], 1);
    mode(T2, s, c->Wu[2], 2);
  } else {
    mode(b, T1, c->Wv[0], 0);
    mode(T1, T2, c->Wv[1], 1);
    launch_blockdiv_f64(ex.stream, T2, T1, 2, n, B, e[0], e[1], e[1]);
    mode(T1, T2, c->Wu[0], 0);
    mode(T2, s, c->Wu[1], 1);
  }
  return hip_check(hipGetLastError(), "apply_prec launch");
}

}  // namespace

int apply_entries(fdg_ctx *c, const Exec &ex, CBatch in, MBatch out, int64_t nent, MBatch t1, MBatch t2,
                  void *t32a, void *t32b, bool gathered_aligned32) {
  const int n = c->n;
  const int64_t N = c->N;
  const bool gathered = in.ptrs || out.ptrs || t1.ptrs || t2.ptrs;
  if (ctx_has_pairs(c)) return apply_blocks(c, ex, in, out, nent, t1, t2, gathered);
  if (c->prec == FDG_PREC_FP32 && fd_fused_supported(n)) {  // fused FP32 passes
    if (gathered) return set_error(FDG_EINVAL, "apply: gathered batches need the FP64 preconditioner");
    TimedLaunch tl(c, 0, ex.stream, ex.timed);
    launch_fd_apply_f32(ex.stream, c->d, n, nent, in.base, out.base, (float *)t32a, (float *)t32b, c->Wv32, c->Wu32,
                        c->lam32, c->ldw);
    return hip_check(hipGetLastError(), "apply_prec launch");
  }
  if (c->prec == FDG_PREC_BF16 && fd_fused_supported(n)) {  // fused BF16 passes
    if (gathered) return set_error(FDG_EINVAL, "apply: gathered batches need the FP64 preconditioner");
    TimedLaunch tl(c, 0, ex.stream, ex.timed);
    launch_fd_apply_bf16(ex.stream, c->d, n, nent, in.base, out.base, (float *)t32a, (float *)t32b,
                         (const void *const *)c->Wv16, (const void *const *)c->Wu16, c->lam32, c->ldw);
    return hip_check(hipGetLastError(), "apply_prec launch");
  }
  if (c->prec != FDG_PREC_FP64) {
    if (gathered) return set_error(FDG_EINVAL, "apply: gathered batches need the FP64 preconditioner");
    TimedLaunch tl(c, 0, ex.stream, ex.timed);
    return fd_apply_lowp(ex.stream, c->prec, c->d, n, nent, in.base, out.base, t32a, t32b,
                         c->prec == FDG_PREC_FP32 ? (const void *const *)c->Wv32 : (const void *const *)c->Wv16,
                         c->prec == FDG_PREC_FP32 ? (const void *const *)c->Wu32 : (const void *const *)c->Wu16,
                         c->lam32, c->ldw);
  }
  if (fd_fused_supported(n)) {
    // 32-byte aligned entries allow 4-wide loads (load width only; the arithmetic is the same)
    const bool a32 = in.ptrs || out.ptrs
                         ? gathered_aligned32
                         : al(in.base, 32) && al(out.base, 32) &&
                               (nent == 1 || (in.stride % 4 == 0 && out.stride % 4 == 0));
    if (c->d == 3) {
      {
        DispatchTimer tm(c, 0, ex.timed);
        launch_slab_f64(ex.stream, in, t1, c->Wv[0], c->Wv[1], c->ldw, n, nent, n, false, nullptr, nullptr, a32,
                        tm.start, tm.stop);
      }
      {
        DispatchTimer tm(c, 3, ex.timed);
        launch_fibre_f64(ex.stream, as_const(t1), t2, c->Wv[2], c->Wu[2], c->ldw, n, nent, c->lam[0], c->lam[1],
                         c->lam[2], tm.start, tm.stop);
      }
      {
        DispatchTimer tm(c, 0, ex.timed);
        launch_slab_f64(ex.stream, as_const(t2), out, c->Wu[0], c->Wu[1], c->ldw, n, nent, n, false, nullptr,
                        nullptr, a32, tm.start, tm.stop);
      }
    } else {
      {
        DispatchTimer tm(c, 0, ex.timed);
        launch_slab_f64(ex.stream, in, t1, c->Wv[0], c->Wv[1], c->ldw, n, nent, 1, true, c->lam[0], c->lam[1], a32,
                        tm.start, tm.stop);
      }
      {
        DispatchTimer tm(c, 0, ex.timed);
        launch_slab_f64(ex.stream, as_const(t1), out, c->Wu[0], c->Wu[1], c->ldw, n, nent, 1, false, nullptr,
                        nullptr, a32, tm.start, tm.stop);
      }
    }
    return hip_check(hipGetLastError(), "apply_prec launch");
  }
  if (gathered) return set_error(FDG_EINVAL, "apply: gathered batches need n <= 256");
  // unfused mode products over a contiguous batch (n > 256)
  const int64_t B = nent;
  const int64_t n2 = (int64_t)n * n;
  double *T1 = t1.base, *T2 = t2.base;
  const double *b = in.base;
  double *s = out.base;
  (void)N;
  auto mode = [&](const double *X, double *Y, const double *W, int l) {
    TimedLaunch tl(c, 0, ex.stream, ex.timed);
    if (l == 0) {
      const int64_t rows = B * (c->d == 3 ? n2 : n);
      launch_modeprod_f64(ex.stream, X, Y, W, c->ldw, n, rows, 0, 1, n, 1);
    } else if (l == 1) {
      const int64_t outer = B * (c->d == 3 ? n : 1);
      launch_modeprod_f64(ex.stream, X, Y, W, c->ldw, n, n, n2, n, 1, outer);
    } else {
      launch_modeprod_f64(ex.stream, X, Y, W, c->ldw, n, n2, n2 * n, n2, 1, B);
    }
  };
  if (c->d == 3) {
    mode(b, T1, c->Wv[0], 0);
    mode(T1, T2, c->Wv[1], 1);
    mode(T2, T1, c->Wv[2], 2);
    launch_divide_f64(ex.stream, T1, 3, n, B, c->lam[0], c->lam[1], c->lam[2]);
    mode(T1, T2, c->Wu[0], 0);
    mode(T2, T1, c->Wu[1], 1);
    mode(T1, s, c->Wu[2], 2);
  } else {
    mode(b, T1, c->Wv[0], 0);
    mode(T1, T2, c->Wv[1], 1);
    launch_divide_f64(ex.stream, T2, 2, n, B, c->lam[0], c->lam[1], nullptr);
    mode(T2, T1, c->Wu[0], 0);
    mode(T1, s, c->Wu[1], 1);
  }
  return hip_check(hipGetLastError(), "apply_prec launch");
}

int residual_partials(const fdg_ctx *c) {
  if (c->op_kind != 1) return 0;
  return kron_residual_partials(c->d, c->n, ctx_bands(c));
}

int residual_entries(fdg_ctx *c, const Exec &ex, CBatch x, CBatch b, MBatch r, int64_t nent, MBatch part) {
  TimedLaunch tl(c, 4, ex.stream, ex.timed);
  if (c->op_kind != 1 || !launch_kron_residual_f64(ex.stream, x, b, r, c->d, c->n, nent, ctx_bands(c), part))
    return set_error(FDG_EINVAL, "residual: the fused form does not apply to this operator");
  return hip_check(hipGetLastError(), "residual launch");
}

int matvec_entries(fdg_ctx *c, const Exec &ex, CBatch x, MBatch y, int64_t nent, MBatch t1, MBatch t2) {
  TimedLaunch tl(c, 1, ex.stream, ex.timed);
  if (c->op_kind == 2) {
    if (c->ell_tensor)
      launch_ell_tensor_f64(ex.stream, x, y, c->n, c->d, c->ell_tw, c->ell_lo, c->ell_val, nent);
    else
      launch_ell_matvec_f64(ex.stream, x, y, c->N, c->N, c->ell_width, c->ell_col, c->ell_val, nent);
    return hip_check(hipGetLastError(), "matvec launch");
  }
  if (c->op_kind == 3) {
    if (!launch_mapped_matvec_f64(ex.stream, x, y, c->n, nent, ctx_mapped(c)))
      return set_error(FDG_EINVAL, "matvec: mapped operator bands wider than 8 or growing by more than 1 per row");
    return hip_check(hipGetLastError(), "matvec launch");
  }
  const KronBands bd = ctx_bands(c);
  if (!launch_kron_matvec_f64(ex.stream, x, y, c->d, c->n, nent, bd, t1, t2))
    return set_error(FDG_EINVAL, "matvec: this operator shape needs a contiguous batch");
  return hip_check(hipGetLastError(), "matvec launch");
}

}  // namespace fdg

namespace {

// The context's own stream and workspace, for the apply / matvec entry points.
int ctx_apply(fdg_ctx *c, const double *b, double *s) {
  int st = ensure_workspace(c);
  if (st != FDG_OK) return st;
  if (c->prec != FDG_PREC_FP64 && (st = ensure_lowp_workspace(c)) != FDG_OK) return st;
  return apply_entries(c, Exec{c->stream, true}, cstrided(b, c->N), mstrided(s, c->N), c->batch,
                       mstrided(c->t1, c->N), mstrided(c->t2, c->N), c->t32a, c->t32b, false);
}

int ctx_matvec(fdg_ctx *c, const double *x, double *y) {
  int st = ensure_workspace(c);
  if (st != FDG_OK) return st;
  return matvec_entries(c, Exec{c->stream, true}, cstrided(x, c->N), mstrided(y, c->N), c->batch,
                        mstrided(c->t1, c->N), mstrided(c->t2, c->N));
}

}  // namespace

namespace {

int ensure_krylov(fdg_ctx *c, int m) {
  if (c->ext_ws) {  // bases carved at attach for restarts up to ext_restart; slots owned
    if (m > c->ext_restart)
      return set_error(FDG_EINVAL, "solve: restart %d exceeds the %d of the attached workspace", m,
                       c->ext_restart);
    if (c->hpin) return FDG_OK;
    HIPCHK(hipHostMalloc((void **)&c->hpin, sizeof(double) * 2 * (size_t)host_doubles(c->ext_restart) * c->batch,
                         hipHostMallocMapped));
    HIPCHK(hipHostGetDevicePointer((void **)&c->hpin_dev, c->hpin, 0));
    c->restart_alloc = c->ext_restart;
    return FDG_OK;
  }
  if (c->restart_alloc >= m) return FDG_OK;
  dfree(c->Vb); dfree(c->Zb); dfree(c->P1); dfree(c->P2); dfree(c->P3); dfree(c->Hcol);
  dfree(c->hbuf); dfree(c->scal);
  if (c->hpin) { (void)hipHostFree(c->hpin); c->hpin = nullptr; }
  c->restart_alloc = 0;
  const size_t NB = (size_t)c->N * c->batch;
  const int G = reduction_blocks(c->N);
  int st;
  if ((st = dalloc(&c->Vb, NB * (m + 1))) != FDG_OK) return st;
  if ((st = dalloc(&c->Zb, NB * m)) != FDG_OK) return st;
  if ((st = dalloc(&c->P1, (size_t)G * (m + 1) * c->batch)) != FDG_OK) return st;
  if ((st = dalloc(&c->P2, (size_t)G * (m + 1) * c->batch)) != FDG_OK) return st;
  if ((st = dalloc(&c->P3, (size_t)G * c->batch)) != FDG_OK) return st;
  if ((st = dalloc(&c->Hcol, (size_t)(m + 2) * c->batch)) != FDG_OK) return st;
  if ((st = dalloc(&c->hbuf, (size_t)2 * (m + 2) * c->batch)) != FDG_OK) return st;
  if ((st = dalloc(&c->scal, (size_t)4 * c->batch)) != FDG_OK) return st;
  // two banks of host-mapped slots: a speculative Arnoldi step writes the other bank
  HIPCHK(hipHostMalloc((void **)&c->hpin, sizeof(double) * 2 * (size_t)host_doubles(m) * c->batch,
                       hipHostMallocMapped));
  HIPCHK(hipHostGetDevicePointer((void **)&c->hpin_dev, c->hpin, 0));

  c->restart_alloc = m;
  return FDG_OK;
}


}  // namespace

// ------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------
extern "C" int fdg_create(fdg_ctx **out, int d, const int32_t *n, int batch, void *hip_stream) {
  clear_error();
  if (!out || !n) return set_error(FDG_EINVAL, "create: NULL argument");
  *out = nullptr;
  if (d != 2 && d != 3) return set_error(FDG_EINVAL, "create: d must be 2 or 3 (got %d)", d);
  for (int l = 0; l < d; ++l)
    if (n[l] != n[0]) return set_error(FDG_EINVAL, "create: all directions must have the same n");
  if (n[0] < 1 || n[0] > 1024) return set_error(FDG_EINVAL, "create: n must be in [1, 1024] (got %d)", n[0]);
  if (batch < 1) return set_error(FDG_EINVAL, "create: batch must be >= 1");
  const int64_t N = ipow(n[0], d);
  if (N * (int64_t)batch > ((int64_t)1 << 40)) return set_error(FDG_EINVAL, "create: problem too large");
  int dev = 0;
  int st = hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (st != FDG_OK) return st;
  // set-up of the no-allocation apply on this device (once per device); a failure is
  // reported by that entry point, not here
  (void)scratch_setup(dev);
  clear_error();
  fdg_ctx *c = new fdg_ctx();
  c->d = d;
  c->n = n[0];
  c->N = N;
  c->batch = batch;
  c->device = dev;
  c->stream = (hipStream_t)hip_stream;
  c->ldw = ((n[0] + 63) / 64) * 64;
  *out = c;
  return FDG_OK;
}

namespace {

// Apply buffers, Krylov bases, partials, BiCGStab vectors and the host-mapped slots; each
// is allocated again on its next use (dalloc skips only non-null pointers).  Carved
// pointers into an attached buffer are dropped, not freed.
void free_workspace(fdg_ctx *c) {
  if (c->ext_ws) {
    c->t1 = c->t2 = c->Vb = c->Zb = c->P1 = c->P2 = c->P3 = c->Hcol = c->hbuf = c->scal = c->bicg = nullptr;
    c->t32a = c->t32b = nullptr;
    c->ext_ws = nullptr;
    c->ext_restart = 0;
  } else {
    dfree(c->t1); dfree(c->t2);
    if (c->t32a) (void)hipFree(c->t32a);
    if (c->t32b) (void)hipFree(c->t32b);
    c->t32a = c->t32b = nullptr;
    dfree(c->Vb); dfree(c->Zb); dfree(c->P1); dfree(c->P2); dfree(c->P3); dfree(c->Hcol);
    dfree(c->hbuf); dfree(c->scal);
    dfree(c->bicg);
  }
  if (c->hpin) (void)hipHostFree(c->hpin);
  c->hpin = c->hpin_dev = nullptr;
  c->restart_alloc = 0;
  if (c->bicg_host) (void)hipHostFree(c->bicg_host);
  c->bicg_host = c->bicg_host_dev = nullptr;
}

// Adds the size of the device allocation at p (0 for NULL) to *sum.
int add_size(const void *p, size_t *sum) {
  if (!p) return FDG_OK;
  size_t sz = 0;
  int st = hip_check(hipMemPtrGetInfo(const_cast<void *>(p), &sz), "hipMemPtrGetInfo");
  if (st == FDG_OK) *sum += sz;
  return st;
}

// Byte offsets of the workspace regions in an attached buffer, each with the same 256
// bytes of slack as an owned allocation and 256-byte aligned.  The FGMRES bases (V, Z)
// and the BiCGStab vectors share one region: a context runs one call at a time and each
// call writes these vectors before reading them.
struct WsLayout {
  size_t t1, t2, t32a, t32b, krylov, zoff, P1, P2, P3, Hcol, hbuf, scal, total;
};

WsLayout ws_layout(int64_t N, int batch, int m) {
  WsLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 256 + 255) / 256 * 256;
    return at;
  };
  const size_t NB = (size_t)N * batch;
  const size_t G = (size_t)reduction_blocks(N);
  L.t1 = take(NB * 8);
  L.t2 = take(NB * 8);
  L.t32a = take(NB * 4);
  L.t32b = take(NB * 4);
  L.zoff = (NB * (m + 1) * 8 + 256 + 255) / 256 * 256;  // Z as aligned as an owned allocation
  L.krylov = take(std::max(L.zoff + NB * m * 8, (8 * (size_t)N + 8 * (size_t)kMaxG + 64) * 8));
  L.P1 = take(G * (m + 1) * batch * 8);
  L.P2 = take(G * (m + 1) * batch * 8);
  L.P3 = take(G * batch * 8);
  L.Hcol = take((size_t)(m + 2) * batch * 8);
  L.hbuf = take((size_t)2 * (m + 2) * batch * 8);
  L.scal = take((size_t)4 * batch * 8);
  L.total = off;
  return L;
}

}  // namespace

extern "C" int fdg_ctx_bytes(const fdg_ctx *c, size_t *held, size_t *workspace) {
  clear_error();
  if (!c) return set_error(FDG_EINVAL, "ctx_bytes: NULL context");
  size_t ws = 0, fixed = 0;
  int st = FDG_OK;
  if (!c->ext_ws)
    for (const void *p : {(const void *)c->t1, (const void *)c->t2, (const void *)c->t32a, (const void *)c->t32b,
                          (const void *)c->Vb, (const void *)c->Zb, (const void *)c->P1, (const void *)c->P2,
                          (const void *)c->P3, (const void *)c->Hcol, (const void *)c->hbuf,
                          (const void *)c->scal, (const void *)c->bicg})
      if (st == FDG_OK) st = add_size(p, &ws);
  for (int l = 0; l < 3 && st == FDG_OK; ++l)
    for (const void *p : {(const void *)c->Wv[l], (const void *)c->Wu[l], (const void *)c->lam[l],
                          (const void *)c->Wv32[l], (const void *)c->Wu32[l], (const void *)c->Wv16[l],
                          (const void *)c->Wu16[l], (const void *)c->lam32[l], (const void *)c->bandM[l],
                          (const void *)c->bandK[l], (const void *)c->bandD[l], (const void *)c->bandlo[l],
                          (const void *)c->mu[l], (const void *)c->role[l], (const void *)c->bstart[l]})
      if (st == FDG_OK) st = add_size(p, &fixed);
  for (const void *p : {(const void *)c->fields, (const void *)c->ell_col, (const void *)c->ell_val,
                        (const void *)c->ell_lo})
    if (st == FDG_OK) st = add_size(p, &fixed);
  if (st != FDG_OK) return st;
  if (held) *held = fixed + ws;
  if (workspace) *workspace = ws;
  return FDG_OK;
}

extern "C" int fdg_release_workspace(fdg_ctx *c) {
  clear_error();
  if (!c) return set_error(FDG_EINVAL, "release_workspace: NULL context");
  int st = hip_check(hipStreamSynchronize(c->stream), "release_workspace: hipStreamSynchronize");
  if (st != FDG_OK) return st;
  free_workspace(c);
  return FDG_OK;
}

extern "C" size_t fdg_workspace_bytes(int d, int n, int batch, int restart) {
  if ((d != 2 && d != 3) || n < 1 || n > 1024 || batch < 1 || restart < 1 || restart > 10000) return 0;
  return ws_layout(ipow(n, d), batch, restart).total;
}

extern "C" int fdg_attach_workspace(fdg_ctx *c, void *dev, size_t bytes, int restart) {
  clear_error();
  if (!c) return set_error(FDG_EINVAL, "attach_workspace: NULL context");
  if (dev && (restart < 1 || restart > 10000))
    return set_error(FDG_EINVAL, "attach_workspace: restart must be in [1, 10000] (got %d)", restart);
  if (dev && reinterpret_cast<uintptr_t>(dev) % 256 != 0)
    return set_error(FDG_EINVAL, "attach_workspace: buffer must be 256-byte aligned");
  const WsLayout L = ws_layout(c->N, c->batch, dev ? restart : 1);
  if (dev && bytes < L.total)
    return set_error(FDG_EINVAL, "attach_workspace: %zu bytes given, %zu needed", bytes, L.total);
  int st = hip_check(hipStreamSynchronize(c->stream), "attach_workspace: hipStreamSynchronize");
  if (st != FDG_OK) return st;
  free_workspace(c);
  if (!dev) return FDG_OK;  // detached: owned workspace again, allocated on next use
  char *w = static_cast<char *>(dev);
  c->t1 = reinterpret_cast<double *>(w + L.t1);
  c->t2 = reinterpret_cast<double *>(w + L.t2);
  c->t32a = w + L.t32a;
  c->t32b = w + L.t32b;
  c->Vb = reinterpret_cast<double *>(w + L.krylov);
  c->Zb = reinterpret_cast<double *>(w + L.krylov + L.zoff);
  c->bicg = c->Vb;
  c->P1 = reinterpret_cast<double *>(w + L.P1);
  c->P2 = reinterpret_cast<double *>(w + L.P2);
  c->P3 = reinterpret_cast<double *>(w + L.P3);
  c->Hcol = reinterpret_cast<double *>(w + L.Hcol);
  c->hbuf = reinterpret_cast<double *>(w + L.hbuf);
  c->scal = reinterpret_cast<double *>(w + L.scal);
  c->ext_ws = w;
  c->ext_restart = restart;
  return FDG_OK;
}

extern "C" int fdg_destroy(fdg_ctx *c) {
  clear_error();
  if (!c) return FDG_OK;
  (void)hipStreamSynchronize(c->stream);
  for (int l = 0; l < 3; ++l) {
    dfree(c->Wv[l]); dfree(c->Wu[l]); dfree(c->lam[l]);
    dfree(c->Wv32[l]); dfree(c->Wu32[l]); dfree(c->Wv16[l]); dfree(c->Wu16[l]); dfree(c->lam32[l]);
    dfree(c->bandM[l]); dfree(c->bandK[l]); dfree(c->bandD[l]); dfree(c->bandlo[l]);
    dfree(c->mu[l]); dfree(c->role[l]); dfree(c->bstart[l]);
  }
  dfree(c->fields);
  dfree(c->ell_col); dfree(c->ell_val); dfree(c->ell_lo);
  free_workspace(c);
  if (c->phase_ev) (void)hipEventDestroy(c->phase_ev);
  for (auto &t : c->timers) {
    for (auto e : t.pool) (void)hipEventDestroy(e);
    for (auto e : t.pending) (void)hipEventDestroy(e);
  }
  delete c;
  return FDG_OK;
}

namespace {

// Block structure of D_l on the device (mu, roles, block starts); mu NULL or all zero:
// n blocks of size 1.  The caller has validated mu.
int store_blocks(fdg_ctx *c, int l, const double *mu) {
  const int n = c->n;
  std::vector<int8_t> role(c->ldw, 0);
  std::vector<double> m(c->ldw, 0.0);
  std::vector<int32_t> start;
  bool any = false;
  for (int i = 0; i < n; ++i) {
    start.push_back(i);
    if (mu && mu[i] != 0.0) {
      role[i] = 1;
      role[i + 1] = 2;
      m[i] = mu[i];
      m[i + 1] = mu[i + 1];
      any = true;
      ++i;
    }
  }
  int st;
  if ((st = dalloc(&c->mu[l], (size_t)c->ldw)) != FDG_OK) return st;
  if ((st = dalloc(&c->role[l], (size_t)c->ldw)) != FDG_OK) return st;
  if ((st = dalloc(&c->bstart[l], (size_t)c->ldw)) != FDG_OK) return st;
  HIPCHK(hipMemcpy(c->mu[l], m.data(), m.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->role[l], role.data(), role.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->bstart[l], start.data(), start.size() * 4, hipMemcpyHostToDevice));
  c->nblocks[l] = (int)start.size();
  c->pairs[l] = any;
  return FDG_OK;
}

}  // namespace

extern "C" int fdg_set_prec_factors(fdg_ctx *c, int l, const double *U, const double *V, const double *lambda) {
  clear_error();
  if (!c || !U || !V || !lambda) return set_error(FDG_EINVAL, "set_prec_factors: NULL argument");
  if (l < 0 || l >= c->d) return set_error(FDG_EINVAL, "set_prec_factors: bad direction %d", l);
  const int n = c->n, ld = c->ldw;
  if (!finite_all(U, (size_t)n * n) || !finite_all(V, (size_t)n * n) || !finite_all(lambda, n))
    return set_error(FDG_EINVAL, "set_prec_factors: non-finite factor");
  double lmin = lambda[0];
  for (int i = 1; i < n; ++i) lmin = std::min(lmin, lambda[i]);
  std::vector<double> wv((size_t)ld * ld, 0.0), wu((size_t)ld * ld, 0.0), lm(ld, 1.0);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) {
      wv[(size_t)k * ld + j] = V[(size_t)j * n + k];
      wu[(size_t)k * ld + j] = U[(size_t)k * n + j];
    }
  for (int i = 0; i < n; ++i) lm[i] = lambda[i];
  int st;
  if ((st = dalloc(&c->Wv[l], wv.size())) != FDG_OK) return st;
  if ((st = dalloc(&c->Wu[l], wu.size())) != FDG_OK) return st;
  if ((st = dalloc(&c->lam[l], lm.size())) != FDG_OK) return st;
  HIPCHK(hipMemcpy(c->Wv[l], wv.data(), wv.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->Wu[l], wu.data(), wu.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->lam[l], lm.data(), lm.size() * 8, hipMemcpyHostToDevice));
  // reduced-precision copies (rounded once, to nearest even)
  std::vector<float> fv(wv.size()), fu(wu.size()), fl(lm.size());
  std::vector<uint16_t> bv(wv.size()), bu(wu.size());
  for (size_t i = 0; i < wv.size(); ++i) {
    fv[i] = (float)wv[i];
    fu[i] = (float)wu[i];
    bv[i] = bf16_bits_from_f64(wv[i]);
    bu[i] = bf16_bits_from_f64(wu[i]);
  }
  for (size_t i = 0; i < lm.size(); ++i) fl[i] = (float)lm[i];
  if ((st = dalloc(&c->Wv32[l], fv.size())) != FDG_OK) return st;
  if ((st = dalloc(&c->Wu32[l], fu.size())) != FDG_OK) return st;
  if ((st = dalloc(&c->Wv16[l], bv.size())) != FDG_OK) return st;
  if ((st = dalloc(&c->Wu16[l], bu.size())) != FDG_OK) return st;
  if ((st = dalloc(&c->lam32[l], fl.size())) != FDG_OK) return st;
  HIPCHK(hipMemcpy(c->Wv32[l], fv.data(), fv.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->Wu32[l], fu.data(), fu.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->Wv16[l], bv.data(), bv.size() * 2, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->Wu16[l], bu.data(), bu.size() * 2, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->lam32[l], fl.data(), fl.size() * 4, hipMemcpyHostToDevice));
  if ((st = store_blocks(c, l, nullptr)) != FDG_OK) return st;
  c->have_factor[l] = true;
  c->lam_min[l] = lmin;
  bool all = true;
  double sum = 0.0;
  for (int q = 0; q < c->d; ++q) {
    all = all && c->have_factor[q];
    sum += c->lam_min[q];
  }
  if (all && !(sum > 0.0)) {
    c->have_factor[l] = false;
    return set_error(FDG_ECOMPLEX, "set_prec_factors: eigenvalue sums can be <= 0");
  }
  return FDG_OK;
}

// Symmetric FD (Sec. 4, after eq. 4.6): U M-orthonormal, so V = U.  The first pass
// reads V^T row by row and the last reads U row by row, so the device keeps U in both
// layouts, as for a general pencil.
extern "C" int fdg_set_prec_factors_sym(fdg_ctx *c, int l, const double *U, const double *lambda) {
  return fdg_set_prec_factors(c, l, U, U, lambda);
}

// Nonsymmetric FD factors with complex eigenvalue pairs (Sec. 4, the remark after
// eq. 4.7): D_l block diagonal, 2 x 2 block [[lambda_c, mu_c], [mu_{c+1}, lambda_{c+1}]]
// = [[a, b], [-b, a]] for a pair.
extern "C" int fdg_set_prec_factors_blocks(fdg_ctx *c, int l, const double *U, const double *V,
                                           const double *lambda, const double *mu) {
  clear_error();
  if (!c || !U || !V || !lambda) return set_error(FDG_EINVAL, "set_prec_factors_blocks: NULL argument");
  if (l < 0 || l >= c->d) return set_error(FDG_EINVAL, "set_prec_factors_blocks: bad direction %d", l);
  const int n = c->n;
  if (mu) {
    for (int i = 0; i < n; ++i) {
      if (!std::isfinite(mu[i])) return set_error(FDG_EINVAL, "set_prec_factors_blocks: non-finite mu");
      if (mu[i] == 0.0) continue;
      if (!(mu[i] > 0.0) || i + 1 >= n || mu[i + 1] != -mu[i] || lambda[i + 1] != lambda[i])
        return set_error(FDG_EINVAL, "set_prec_factors_blocks: index %d does not start a pair "
                                     "(mu[c] > 0, mu[c+1] = -mu[c], lambda[c+1] = lambda[c])", i);
      ++i;
    }
  }
  int st = fdg_set_prec_factors(c, l, U, V, lambda);
  if (st != FDG_OK) return st;
  return store_blocks(c, l, mu);
}

extern "C" int fdg_set_precision(fdg_ctx *c, int prec) {
  clear_error();
  if (!c) return set_error(FDG_EINVAL, "set_precision: NULL context");
  if (prec != FDG_PREC_FP64 && prec != FDG_PREC_FP32 && prec != FDG_PREC_BF16)
    return set_error(FDG_EINVAL, "set_precision: unknown precision %d", prec);
  c->prec = prec;
  return FDG_OK;
}

namespace {

// Row bands of the univariate factors F[0..nf) of direction l (union of their non-zero
// patterns, one window [lo_i, lo_i + w) per row, non-decreasing lo) uploaded to the
// device as bandM, bandK (and bandD for three factors).
int store_bands(fdg_ctx *c, int l, const double *const *F, int nf, const char *who) {
  const int n = c->n;
  for (int f = 0; f < nf; ++f)
    if (!finite_all(F[f], (size_t)n * n)) return set_error(FDG_EINVAL, "%s: non-finite factor", who);
  std::vector<int> lo(n), hi(n);
  int w = 1;
  for (int i = 0; i < n; ++i) {
    int a = n, b = -1;
    for (int j = 0; j < n; ++j) {
      bool nz = false;
      for (int f = 0; f < nf; ++f) nz = nz || F[f][(size_t)i * n + j] != 0.0;
      if (nz) { a = std::min(a, j); b = std::max(b, j); }
    }
    if (b < 0) { a = 0; b = 0; }
    lo[i] = a;
    hi[i] = b;
    w = std::max(w, b - a + 1);
  }
  for (int i = 1; i < n; ++i)
    if (lo[i] < lo[i - 1]) return set_error(FDG_EINVAL, "%s: band starts must not decrease (row %d)", who, i);
  if (w > kron_window_max()) return set_error(FDG_EINVAL, "%s: band wider than %d", who, kron_window_max());
  std::vector<double> band[3];
  for (int f = 0; f < nf; ++f) band[f].assign((size_t)n * w, 0.0);
  std::vector<int32_t> blo(n);
  for (int i = 0; i < n; ++i) {
    const int s = std::min(lo[i], n - w);  // window [s, s+w) covers [lo, hi] and stays inside
    blo[i] = s;
    for (int f = 0; f < nf; ++f)
      for (int t = 0; t < w; ++t) band[f][(size_t)i * w + t] = F[f][(size_t)i * n + s + t];
  }
  double **dst[3] = {&c->bandM[l], &c->bandK[l], &c->bandD[l]};
  dfree(c->bandM[l]); dfree(c->bandK[l]); dfree(c->bandD[l]); dfree(c->bandlo[l]);
  int st;
  for (int f = 0; f < nf; ++f) {
    if ((st = dalloc(dst[f], band[f].size())) != FDG_OK) return st;
    HIPCHK(hipMemcpy(*dst[f], band[f].data(), band[f].size() * 8, hipMemcpyHostToDevice));
  }
  if ((st = dalloc(&c->bandlo[l], blo.size())) != FDG_OK) return st;
  HIPCHK(hipMemcpy(c->bandlo[l], blo.data(), blo.size() * 4, hipMemcpyHostToDevice));
  c->bandw[l] = w;
  int rows4 = 0;
  for (int i = 0; i < n; ++i) rows4 = std::max(rows4, blo[std::min(i + 3, n - 1)] + w - blo[i]);
  c->bandrows4[l] = rows4;
  int rows16 = 0, step = 0;
  for (int i = 0; i < n; i += 16) rows16 = std::max(rows16, blo[std::min(i + 15, n - 1)] + w - blo[i]);
  for (int i = 0; i + 1 < n; ++i) step = std::max(step, blo[i + 1] - blo[i]);
  c->bandrows16[l] = rows16;
  c->bandstep[l] = step;
  c->have_op[l] = true;
  return FDG_OK;
}

}  // namespace

extern "C" int fdg_set_operator_kron(fdg_ctx *c, int l, const double *M, const double *K) {
  clear_error();
  if (!c || !M || !K) return set_error(FDG_EINVAL, "set_operator_kron: NULL argument");
  if (l < 0 || l >= c->d) return set_error(FDG_EINVAL, "set_operator_kron: bad direction %d", l);
  if (c->op_kind == 2 || c->op_kind == 3)
    return set_error(FDG_EINVAL, "set_operator_kron: context already has another operator");
  const double *F[2] = {M, K};
  const int st = store_bands(c, l, F, 2, "set_operator_kron");
  if (st != FDG_OK) return st;
  c->op_kind = 1;
  return FDG_OK;
}

extern "C" int fdg_set_operator_mapped(fdg_ctx *c, int l, const double *M, const double *D, const double *K) {
  clear_error();
  if (!c || !M || !D || !K) return set_error(FDG_EINVAL, "set_operator_mapped: NULL argument");
  if (c->d != 3) return set_error(FDG_EINVAL, "set_operator_mapped: 3D contexts only");
  if (l < 0 || l >= 3) return set_error(FDG_EINVAL, "set_operator_mapped: bad direction %d", l);
  if (c->op_kind == 1 || c->op_kind == 2)
    return set_error(FDG_EINVAL, "set_operator_mapped: context already has another operator");
  const double *F[3] = {M, K, D};
  const int st = store_bands(c, l, F, 3, "set_operator_mapped");
  if (st != FDG_OK) return st;
  c->op_kind = 3;
  return FDG_OK;
}

extern "C" int fdg_set_operator_fields(fdg_ctx *c, const double *coef) {
  clear_error();
  if (!c || !coef) return set_error(FDG_EINVAL, "set_operator_fields: NULL argument");
  if (c->d != 3) return set_error(FDG_EINVAL, "set_operator_fields: 3D contexts only");
  if (c->op_kind == 1 || c->op_kind == 2)
    return set_error(FDG_EINVAL, "set_operator_fields: context already has another operator");
  const size_t cnt = (size_t)9 * c->N;
  if (!finite_all(coef, cnt)) return set_error(FDG_EINVAL, "set_operator_fields: non-finite coefficient");
  int st;
  if ((st = dalloc(&c->fields, cnt)) != FDG_OK) return st;
  HIPCHK(hipMemcpy(c->fields, coef, cnt * 8, hipMemcpyHostToDevice));
  c->have_fields = true;
  c->op_kind = 3;
  return FDG_OK;
}

namespace {

// True when row (i1, i2, i3) of the CSR couples exactly the columns (j1, j2, j3) with
// j_l in a window [a_l(i_l), b_l(i_l)] that depends on i_l alone, listed in ascending
// order (the pattern of every operator assembled on the tensor grid).  Returns the window
// starts shifted down so that lo + w <= n for the common widths w[l] = max window length
// (direction-major, 3 n entries; zeros for direction 3 in 2D), total slots <= 4096.
bool tensor_pattern(const fdg_ctx *c, const int64_t *rowptr, const int32_t *col, std::vector<int32_t> &lo,
                    int w[3]) {
  const int n = c->n, d = c->d;
  const int64_t N = c->N;
  std::vector<int> a((size_t)3 * n, n), b((size_t)3 * n, -1);
  auto split = [&](int64_t r, int (&i)[3]) {
    i[0] = (int)(r % n);
    i[1] = (int)((r / n) % n);
    i[2] = d == 3 ? (int)(r / ((int64_t)n * n)) : 0;
  };
  for (int64_t r = 0; r < N; ++r) {
    if (rowptr[r + 1] == rowptr[r]) return false;
    int i[3];
    split(r, i);
    for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
      int j[3];
      split(col[e], j);
      for (int l = 0; l < 3; ++l) {
        int &lo_l = a[(size_t)l * n + i[l]], &hi_l = b[(size_t)l * n + i[l]];
        lo_l = std::min(lo_l, j[l]);
        hi_l = std::max(hi_l, j[l]);
      }
    }
  }
  int64_t slots = 1;
  for (int l = 0; l < 3; ++l) {
    w[l] = 1;
    if (l >= d) continue;
    for (int i = 0; i < n; ++i) w[l] = std::max(w[l], b[(size_t)l * n + i] - a[(size_t)l * n + i] + 1);
    slots *= w[l];
  }
  if (slots > 4096) return false;
  for (int64_t r = 0; r < N; ++r) {  // each row must list its window product in order
    int i[3];
    split(r, i);
    int lo3[3], hi3[3];
    for (int l = 0; l < 3; ++l) {
      lo3[l] = l < d ? a[(size_t)l * n + i[l]] : 0;
      hi3[l] = l < d ? b[(size_t)l * n + i[l]] : 0;
    }
    int64_t e = rowptr[r];
    for (int j3 = lo3[2]; j3 <= hi3[2]; ++j3)
      for (int j2 = lo3[1]; j2 <= hi3[1]; ++j2)
        for (int j1 = lo3[0]; j1 <= hi3[0]; ++j1) {
          if (e >= rowptr[r + 1] || col[e] != j1 + (int64_t)n * (j2 + (int64_t)n * j3)) return false;
          ++e;
        }
    if (e != rowptr[r + 1]) return false;
  }
  lo.assign((size_t)3 * n, 0);
  for (int l = 0; l < d; ++l)
    for (int i = 0; i < n; ++i) lo[(size_t)l * n + i] = std::min(a[(size_t)l * n + i], n - w[l]);
  return true;
}

}  // namespace

extern "C" int fdg_set_operator_csr(fdg_ctx *c, int64_t nrows, int64_t nnz, const int64_t *rowptr,
                                    const int32_t *col, const double *val) {
  clear_error();
  if (!c || !rowptr || (nnz > 0 && (!col || !val))) return set_error(FDG_EINVAL, "set_operator_csr: NULL argument");
  if (c->op_kind == 1) return set_error(FDG_EINVAL, "set_operator_csr: context already has a Kronecker operator");
  if (nrows != c->N) return set_error(FDG_EINVAL, "set_operator_csr: nrows %lld != N %lld", (long long)nrows, (long long)c->N);
  if (rowptr[0] != 0 || rowptr[nrows] != nnz) return set_error(FDG_EINVAL, "set_operator_csr: rowptr ends do not match nnz");
  int width = 0;
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t len = rowptr[r + 1] - rowptr[r];
    if (len < 0) return set_error(FDG_EINVAL, "set_operator_csr: rowptr decreases at row %lld", (long long)r);
    if (len > 4096) return set_error(FDG_EINVAL, "set_operator_csr: row %lld longer than 4096", (long long)r);
    width = std::max(width, (int)len);
  }
  for (int64_t e = 0; e < nnz; ++e) {
    if (col[e] < 0 || col[e] >= nrows) return set_error(FDG_EINVAL, "set_operator_csr: column out of range at %lld", (long long)e);
    if (!std::isfinite(val[e])) return set_error(FDG_EINVAL, "set_operator_csr: non-finite value at %lld", (long long)e);
  }
  if (width == 0) width = 1;
  dfree(c->ell_col); dfree(c->ell_val); dfree(c->ell_lo);
  c->ell_tensor = false;
  int st;
  // A pattern that is the product of per-direction windows (every assembled operator of
  // this library: collocation and Galerkin stencils on the tensor grid) is stored with
  // implicit columns: 8 instead of 12 bytes per slot, and no dependent column load.
  std::vector<int32_t> tlo;
  int tw[3];
  if (tensor_pattern(c, rowptr, col, tlo, tw)) {
    const int64_t slots = (int64_t)tw[0] * tw[1] * tw[2];
    const size_t cnt = (size_t)slots * nrows;
    std::vector<double> ev(cnt, 0.0);
    const int n = c->n;
    for (int64_t r = 0; r < nrows; ++r) {
      const int i[3] = {(int)(r % n), (int)((r / n) % n), c->d == 3 ? (int)(r / ((int64_t)n * n)) : 0};
      for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const int64_t j = col[e];
        const int jj[3] = {(int)(j % n), (int)((j / n) % n), c->d == 3 ? (int)(j / ((int64_t)n * n)) : 0};
        int t[3];
        for (int l = 0; l < 3; ++l) t[l] = jj[l] - tlo[(size_t)l * n + i[l]];
        const int64_t slot = ((int64_t)t[2] * tw[1] + t[1]) * tw[0] + t[0];
        ev[(size_t)slot * nrows + r] = val[e];
      }
    }
    if ((st = dalloc(&c->ell_val, cnt)) != FDG_OK) return st;
    if ((st = dalloc(&c->ell_lo, tlo.size())) != FDG_OK) return st;
    HIPCHK(hipMemcpy(c->ell_val, ev.data(), cnt * 8, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->ell_lo, tlo.data(), tlo.size() * 4, hipMemcpyHostToDevice));
    for (int l = 0; l < 3; ++l) c->ell_tw[l] = tw[l];
    c->ell_tensor = true;
    c->ell_width = (int)slots;
    c->op_kind = 2;
    return FDG_OK;
  }
  const size_t cnt = (size_t)width * nrows;
  std::vector<int32_t> ec(cnt);
  std::vector<double> ev(cnt, 0.0);
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t b = rowptr[r], len = rowptr[r + 1] - b;
    for (int t = 0; t < width; ++t) {
      const size_t e = (size_t)t * nrows + r;
      if (t < len) {
        ec[e] = col[b + t];
        ev[e] = val[b + t];
      } else {
        ec[e] = (int32_t)r;  // padding: a valid column with a zero coefficient
      }
    }
  }
  if ((st = dalloc(&c->ell_col, cnt)) != FDG_OK) return st;
  if ((st = dalloc(&c->ell_val, cnt)) != FDG_OK) return st;
  HIPCHK(hipMemcpy(c->ell_col, ec.data(), cnt * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->ell_val, ev.data(), cnt * 8, hipMemcpyHostToDevice));
  c->ell_width = width;
  c->op_kind = 2;
  return FDG_OK;
}

extern "C" int fdg_apply_prec(fdg_ctx *c, const double *b, double *s) {
  clear_error();
  if (!c || !b || !s) return set_error(FDG_EINVAL, "apply_prec: NULL argument");
  if (b == s) return set_error(FDG_EINVAL, "apply_prec: input and output alias");
  int st = check_ready_prec(c);
  if (st != FDG_OK) return st;
  return ctx_apply(c, b, s);
}

extern "C" int fdg_matvec(fdg_ctx *c, const double *x, double *y) {
  clear_error();
  if (!c || !x || !y) return set_error(FDG_EINVAL, "matvec: NULL argument");
  if (x == y) return set_error(FDG_EINVAL, "matvec: input and output alias");
  int st = check_ready_op(c);
  if (st != FDG_OK) return st;
  return ctx_matvec(c, x, y);
}

extern "C" int fdg_solve(fdg_ctx *c, const double *b, double *x, double rtol, int restart, int maxit, int flags,
                         fdg_info *info) {
  clear_error();
  if (!c || !b || !x) return set_error(FDG_EINVAL, "solve: NULL argument");
  if (b == x) return set_error(FDG_EINVAL, "solve: b and x alias");
  if (c->batch != 1) return set_error(FDG_EINVAL, "solve: context batch must be 1");
  if (!(rtol >= 0.0) || restart < 1 || restart > 255 || maxit < 0)
    return set_error(FDG_EINVAL, "solve: bad rtol/restart/maxit");
  int st;
  if ((st = check_ready_prec(c)) != FDG_OK) return st;
  if ((st = check_ready_op(c)) != FDG_OK) return st;
  if ((st = ensure_workspace(c)) != FDG_OK) return st;
  if (c->prec != FDG_PREC_FP64 && (st = ensure_lowp_workspace(c)) != FDG_OK) return st;
  if ((st = ensure_krylov(c, restart)) != FDG_OK) return st;
  RunBufs rb;
  rb.V = c->Vb;
  rb.Z = c->Zb;
  rb.t1 = c->t1;
  rb.t2 = c->t2;
  rb.t32a = c->t32a;
  rb.t32b = c->t32b;
  rb.P1 = c->P1;
  rb.P2 = c->P2;
  rb.P3 = c->P3;
  rb.Hcol = c->Hcol;
  rb.h1 = c->hbuf;
  rb.scal = c->scal;
  rb.hh = c->hpin;
  rb.hh_dev = c->hpin_dev;
  if (!c->phase_ev) HIPCHK(hipEventCreateWithFlags(&c->phase_ev, hipEventDisableTiming));
  // device time split: every kernel timer class on for this solve (after clearing what
  // earlier launches left in them), the previous on/off states restored at the end
  const bool split = (flags & FDG_SOLVE_TIME_SPLIT) != 0;
  struct TimerRestore {  // puts the timer on/off states back on every way out
    fdg_ctx *c = nullptr;
    bool on[kTimerClasses] = {};
    ~TimerRestore() {
      if (c)
        for (int k = 0; k < kTimerClasses; ++k) c->timers[k].on = on[k];
    }
  } restore;
  if (split) {
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < kTimerClasses; ++k) restore.on[k] = c->timers[k].on;
    restore.c = c;
    for (int k = 0; k < kTimerClasses; ++k) {
      int64_t cnt;
      double ms;
      if ((st = timer_collect(c, k, &cnt, &ms)) != FDG_OK) return st;
      c->timers[k].on = true;
    }
  }
  double host_ms = 0.0;  // Givens updates, phase choice and launches
  auto host_clock = [] { return std::chrono::steady_clock::now(); };
  SolveRun run;
  run.init(c, rb, restart, b, x, rtol, maxit, flags);
  if (!(flags & FDG_SOLVE_NO_AHEAD)) run.bank_stride = (size_t)host_doubles(restart);
  SolveRun *rp = &run;
  const Exec ex{c->stream, true};
  bool stream_idle = true;
  bool queued = false;  // the current phase is already on the stream (an adopted speculation)
  Phase spec;
  bool spec_queued = false;
  while (!run.finished()) {
    auto h0 = host_clock();
    if (!queued) {
      // the previous phase's last kernel may still be retiring (its results were read);
      // the slots armed here are ones it has already written, so it cannot overwrite them
      run.arm();
      if ((st = enqueue_phase(ex, &rp, 1, nullptr)) != FDG_OK) return st;
    }
    // the next Arnoldi step needs nothing from the host: queue it behind this one (other
    // bank of slots) while the host waits, unless the cycle may end here
    if (!spec_queued && run.speculative(&spec)) {
      const Phase cur = run.phase();
      run.arm(spec);
      run.set_phase(spec);
      st = enqueue_phase(ex, &rp, 1, nullptr);
      run.set_phase(cur);
      if (st != FDG_OK) return st;
      spec_queued = true;
    }
    host_ms += std::chrono::duration<double, std::milli>(host_clock() - h0).count();
    HIPCHK(hipEventRecord(c->phase_ev, c->stream));
    stream_idle = false;
    // the host needs the phase's scalars, not the end of its last kernel: poll the armed
    // host-mapped slots, and the phase event every few rounds (no blocking wake-up)
    hipError_t e = hipErrorNotReady;
    for (unsigned k = 1; !run.ready(); ++k) {
      if ((k & 63) == 0 && (e = hipEventQuery(c->phase_ev)) != hipErrorNotReady) break;
    }
    if (e != hipErrorNotReady) {  // the stream finished first (or failed)
      (void)hipGetLastError();
      HIPCHK(e);
      stream_idle = true;
    }
    if (!run.ready()) {  // a phase without armed slots: its results need the whole stream
      while ((e = hipEventQuery(c->phase_ev)) == hipErrorNotReady) {
      }
      (void)hipGetLastError();
      HIPCHK(e);
      stream_idle = true;
    }
    const int consumed_bank = run.phase().bank;
    auto h1 = host_clock();
    run.consume();
    host_ms += std::chrono::duration<double, std::milli>(host_clock() - h1).count();
    // the next phase: the queued speculation when consume() chose the same step, else a
    // new phase in the bank just read (a discarded speculation still writes the other)
    Phase next = run.phase();
    queued = spec_queued && next.steps == spec.steps && next.j == spec.j;
    next.bank = queued ? spec.bank : consumed_bank;
    run.set_phase(next);
    spec_queued = false;  // adopted, or discarded (it runs ahead of the next phase, harmlessly)
  }
  if (!stream_idle) {  // x and the buffers belong to the caller again only after the stream
    hipError_t e;
    while ((e = hipEventQuery(c->phase_ev)) == hipErrorNotReady) {
    }
    (void)hipGetLastError();
    HIPCHK(e);
  }
  fdg_info out = run.info();
  out.t_host_ms = host_ms;
  if (split) {
    HIPCHK(hipStreamSynchronize(c->stream));
    double ms[kTimerClasses];
    for (int k = 0; k < kTimerClasses; ++k) {
      int64_t cnt;
      if ((st = timer_collect(c, k, &cnt, &ms[k])) != FDG_OK) return st;
    }
    out.t_apply_ms = ms[0] + ms[3];   // slab passes (or mode products) and fibre passes
    out.t_matvec_ms = ms[1] + ms[4];  // matvecs and fused residual matvecs
    out.t_orth_ms = ms[2];            // Gram-Schmidt and the other vector kernels
  }
  if (info) *info = out;
  return run.status();
}

extern "C" size_t fdg_operator_bytes(const fdg_ctx *c) {
  if (!c) return 0;
  const size_t N = (size_t)c->N;
  if (c->op_kind == 2) return (size_t)c->ell_width * N * (c->ell_tensor ? 8 : 12) + (c->ell_tensor ? 12 * (size_t)c->n : 0);
  if (c->op_kind == 3) return 9 * N * 8;
  if (c->op_kind == 1) {
    size_t b = 0;
    for (int l = 0; l < c->d; ++l) b += (size_t)c->n * c->bandw[l] * 16 + (size_t)c->n * 4;
    return b;
  }
  return 0;
}

extern "C" size_t fdg_footprint_bytes(int d, int n, int batch, int prec, int restart) {
  if ((d != 2 && d != 3) || n < 1 || batch < 1 || restart < 0) return 0;
  const size_t N = (size_t)ipow(n, d) * batch;
  const size_t ld = ((size_t)(n + 63) / 64) * 64;
  size_t bytes = 2 * N * 8;                       // apply ping-pong buffers
  if (prec != FDG_PREC_FP64) bytes += 2 * N * 4;  // low-precision intermediates
  bytes += (size_t)(2 * restart + 1) * N * 8;     // Krylov bases V (m+1) and Z (m)
  bytes += (size_t)d * (2 * ld * ld * (8 + 4 + 2) + ld * 12);  // factors in three precisions
  bytes += (size_t)reduction_blocks((int64_t)ipow(n, d)) * (2 * restart + 3) * 8 * batch + 4096;
  return bytes;
}

extern "C" int fdg_timer_enable(fdg_ctx *c, int kernel, int enable) {
  clear_error();
  if (!c || kernel < 0 || kernel >= kTimerClasses) return set_error(FDG_EINVAL, "timer_enable: bad argument");
  c->timers[kernel].on = enable != 0;
  return FDG_OK;
}

namespace fdg {

// Number and summed duration (ms) of the timed launches of class k since the last read;
// the stream must have drained.  Resets the class.
int timer_collect(fdg_ctx *c, int k, int64_t *launches, double *total_ms) {
  TimerState &t = c->timers[k];
  double sum = 0.0;
  int64_t cnt = 0;
  for (size_t i = 0; i + 1 < t.pending.size(); i += 2) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, t.pending[i], t.pending[i + 1]));
    sum += ms;
    ++cnt;
  }
  for (auto e : t.pending) t.pool.push_back(e);
  t.pending.clear();
  *launches = cnt;
  *total_ms = sum;
  return FDG_OK;
}

}  // namespace fdg

extern "C" int fdg_timer_read(fdg_ctx *c, int kernel, int64_t *launches, double *total_ms) {
  clear_error();
  if (!c || kernel < 0 || kernel >= kTimerClasses || !launches || !total_ms)
    return set_error(FDG_EINVAL, "timer_read: bad argument");
  HIPCHK(hipStreamSynchronize(c->stream));
  return timer_collect(c, kernel, launches, total_ms);
}
