// Internal definition of the device context shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "batch_addr.h"
#include "common.h"

namespace fdg {
constexpr int kTimerClasses = 5;

struct TimerState {
  bool on = false;
  std::vector<hipEvent_t> pool;     // free events
  std::vector<hipEvent_t> pending;  // start, stop, start, stop, ...
};

}  // namespace fdg

struct fdg_ctx {
  int d = 0, n = 0, batch = 1, device = 0;
  int64_t N = 0;
  hipStream_t stream = nullptr;
  int prec = FDG_PREC_FP64;
  // preconditioner factors, zero-padded ldw x ldw
  int ldw = 0;
  bool have_factor[3] = {false, false, false};
  double *Wv[3] = {nullptr, nullptr, nullptr};  // V_l^T: Y = W X applies V_l^T along mode l
  double *Wu[3] = {nullptr, nullptr, nullptr};  // U_l
  double *lam[3] = {nullptr, nullptr, nullptr};
  float *Wv32[3] = {nullptr, nullptr, nullptr}, *Wu32[3] = {nullptr, nullptr, nullptr};
  uint16_t *Wv16[3] = {nullptr, nullptr, nullptr}, *Wu16[3] = {nullptr, nullptr, nullptr};
  float *lam32[3] = {nullptr, nullptr, nullptr};
  double lam_min[3] = {0, 0, 0};
  // blocks of D_l (complex eigenvalue pairs are 2 x 2 blocks): imaginary parts, index
  // roles, block starts and block counts; kept for every direction with factors
  bool pairs[3] = {false, false, false};
  double *mu[3] = {nullptr, nullptr, nullptr};
  int8_t *role[3] = {nullptr, nullptr, nullptr};
  int32_t *bstart[3] = {nullptr, nullptr, nullptr};
  int nblocks[3] = {0, 0, 0};
  // operator
  int op_kind = 0;  // 0 none, 1 Kronecker bands, 2 ELL, 3 mapped (matrix-free)
  bool have_op[3] = {false, false, false};
  double *bandM[3] = {nullptr, nullptr, nullptr}, *bandK[3] = {nullptr, nullptr, nullptr};
  double *bandD[3] = {nullptr, nullptr, nullptr};  // first-derivative bands (mapped operator)
  double *fields = nullptr;                        // 9 N coefficient fields (mapped operator)
  bool have_fields = false;
  int32_t *bandlo[3] = {nullptr, nullptr, nullptr};
  int bandw[3] = {0, 0, 0};
  int bandrows4[3] = {0, 0, 0}, bandrows16[3] = {0, 0, 0}, bandstep[3] = {0, 0, 0};
  int32_t *ell_col = nullptr;
  double *ell_val = nullptr;
  int ell_width = 0;
  bool ell_tensor = false;       // implicit columns: windows lo_l, widths ell_tw (see set_operator_csr)
  int32_t *ell_lo = nullptr;     // 3 n window starts (direction-major)
  int ell_tw[3] = {1, 1, 1};
  // workspace
  double *t1 = nullptr, *t2 = nullptr;
  void *t32a = nullptr, *t32b = nullptr;
  int restart_alloc = 0;
  double *Vb = nullptr, *Zb = nullptr, *P1 = nullptr, *P2 = nullptr, *P3 = nullptr, *Hcol = nullptr,
         *hbuf = nullptr, *scal = nullptr;
  double *hpin = nullptr;      // pinned, device-mapped host memory for the scalars the host needs
  double *hpin_dev = nullptr;  // its device address
  hipEvent_t phase_ev = nullptr;  // end of a solve phase, polled by the host
  double *bicg = nullptr;          // BiCGStab vectors and partials (allocated on first use)
  double *bicg_host = nullptr;     // BiCGStab host-mapped scalars and its device address
  double *bicg_host_dev = nullptr;
  // workspace carved from a caller's buffer (fdg_attach_workspace) instead of owned:
  // the device pointers above then point into it and are never freed here
  char *ext_ws = nullptr;
  int ext_restart = 0;
  fdg::TimerState timers[fdg::kTimerClasses];
};

namespace fdg {

inline int hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return FDG_OK;
  if (e == hipErrorOutOfMemory) return set_error(FDG_ENOMEM, "%s: out of device memory", what);
  return set_error(FDG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(call)                                  \
  do {                                                \
    int _st = hip_check((call), #call);               \
    if (_st != FDG_OK) return _st;                    \
  } while (0)

template <typename T>
inline int dalloc(T **p, size_t count) {
  if (*p) return FDG_OK;
  return hip_check(hipMalloc((void **)p, count * sizeof(T) + 256), "hipMalloc");
}

template <typename T>
inline void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

// Brackets one launch of timer class c on stream s with events when that timer is on
// and the caller asks for timing.
struct TimedLaunch {
  fdg_ctx *ctx;
  int c;
  hipStream_t s;
  hipEvent_t stop = nullptr;
  TimedLaunch(fdg_ctx *x, int cls, hipStream_t st, bool want) : ctx(x), c(cls), s(st) {
    TimerState &t = ctx->timers[c];
    if (!want || !t.on) return;
    hipEvent_t a, b;
    if (t.pool.size() >= 2) {
      a = t.pool.back(); t.pool.pop_back();
      b = t.pool.back(); t.pool.pop_back();
    } else {
      // timing-only events: no system-scope fence (no cache write-back) when recorded
      if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return;
      if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
    }
    (void)hipEventRecord(a, s);
    t.pending.push_back(a);
    stop = b;
  }
  ~TimedLaunch() {
    if (!stop) return;
    (void)hipEventRecord(stop, s);
    ctx->timers[c].pending.push_back(stop);
  }
};

// Event pair for one kernel of timer class c, recorded by the kernel's own dispatch
// (hipExtLaunchKernel: no extra queue packets between kernels), when that timer is on
// and the caller asks for timing; start == nullptr otherwise.
struct DispatchTimer {
  hipEvent_t start = nullptr, stop = nullptr;
  DispatchTimer(fdg_ctx *ctx, int c, bool want) {
    TimerState &t = ctx->timers[c];
    if (!want || !t.on) return;
    hipEvent_t a, b;
    if (t.pool.size() >= 2) {
      a = t.pool.back(); t.pool.pop_back();
      b = t.pool.back(); t.pool.pop_back();
    } else {
      if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess) return;
      if (hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess) {
        (void)hipEventDestroy(a);
        return;
      }
    }
    t.pending.push_back(a);
    t.pending.push_back(b);
    start = a;
    stop = b;
  }
};

// Where a launch goes: the stream, and whether the context's kernel timers record it.
struct Exec {
  hipStream_t stream = nullptr;
  bool timed = false;
};

// Largest number of entries one gathered launch takes.
constexpr int kMaxGroupEntries = 64;

// P^{-1} for nent batch entries (entry e at in.at(e) / out.at(e)), with per-entry scratch
// t1, t2 (N doubles each) and, for a low-precision context, t32a, t32b (N floats each,
// contiguous over the entries).  A gathered batch (pointer tables) needs a context that
// groupable() accepts; strided batches take every path.  gathered_aligned32: every
// gathered entry pointer is 32-byte aligned (ignored for strided batches).
int apply_entries(fdg_ctx *c, const Exec &ex, CBatch in, MBatch out, int64_t nent, MBatch t1, MBatch t2,
                  void *t32a, void *t32b, bool gathered_aligned32);
// y = A x for nent batch entries, scratch t1, t2 as for apply_entries.
int matvec_entries(fdg_ctx *c, const Exec &ex, CBatch x, MBatch y, int64_t nent, MBatch t1, MBatch t2);
// r = b - A x with one partial sum of |r|^2 per workgroup written to part.at(e)[g],
// g < residual_partials(c); only for contexts where residual_partials(c) > 0.
int residual_entries(fdg_ctx *c, const Exec &ex, CBatch x, CBatch b, MBatch r, int64_t nent, MBatch part);
int residual_partials(const fdg_ctx *c);
// FDG_OK when the preconditioner factors and the operator are set, else FDG_ENOTREADY.
int ctx_ready(fdg_ctx *c);
// FDG_OK when the preconditioner factors of every direction are set, else FDG_ENOTREADY.
int ctx_ready_prec(fdg_ctx *c);
// Device address of the no-allocation apply's scratch array on device dev (current),
// looked up once per device; called when a context is created.
int scratch_setup(int dev);
// Number and summed duration (ms) of the timed launches of kernel timer class k since the
// last read, after the context stream has drained; resets the class.
int timer_collect(fdg_ctx *c, int k, int64_t *launches, double *total_ms);
// Some direction's pencil has complex eigenvalue pairs (block-diagonal D).
bool ctx_has_pairs(const fdg_ctx *c);
// Apply/matvec scratch t1, t2 (and t32a, t32b for a reduced-precision context).
int ensure_solve_workspace(fdg_ctx *c);
// The context's apply and matvec accept gathered batches (FP64 fused FD passes and a
// matvec form with per-entry scratch).
bool groupable(const fdg_ctx *c);

}  // namespace fdg
