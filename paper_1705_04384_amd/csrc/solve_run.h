// One flexible GMRES solve as a host-side state machine over device phases.
//
// A solve alternates between a phase of device work (kernels enqueued on a stream) and a
// host step that reads the few scalars the phase left in host-mapped memory (Hessenberg
// column, norms), updates the Givens least-squares problem in FP64 and chooses the next
// phase.  The single-solve entry point drives one run: it polls the phase's host-mapped
// slots (armed before the launch) rather than the stream, and may queue the next Arnoldi
// step before reading the current one (two banks of slots).  The request server drives
// many runs, one bank each, and launches the phases of runs that share a context and a
// step mask together (gathered batch entries).  Both use the same kernels with the same
// per-entry reduction order, so a solve gives the same bits alone or inside any mix.
#pragma once

#include <chrono>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "context.h"
#include "kernels.h"

namespace fdg {

// Device memory of one solve (N doubles each unless stated).
struct RunBufs {
  double *V = nullptr;                    // (m+1) N: Arnoldi basis
  double *Z = nullptr;                    // m N: preconditioned directions
  double *t1 = nullptr, *t2 = nullptr;    // apply / matvec scratch
  void *t32a = nullptr, *t32b = nullptr;  // low-precision apply scratch, N floats each
  double *P1 = nullptr, *P2 = nullptr;    // G (m+1) partial sums each
  double *P3 = nullptr;                   // G partial sums
  double *Hcol = nullptr, *h1 = nullptr;  // m+2 each
  double *scal = nullptr;                 // 2: ||b||, residual norm
  volatile double *hh = nullptr;          // host-mapped, host_doubles(m): see below
  double *hh_dev = nullptr;               // device address of hh
};

// Host-mapped doubles of one solve: Hessenberg column [0, m+2), ||b|| at m+2, and from
// m+4 the per-block partial sums of a squared norm (at most kHostPartials), which the
// host adds in block order.
constexpr int kHostPartials = 4096;
inline int host_doubles(int m) { return m + 4 + kHostPartials; }

// Device bytes of RunBufs for a solve on c with restart m (each piece 256-aligned).
size_t run_bytes(const fdg_ctx *c, int m);
// Carves RunBufs out of [base, base + run_bytes(...)); hh / hh_dev are set by the caller.
RunBufs carve_run(char *base, const fdg_ctx *c, int m);

// Steps of a phase, executed in this order.
enum : unsigned {
  kStepBDots = 1u << 0,    // P3 = partials of |b|^2
  kStepBNorm = 1u << 1,    // |b| -> scal[0], hh[m+2]
  kStepBScale = 1u << 2,   // V0 = b / |b|; |b| -> scal[0], hh[m+2]
  kStepLincomb = 1u << 3,  // x = (x or 0) + Z y
  kStepRes = 1u << 4,      // V0 = b - A x (via Z0 unless fused); |V0|^2 partials -> hh[m+4 ..]
  kStepScaleV = 1u << 5,   // V_j /= div (the norm the host formed from the partials)
  kStepIter = 1u << 6,     // Z_j = P^-1 V_j; w = V_{j+1} = A Z_j; CGS2; column -> hh,
                           // partials of |w|^2 -> hh[m+4 ..] (w is scaled by the next phase)
  kStepZeroX = 1u << 7,    // x = 0
  kStepScaleVDev = 1u << 8,  // V_j /= sqrt(sum of the |w|^2 partials in P3), formed on the device
};

struct Phase {
  unsigned steps = 0;      // 0: the solve is finished
  int j = 0;               // Arnoldi index of kStepIter / kStepScaleV
  int k = 0;               // coefficients of kStepLincomb
  bool overwrite = false;  // kStepLincomb starts from x = 0
  double div = 1.0;        // divisor of kStepScaleV
  int bank = 0;            // bank of host-mapped slots the phase writes (see bank_stride)
};

class SolveRun {
 public:
  // Binds a solve of A x = b (device vectors of ctx->N doubles) to its buffers and sets
  // the first phase.  Arguments are validated by the caller.
  void init(fdg_ctx *c, const RunBufs &bufs, int restart, const double *b, double *x, double rtol, int maxit,
            int flags);
  // The phase to enqueue next (or in flight).
  const Phase &phase() const { return ph_; }
  bool finished() const { return ph_.steps == 0; }
  // The phase in flight has completed (stream or event synchronised): read its results,
  // advance the least-squares state and set the next phase.
  void consume();
  // Host-mapped slots the phase about to be enqueued writes and consume() reads (the
  // Hessenberg column, ||b||, the per-block norm partials): arm() fills them with a
  // signalling-NaN pattern that no kernel stores (arithmetic yields quiet NaNs); ready()
  // is true once every armed slot holds a kernel's value, which a host can poll instead
  // of waiting for the end of the last kernel.  A phase without such slots arms nothing
  // and is never ready (wait for the stream instead).
  void arm() { arm(ph_); }
  void arm(const Phase &p);  // the slots of phase p (not necessarily the current one)
  bool ready() const;
  // The next Arnoldi step (v_{j+1} scaled on the device, then step j + 1) when the phase
  // in flight is step j and the host expects to continue the cycle after it: the caller
  // may enqueue it before reading step j's results, in the other bank of slots.  The
  // continuation is taken only while the residual estimate is well above the target, so
  // a step launched in vain (a cycle that ends after all) is rare.
  bool speculative(Phase *next) const;
  // Replaces the current phase (the caller enqueues a speculative phase, or adopts one
  // that consume() chose after all, with its bank).
  void set_phase(const Phase &p) { ph_ = p; }
  int status() const { return status_; }
  const fdg_info &info() const { return info_; }
  const Coeffs &coeffs() const { return y_; }

  fdg_ctx *ctx = nullptr;
  RunBufs buf;
  int m = 0;
  int64_t N = 0;
  int G = 0;
  int res_parts = 0;  // partials of the fused residual matvec, 0 if it does not apply
  // Host-mapped slots of bank k start at buf.hh + k * bank_stride (0: one bank, no
  // speculation; the request server uses one bank per run).
  size_t bank_stride = 0;
  volatile double *hh(int bank) const { return buf.hh + (size_t)bank * bank_stride; }
  double *hh_dev(int bank) const { return buf.hh_dev + (size_t)bank * bank_stride; }
  const double *b = nullptr;
  double *x = nullptr;

 private:
  double &Hij(int i, int jj) { return H_[(size_t)i * m + jj]; }
  double host_norm(int count) const;  // sqrt of the block-ordered sum of count partials in hh
  double tree_norm() const;           // sqrt of the G partials summed in the device's order
  void finish(bool converged);
  void zero_then_finish(bool converged);

  struct Armed {
    int hcol = 0, parts = 0;  // armed slots: hh[0, hcol), hh[m+4, m+4+parts)
    bool bnorm = false;       // and hh[m+2]
  };
  Armed armed_[2];
  Phase ph_;
  double rtol_ = 0.0, bnorm_ = -1.0, target_ = 0.0, last_est_ = 1.0, rbeta_ = 0.0;
  int limit_ = 0, total_ = 0, restarts_ = 0, status_ = FDG_OK;
  bool fixed_ = false, x_nonzero_ = false, breakdown_ = false, pending_conv_ = false;
  std::vector<double> H_, cs_, sn_, g_;
  Coeffs y_;
  fdg_info info_{};
  std::chrono::steady_clock::time_point t0_;
};

// Bump allocator over a pinned host staging buffer mirrored in device memory: pointer
// tables of gathered launches are written on the host and copied once per phase group.
struct TableArena {
  char *host = nullptr;
  char *dev = nullptr;
  size_t cap = 0, used = 0, flushed = 0;
  void reset() { used = flushed = 0; }
  // Host and device addresses of a fresh 16-byte aligned block, or false when full.
  bool alloc(size_t bytes, void **h, void **d);
  // Copies the blocks allocated since the last flush to the device on stream s.
  int flush(hipStream_t s);
};

// Enqueues the current phase of nrun runs (same context, same step mask; nrun <= the
// group limit) on ex.stream.  One run uses plain pointers; several use pointer tables
// from tab, which must then be non-null.
int enqueue_phase(const Exec &ex, SolveRun *const *runs, int nrun, TableArena *tab);

}  // namespace fdg
