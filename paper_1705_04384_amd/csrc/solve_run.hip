// Flexible GMRES (Sec. 3: right preconditioning by the FD solve of eq. 4.9) as a phase
// state machine, and the launcher of a phase for one run or a group of runs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "reduce.h"
#include "solve_run.h"

namespace fdg {

namespace {

inline size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }
inline bool al(const void *p, int bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; }

}  // namespace

size_t run_bytes(const fdg_ctx *c, int m) {
  const int64_t N = c->N;
  const bool lowp = c->prec != FDG_PREC_FP64;
  const size_t n8 = (size_t)N * 8;
  const int G = reduction_blocks(N);
  size_t s = up256(n8 * (m + 1)) + up256(n8 * m) + 2 * up256(n8);
  if (lowp) s += 2 * up256((size_t)N * 4);
  s += 2 * up256((size_t)G * (m + 1) * 8) + up256((size_t)G * 8);
  s += 2 * up256((size_t)(m + 2) * 8) + up256(2 * 8);
  return s;
}

RunBufs carve_run(char *base, const fdg_ctx *c, int m) {
  const int64_t N = c->N;
  const bool lowp = c->prec != FDG_PREC_FP64;
  const size_t n8 = (size_t)N * 8;
  const int G = reduction_blocks(N);
  RunBufs r;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *p = base + off;
    off += up256(bytes);
    return p;
  };
  r.V = (double *)take(n8 * (m + 1));
  r.Z = (double *)take(n8 * m);
  r.t1 = (double *)take(n8);
  r.t2 = (double *)take(n8);
  if (lowp) {
    r.t32a = take((size_t)N * 4);
    r.t32b = take((size_t)N * 4);
  }
  r.P1 = (double *)take((size_t)G * (m + 1) * 8);
  r.P2 = (double *)take((size_t)G * (m + 1) * 8);
  r.P3 = (double *)take((size_t)G * 8);
  r.Hcol = (double *)take((size_t)(m + 2) * 8);
  r.h1 = (double *)take((size_t)(m + 2) * 8);
  r.scal = (double *)take(2 * 8);
  return r;
}

// ------------------------------------------------------------------------------------
// Host side of one solve
// ------------------------------------------------------------------------------------
void SolveRun::init(fdg_ctx *c, const RunBufs &bufs, int restart, const double *bv, double *xv, double rtol,
                    int maxit, int flags) {
  ctx = c;
  buf = bufs;
  m = restart;
  N = c->N;
  G = reduction_blocks(N);
  res_parts = residual_partials(c);
  if (res_parts > kHostPartials) res_parts = 0;
  b = bv;
  x = xv;
  rtol_ = rtol;
  limit_ = maxit;
  fixed_ = (flags & FDG_SOLVE_FIXED_ITERS) != 0;
  x_nonzero_ = (flags & FDG_SOLVE_USE_X0) != 0;
  bnorm_ = -1.0;
  target_ = 0.0;
  last_est_ = 1.0;
  rbeta_ = 0.0;
  total_ = restarts_ = 0;
  breakdown_ = false;
  status_ = FDG_OK;
  H_.assign((size_t)(m + 1) * m, 0.0);
  cs_.assign(m, 0.0);
  sn_.assign(m, 0.0);
  g_.assign(m + 1, 0.0);
  std::memset(&info_, 0, sizeof(info_));
  t0_ = std::chrono::steady_clock::now();
  ph_ = Phase{};
  if (x_nonzero_) {
    // ||b||, then r = b - A x (||r|| decides whether to iterate)
    ph_.steps = kStepBDots | kStepBNorm | kStepRes;
  } else if (limit_ == 0) {
    ph_.steps = kStepBDots | kStepBNorm;  // nothing to iterate: x = 0
  } else {
    // x = 0: r = b, v0 = b / ||b||; ||b|| reaches the host with the first column
    ph_.steps = kStepBDots | kStepBScale | kStepIter;
    ph_.j = 0;
  }
}

void SolveRun::finish(bool converged) {
  info_.converged = converged ? 1 : 0;
  info_.iterations = total_;
  info_.restarts = restarts_;
  info_.breakdown = breakdown_ ? 1 : 0;
  info_.rel_res_est = last_est_;
  info_.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0_).count();
  status_ = converged ? FDG_OK : FDG_NOT_CONVERGED;
  ph_ = Phase{};
}

double SolveRun::host_norm(int count) const {
  const volatile double *h = hh(ph_.bank);
  double sum = 0.0;
  for (int g = 0; g < count; ++g) sum += h[m + 4 + g];
  return std::sqrt(sum);
}

// The order of sum_partials: lane l adds partials l, l + 64, l + 128, l + 192 to 0, then
// an xor butterfly over the 64 lanes.  The device scales v_{j+1} by the square root of
// this sum, and the Hessenberg entry is the same number.
double SolveRun::tree_norm() const {
  const volatile double *h = hh(ph_.bank) + m + 4;
  double v[64];
  for (int l = 0; l < 64; ++l) {
    double s = 0.0;
    for (int k = 0; k < kMaxG / 64; ++k) {
      const int g = l + 64 * k;
      s += g < G ? h[g] : 0.0;
    }
    v[l] = s;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    double t[64];
    for (int l = 0; l < 64; ++l) t[l] = v[l] + v[l ^ off];
    for (int l = 0; l < 64; ++l) v[l] = t[l];
  }
  return std::sqrt(v[0]);
}

namespace {
constexpr uint64_t kUnwritten = 0x7FF4DEADBEEF0001ull;  // signalling NaN: never a kernel result
}

void SolveRun::arm(const Phase &p) {
  const unsigned st = p.steps;
  Armed &a = armed_[p.bank];
  a = Armed{};
  if (st == 0 || (st & kStepZeroX)) return;
  if (st & (kStepBNorm | kStepBScale)) a.bnorm = true;
  if (st & kStepIter) {
    a.hcol = p.j + 1;
    a.parts = G;
  } else if (st & kStepRes) {
    a.parts = res_parts > 0 ? res_parts : G;
  }
  volatile uint64_t *w = reinterpret_cast<volatile uint64_t *>(hh(p.bank));
  for (int q = 0; q < a.hcol; ++q) w[q] = kUnwritten;
  if (a.bnorm) w[m + 2] = kUnwritten;
  for (int g = 0; g < a.parts; ++g) w[m + 4 + g] = kUnwritten;
}

bool SolveRun::ready() const {
  const Armed &a = armed_[ph_.bank];
  if (a.hcol == 0 && a.parts == 0 && !a.bnorm) return false;
  const volatile uint64_t *w = reinterpret_cast<const volatile uint64_t *>(hh(ph_.bank));
  for (int g = a.parts - 1; g >= 0; --g)
    if (w[m + 4 + g] == kUnwritten) return false;
  for (int q = 0; q < a.hcol; ++q)
    if (w[q] == kUnwritten) return false;
  return !a.bnorm || w[m + 2] != kUnwritten;
}

bool SolveRun::speculative(Phase *next) const {
  if (bank_stride == 0 || !(ph_.steps & kStepIter) || breakdown_) return false;
  const int j = ph_.j;
  if (j + 2 > m || total_ + 2 > limit_) return false;  // step j ends the cycle or the budget
  // estimates exist from the first consumed step on; margin 20 on the relative estimate
  if (!fixed_ && (total_ < 1 || !(last_est_ > 20.0 * rtol_))) return false;
  Phase p;
  p.steps = kStepScaleVDev | kStepIter;
  p.j = j + 1;
  p.bank = 1 - ph_.bank;
  *next = p;
  return true;
}

void SolveRun::zero_then_finish(bool converged) {
  pending_conv_ = converged;
  ph_ = Phase{};
  ph_.steps = kStepZeroX;
}

void SolveRun::consume() {
  const unsigned st = ph_.steps;
  if (st == 0) return;
  if (st & kStepZeroX) {
    finish(pending_conv_);
    return;
  }
  const volatile double *hb = hh(ph_.bank);
  auto learn_bnorm = [&]() {
    bnorm_ = hb[m + 2];
    target_ = rtol_ * bnorm_;
  };
  if (st & kStepRes) {  // true residual r = b - A x in V0, its norm from the partials
    if (bnorm_ < 0.0) learn_bnorm();
    const double beta = host_norm(res_parts > 0 ? res_parts : G);
    if (bnorm_ == 0.0) {  // b = 0: the solution is x = 0 exactly
      info_.rel_res_true = 0.0;
      last_est_ = 0.0;
      zero_then_finish(true);
      return;
    }
    rbeta_ = beta;
    info_.rel_res_true = beta / bnorm_;
    if ((!fixed_ && beta <= target_) || total_ >= limit_) {
      finish(rbeta_ <= target_);
      return;
    }
    std::fill(g_.begin(), g_.end(), 0.0);  // next cycle from v0 = r / ||r||
    g_[0] = beta;
    ph_ = Phase{};
    ph_.steps = kStepScaleV | kStepIter;
    ph_.j = 0;
    ph_.div = beta;
    return;
  }
  if (!(st & kStepIter)) {  // ||b|| only (no iteration allowed, x = 0)
    learn_bnorm();
    info_.rel_res_true = bnorm_ > 0.0 ? 1.0 : 0.0;
    last_est_ = 0.0;
    zero_then_finish(bnorm_ == 0.0);
    return;
  }
  // an Arnoldi step completed: Hessenberg column j in hh[0 .. j], |w|^2 partials
  const int j = ph_.j;
  if (bnorm_ < 0.0) {
    learn_bnorm();
    g_[0] = bnorm_;
    if (bnorm_ == 0.0) {
      info_.rel_res_true = 0.0;
      last_est_ = 0.0;
      zero_then_finish(true);
      return;
    }
  }
  const int nv = j + 1;
  for (int q = 0; q < nv; ++q) Hij(q, j) = hb[q];
  Hij(nv, j) = tree_norm();
  double wn0 = 0.0;
  for (int q = 0; q <= nv; ++q) wn0 += Hij(q, j) * Hij(q, j);
  wn0 = std::sqrt(wn0);
  const double hn = Hij(j + 1, j);
  for (int i = 0; i < j; ++i) {  // earlier rotations
    const double a = Hij(i, j), bb = Hij(i + 1, j);
    Hij(i, j) = cs_[i] * a + sn_[i] * bb;
    Hij(i + 1, j) = -sn_[i] * a + cs_[i] * bb;
  }
  {  // new rotation zeroing h_{j+1,j}
    const double a = Hij(j, j), bb = Hij(j + 1, j);
    if (bb == 0.0) {
      cs_[j] = 1.0;
      sn_[j] = 0.0;
    } else {
      const double r = std::hypot(a, bb);
      cs_[j] = a / r;
      sn_[j] = bb / r;
      Hij(j, j) = r;
    }
    Hij(j + 1, j) = 0.0;
  }
  g_[j + 1] = -sn_[j] * g_[j];
  g_[j] = cs_[j] * g_[j];
  ++total_;
  last_est_ = std::fabs(g_[j + 1]) / bnorm_;
  breakdown_ = hn <= 1e-14 * wn0;
  const bool end_cycle =
      total_ >= limit_ || breakdown_ || j + 1 >= m || (!fixed_ && std::fabs(g_[j + 1]) <= target_);
  if (!end_cycle) {  // v_{j+1} = w / h_{j+1,j} (the norm formed on the device), next step
    const int bank = ph_.bank;
    ph_ = Phase{};
    ph_.steps = kStepScaleVDev | kStepIter;
    ph_.j = j + 1;
    ph_.bank = bank;
    return;
  }
  const int k = j + 1;
  for (int i = k - 1; i >= 0; --i) {  // back-substitution R y = g
    double s = g_[i];
    for (int q = i + 1; q < k; ++q) s -= Hij(i, q) * y_.v[q];
    y_.v[i] = s / Hij(i, i);
  }
  ph_ = Phase{};
  ph_.steps = kStepLincomb | kStepRes;
  ph_.k = k;
  ph_.overwrite = !x_nonzero_;
  x_nonzero_ = true;
  ++restarts_;
}

// ------------------------------------------------------------------------------------
// Pointer tables
// ------------------------------------------------------------------------------------
bool TableArena::alloc(size_t bytes, void **h, void **d) {
  const size_t off = (used + 15) & ~(size_t)15;
  if (off + bytes > cap) return false;
  *h = host + off;
  *d = dev + off;
  used = off + bytes;
  return true;
}

int TableArena::flush(hipStream_t s) {
  if (used > flushed) {
    HIPCHK(hipMemcpyAsync(dev + flushed, host + flushed, used - flushed, hipMemcpyHostToDevice, s));
    flushed = used;
  }
  return FDG_OK;
}

namespace {

// Descriptors of one operand over the runs of a group: plain pointers for one run,
// a device pointer table otherwise.
struct Gather {
  SolveRun *const *runs;
  int n;
  TableArena *tab;
  bool full = false;

  template <class F>
  CBatch c(F f) {
    if (n == 1) return cstrided(f(*runs[0]), 0);
    void *h, *d;
    if (!tab->alloc(sizeof(void *) * n, &h, &d)) { full = true; return CBatch{}; }
    const double **hp = (const double **)h;
    for (int e = 0; e < n; ++e) hp[e] = f(*runs[e]);
    return cgather((const double *const *)d);
  }
  template <class F>
  MBatch m(F f) {
    if (n == 1) return mstrided(f(*runs[0]), 0);
    void *h, *d;
    if (!tab->alloc(sizeof(void *) * n, &h, &d)) { full = true; return MBatch{}; }
    double **hp = (double **)h;
    for (int e = 0; e < n; ++e) hp[e] = f(*runs[e]);
    return mgather((double *const *)d);
  }
  template <class F>
  IBatch i(F f) {
    if (n == 1) return IBatch{f(*runs[0]), nullptr};
    void *h, *d;
    if (!tab->alloc(sizeof(int32_t) * n, &h, &d)) { full = true; return IBatch{}; }
    int32_t *hp = (int32_t *)h;
    for (int e = 0; e < n; ++e) hp[e] = f(*runs[e]);
    return IBatch{0, (const int32_t *)d};
  }
  // Divisors of kStepScaleV, one per entry (several runs only).
  const double *dtab() {
    if (n == 1) return nullptr;
    void *h, *d;
    if (!tab->alloc(sizeof(double) * n, &h, &d)) { full = true; return nullptr; }
    double *hp = (double *)h;
    for (int e = 0; e < n; ++e) hp[e] = runs[e]->phase().div;
    return (const double *)d;
  }
  // Least-squares coefficients, 256 per entry (several runs only).
  const double *ytab() {
    if (n == 1) return nullptr;
    void *h, *d;
    if (!tab->alloc(sizeof(double) * 256 * n, &h, &d)) { full = true; return nullptr; }
    double *hp = (double *)h;
    for (int e = 0; e < n; ++e) {
      const int k = runs[e]->phase().k;
      std::memcpy(hp + (size_t)e * 256, runs[e]->coeffs().v, sizeof(double) * k);
    }
    return (const double *)d;
  }
};

}  // namespace

int enqueue_phase(const Exec &ex, SolveRun *const *runs, int nrun, TableArena *tab) {
  if (nrun < 1) return FDG_OK;
  if (nrun > kMaxGroupEntries || (nrun > 1 && !tab))
    return set_error(FDG_EINVAL, "enqueue_phase: bad group of %d runs", nrun);
  SolveRun &r0 = *runs[0];
  fdg_ctx *c = r0.ctx;
  const unsigned steps = r0.phase().steps;
  const int64_t N = r0.N;
  const int G = r0.G, m = r0.m, ldp = m + 1;
  hipStream_t s = ex.stream;
  (void)hipGetLastError();  // launches below are checked on their own

  if (steps & kStepZeroX) {
    for (int e = 0; e < nrun; ++e) HIPCHK(hipMemsetAsync(runs[e]->x, 0, sizeof(double) * N, s));
    return FDG_OK;
  }
  using R = const SolveRun &;
  Gather ga{runs, nrun, tab};
  // operands (built before any launch: one table copy per group)
  const CBatch B = ga.c([](R r) { return r.b; });
  const CBatch Vb = ga.c([](R r) { return (const double *)r.buf.V; });
  const MBatch V0 = ga.m([](R r) { return r.buf.V; });
  const MBatch T1 = ga.m([](R r) { return r.buf.t1; });
  const MBatch T2 = ga.m([](R r) { return r.buf.t2; });
  const MBatch P3 = ga.m([](R r) { return r.buf.P3; });
  const MBatch Sb = ga.m([](R r) { return r.buf.scal; });
  const MBatch Hb = ga.m([m](R r) { return r.hh_dev(r.phase().bank) + m + 2; });
  const MBatch Hp = ga.m([m](R r) { return r.hh_dev(r.phase().bank) + m + 4; });  // host-summed partials
  MBatch X, Z0, Vj, Zj, Vj1, P1, P2, H1, Hc, Hh;
  CBatch Zb;
  IBatch K, OW, NV;
  const double *ytab = nullptr, *dtab = nullptr;
  if (steps & (kStepLincomb | kStepRes)) {
    X = ga.m([](R r) { return r.x; });
    Z0 = ga.m([](R r) { return r.buf.Z; });
  }
  if (steps & kStepLincomb) {
    Zb = as_const(Z0);
    K = ga.i([](R r) { return r.phase().k; });
    OW = ga.i([](R r) { return r.phase().overwrite ? 1 : 0; });
    ytab = ga.ytab();
  }
  if (steps & (kStepIter | kStepScaleV | kStepScaleVDev)) {
    Vj = ga.m([](R r) { return r.buf.V + (size_t)r.phase().j * r.N; });
  }
  if (steps & kStepScaleV) dtab = ga.dtab();
  if (steps & kStepIter) {
    Zj = ga.m([](R r) { return r.buf.Z + (size_t)r.phase().j * r.N; });
    Vj1 = ga.m([](R r) { return r.buf.V + (size_t)(r.phase().j + 1) * r.N; });
    NV = ga.i([](R r) { return r.phase().j + 1; });
    P1 = ga.m([](R r) { return r.buf.P1; });
    P2 = ga.m([](R r) { return r.buf.P2; });
    H1 = ga.m([](R r) { return r.buf.h1; });
    Hc = ga.m([](R r) { return r.buf.Hcol; });
    Hh = ga.m([](R r) { return r.hh_dev(r.phase().bank); });
  }
  if (ga.full) return set_error(FDG_ENOMEM, "enqueue_phase: pointer-table arena full");
  if (nrun > 1) {
    int st = tab->flush(s);
    if (st != FDG_OK) return st;
  }
  // 2-wide accesses of b; the Krylov buffers are 256-byte aligned with an even or odd N
  // handled inside the launchers
  bool b16 = true, x16 = true;
  for (int e = 0; e < nrun; ++e) {
    b16 = b16 && al(runs[e]->b, 16);
    x16 = x16 && al(runs[e]->x, 16);
  }
  bool a32 = true;  // 32-byte alignment of every V_j / Z_j (load width of the FD passes)
  if (steps & kStepIter)
    for (int e = 0; e < nrun; ++e) {
      const SolveRun &r = *runs[e];
      a32 = a32 && al(r.buf.V + (size_t)r.phase().j * N, 32) && al(r.buf.Z + (size_t)r.phase().j * N, 32);
    }
  const bool timed = ex.timed;
  const IBatch one{1, nullptr};
  int st = FDG_OK;

  if (steps & kStepBDots) {
    TimedLaunch tl(c, 2, s, timed);
    launch_dots(s, B, 0, one, B, N, nrun, G, 1, P3, b16);
  }
  if (steps & kStepBNorm) {
    TimedLaunch tl(c, 2, s, timed);
    launch_norm_reduce(s, as_const(P3), G, nrun, Sb, Hb);
  }
  if (steps & kStepBScale) {
    TimedLaunch tl(c, 2, s, timed);
    launch_scale_reduce(s, B, V0, as_const(P3), G, N, nrun, Sb, Hb, b16);
  }
  if (steps & kStepLincomb) {
    TimedLaunch tl(c, 2, s, timed);
    launch_lincomb(s, X, Zb, N, K, r0.coeffs(), ytab, N, nrun, OW, x16);
  }
  if (steps & kStepRes) {
    if (r0.res_parts > 0) {  // r = b - A x fused into the matvec
      if ((st = residual_entries(c, ex, as_const(X), B, V0, nrun, Hp)) != FDG_OK) return st;
    } else {
      if ((st = matvec_entries(c, ex, as_const(X), Z0, nrun, T1, T2)) != FDG_OK) return st;
      TimedLaunch tl(c, 2, s, timed);
      launch_residual(s, B, as_const(Z0), V0, N, nrun, G, Hp, b16);
    }
  }
  if (steps & kStepScaleV) {  // v_j = w / ||w|| with the norm formed on the host
    TimedLaunch tl(c, 2, s, timed);
    launch_scale_by(s, as_const(Vj), Vj, dtab, r0.phase().div, N, nrun, true);
  }
  if (steps & kStepScaleVDev) {  // v_j = w / ||w|| with the norm formed from P3 on the device
    TimedLaunch tl(c, 2, s, timed);
    launch_scale_reduce(s, as_const(Vj), Vj, as_const(P3), G, N, nrun, MBatch{}, MBatch{}, true);
  }
  if (steps & kStepIter) {
    if ((st = apply_entries(c, ex, as_const(Vj), Zj, nrun, T1, T2, r0.buf.t32a, r0.buf.t32b, a32)) != FDG_OK)
      return st;
    if ((st = matvec_entries(c, ex, as_const(Zj), Vj1, nrun, T1, T2)) != FDG_OK) return st;
    {  // classical Gram-Schmidt: h1 = V^T w
      TimedLaunch tl(c, 2, s, timed);
      launch_dots(s, Vb, N, NV, as_const(Vj1), N, nrun, G, ldp, P1, true);
    }
    {  // w -= V h1; h2 = V^T w (reorthogonalisation)
      TimedLaunch tl(c, 2, s, timed);
      launch_update_dots(s, Vb, N, NV, as_const(P1), G, ldp, Vj1, N, nrun, P2, H1, true);
    }
    {  // w -= V h2; Hessenberg column h1 + h2 (device and host-mapped); |w|^2 partials
      TimedLaunch tl(c, 2, s, timed);
      launch_update_norm(s, Vb, N, NV, as_const(P2), G, ldp, Vj1, N, nrun, Hp, as_const(H1), Hc, Hh, true, P3);
    }
  }
  return hip_check(hipGetLastError(), "solve phase launch");
}

}  // namespace fdg
