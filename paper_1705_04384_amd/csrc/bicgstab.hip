// Preconditioned BiCGStab (Sec. 5: every experiment of the paper solves with BiCGStab
// preconditioned by the FD solve of P; van der Vorst's method, one BiCG half step and
// one GMRES(1) half step per iteration), right preconditioned, on one context.
//
// Device side: the scalars of the recurrence (rho = r~.r, r~.v, t.s, t.t) are never
// moved to the host.  Each is kept as G block partials, double-buffered by the parity of
// the iteration, and every consumer kernel sums the partials itself in a fixed order
// (sum_partials), so alpha, beta and omega need no host round trip and no extra launch.
// The host waits twice per iteration, for |s| and |r| (sums of G partials in host-mapped
// memory, added in block order), and decides convergence; a recursive residual below
// the tolerance is confirmed with the true residual |b - A x| in FP64.
//
// Iteration i (parity a = i & 1, previous c = a ^ 1):
//   dir:    p = r (i = 1) or r + beta (p - omega' v), beta = (rho / rho') (alpha' / omega')
//   ph = P^{-1} p,  v = A ph,  Pv[a] = partials of r~.v
//   half:   alpha = rho / r~.v;  s = r - alpha v;  x += alpha ph;  |s|^2 partials -> host
//   sh = P^{-1} s,  t = A sh,  Pts[a], Ptt[a] = partials of t.s, t.t
//   update: omega = t.s / t.t;  x += omega sh;  r = s - omega t;
//           |r|^2 partials -> host;  Prho[c] = partials of r~.r (rho of iteration i + 1)
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>

#include "context.h"
#include "kernels.h"
#include "reduce.h"

namespace fdg {
namespace {

constexpr int kStream = 256;  // threads of the streaming kernel

// Block total of one value per thread (waves in index order); valid in thread 0.
__device__ inline double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kRedWaves; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Device buffers of one BiCGStab solve (N doubles each unless stated).
struct BiBufs {
  double *r, *rh, *p, *v, *ph, *s, *sh, *t;
  double *Prho[2], *Pv[2], *Pts[2], *Ptt[2];  // G partials each
  volatile double *hh;                         // host-mapped, host_doubles(G)
  double *hh_dev;
};

// host-mapped layout: [0,G) |s|^2, [G,2G) |r|^2, [2G,3G) |b|^2, [3G,4G) true residual,
// then rho, r~.v, omega at 4G + 0..2
inline int host_doubles(int G) { return 4 * G + 8; }

// r = b - Ax (Ax null: r = b), r~ = r, x = 0 when zero_x; partials of |b|^2 and |r|^2 to
// the host, of r~.r = |r|^2 to Prho (rho of the first iteration).
__global__ __launch_bounds__(kRed) void k_bi_init(const double *__restrict__ b, const double *__restrict__ Ax,
                                                  double *__restrict__ r, double *__restrict__ rh,
                                                  double *__restrict__ x, int zero_x, int64_t N, int G,
                                                  double *__restrict__ Prho, double *hb, double *hr) {
  __shared__ double red[kRedWaves];
  int64_t beg, end;
  chunk_of(N, G, blockIdx.x, beg, end);
  double sb = 0.0, sr = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kRed) {
    const double bi = b[i];
    const double ri = Ax ? bi - Ax[i] : bi;
    r[i] = ri;
    rh[i] = ri;
    if (zero_x) x[i] = 0.0;
    sb = fma(bi, bi, sb);
    sr = fma(ri, ri, sr);
  }
  sb = block_sum(sb, red);
  sr = block_sum(sr, red);
  if (threadIdx.x == 0) {
    hb[blockIdx.x] = sb;
    hr[blockIdx.x] = sr;
    Prho[blockIdx.x] = sr;
  }
}

// p = r (first) or p = r + beta (p - omega' v) with beta = (rho / rho') (alpha' / omega'),
// alpha' = rho' / (r~.v)', omega' = (t.s)' / (t.t)' -- all from partials.
__global__ __launch_bounds__(kStream) void k_bi_dir(const double *__restrict__ r, double *__restrict__ p,
                                                    const double *__restrict__ v, int64_t N, int first, int G,
                                                    const double *Prho, const double *Prho_o, const double *Pv_o,
                                                    const double *Pts_o, const double *Ptt_o) {
  const int64_t i = (int64_t)blockIdx.x * kStream + threadIdx.x;
  if (first) {
    if (i < N) p[i] = r[i];
    return;
  }
  const double rho = sum_partials(Prho, G, 1, 0), rho_o = sum_partials(Prho_o, G, 1, 0);
  const double alpha_o = rho_o / sum_partials(Pv_o, G, 1, 0);
  const double omega_o = sum_partials(Pts_o, G, 1, 0) / sum_partials(Ptt_o, G, 1, 0);
  const double beta = (rho / rho_o) * (alpha_o / omega_o);
  if (i < N) p[i] = fma(beta, fma(-omega_o, v[i], p[i]), r[i]);
}

// partials of x.y
__global__ __launch_bounds__(kRed) void k_bi_dot(const double *__restrict__ x, const double *__restrict__ y,
                                                 int64_t N, int G, double *__restrict__ P) {
  __shared__ double red[kRedWaves];
  int64_t beg, end;
  chunk_of(N, G, blockIdx.x, beg, end);
  double a = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kRed) a = fma(x[i], y[i], a);
  a = block_sum(a, red);
  if (threadIdx.x == 0) P[blockIdx.x] = a;
}

// partials of t.s and t.t
__global__ __launch_bounds__(kRed) void k_bi_dot_ts(const double *__restrict__ t, const double *__restrict__ s,
                                                    int64_t N, int G, double *__restrict__ Pts,
                                                    double *__restrict__ Ptt) {
  __shared__ double red[kRedWaves];
  int64_t beg, end;
  chunk_of(N, G, blockIdx.x, beg, end);
  double a = 0.0, c = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kRed) {
    const double ti = t[i];
    a = fma(ti, s[i], a);
    c = fma(ti, ti, c);
  }
  a = block_sum(a, red);
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    Pts[blockIdx.x] = a;
    Ptt[blockIdx.x] = c;
  }
}

// alpha = rho / r~.v; s = r - alpha v; x += alpha ph; partials of |s|^2 -> hs.  Nothing
// is written but the scalars when rho or r~.v is zero (breakdown, seen by the host).
__global__ __launch_bounds__(kRed) void k_bi_half(const double *__restrict__ r, const double *__restrict__ v,
                                                  const double *__restrict__ ph, double *__restrict__ x,
                                                  double *__restrict__ s, int64_t N, int G, const double *Prho,
                                                  const double *Pv, double *hs, double *hscal) {
  __shared__ double red[kRedWaves];
  const double rho = sum_partials(Prho, G, 1, 0), rv = sum_partials(Pv, G, 1, 0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    hscal[0] = rho;
    hscal[1] = rv;
  }
  if (rho == 0.0 || rv == 0.0) return;
  const double alpha = rho / rv;
  int64_t beg, end;
  chunk_of(N, G, blockIdx.x, beg, end);
  double a = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kRed) {
    const double si = fma(-alpha, v[i], r[i]);
    s[i] = si;
    x[i] = fma(alpha, ph[i], x[i]);
    a = fma(si, si, a);
  }
  a = block_sum(a, red);
  if (threadIdx.x == 0) hs[blockIdx.x] = a;
}

// omega = t.s / t.t (0 when t = 0); x += omega sh; r = s - omega t; partials of |r|^2 ->
// hr and of r~.r -> Prho_next.
__global__ __launch_bounds__(kRed) void k_bi_update(const double *__restrict__ s, const double *__restrict__ t,
                                                    const double *__restrict__ sh, const double *__restrict__ rh,
                                                    double *__restrict__ x, double *__restrict__ r, int64_t N,
                                                    int G, const double *Pts, const double *Ptt, double *hr,
                                                    double *__restrict__ Prho_next, double *hscal) {
  __shared__ double red[kRedWaves];
  const double ts = sum_partials(Pts, G, 1, 0), tt = sum_partials(Ptt, G, 1, 0);
  const double omega = tt != 0.0 ? ts / tt : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) hscal[2] = omega;
  int64_t beg, end;
  chunk_of(N, G, blockIdx.x, beg, end);
  double a = 0.0, c = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kRed) {
    const double ri = fma(-omega, t[i], s[i]);
    r[i] = ri;
    x[i] = fma(omega, sh[i], x[i]);
    a = fma(ri, ri, a);
    c = fma(rh[i], ri, c);
  }
  a = block_sum(a, red);
  c = block_sum(c, red);
  if (threadIdx.x == 0) {
    hr[blockIdx.x] = a;
    Prho_next[blockIdx.x] = c;
  }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Device buffers of the context's BiCGStab solve, allocated on first use.
int ensure_bicg(fdg_ctx *c, BiBufs &B) {
  const size_t N = (size_t)c->N;
  int st;
  if (!c->bicg) {
    if ((st = dalloc(&c->bicg, 8 * N + 8 * (size_t)kMaxG + 64)) != FDG_OK) return st;
  }
  if (!c->bicg_host) {
    HIPCHK(hipHostMalloc((void **)&c->bicg_host, sizeof(double) * host_doubles(kMaxG), hipHostMallocMapped));
    HIPCHK(hipHostGetDevicePointer((void **)&c->bicg_host_dev, c->bicg_host, 0));
  }
  double *q = c->bicg;
  double **vec[8] = {&B.r, &B.rh, &B.p, &B.v, &B.ph, &B.s, &B.sh, &B.t};
  for (int k = 0; k < 8; ++k) *vec[k] = q + (size_t)k * N;
  double *P = q + 8 * N;
  for (int k = 0; k < 2; ++k) {
    B.Prho[k] = P + (size_t)(0 + k) * kMaxG;
    B.Pv[k] = P + (size_t)(2 + k) * kMaxG;
    B.Pts[k] = P + (size_t)(4 + k) * kMaxG;
    B.Ptt[k] = P + (size_t)(6 + k) * kMaxG;
  }
  B.hh = c->bicg_host;
  B.hh_dev = c->bicg_host_dev;
  return FDG_OK;
}

double host_sum(volatile const double *h, int G) {
  double s = 0.0;
  for (int g = 0; g < G; ++g) s += h[g];
  return s;
}

}  // namespace
}  // namespace fdg

using namespace fdg;

extern "C" int fdg_bicgstab(fdg_ctx *c, const double *b, double *x, double rtol, int maxit, int flags,
                            fdg_info *info) {
  clear_error();
  const auto t0 = std::chrono::steady_clock::now();
  if (!c || !b || !x) return set_error(FDG_EINVAL, "bicgstab: NULL argument");
  if (b == x) return set_error(FDG_EINVAL, "bicgstab: b and x alias");
  if (c->batch != 1) return set_error(FDG_EINVAL, "bicgstab: context batch must be 1");
  if (!(rtol >= 0.0) || maxit < 0) return set_error(FDG_EINVAL, "bicgstab: bad rtol/maxit");
  int st;
  if ((st = ctx_ready(c)) != FDG_OK) return st;
  if ((st = ensure_solve_workspace(c)) != FDG_OK) return st;
  const int64_t N = c->N;
  const int G = reduction_blocks(N);
  BiBufs B;
  if ((st = ensure_bicg(c, B)) != FDG_OK) return st;
  if (!c->phase_ev) HIPCHK(hipEventCreateWithFlags(&c->phase_ev, hipEventDisableTiming));
  const hipStream_t s = c->stream;
  const Exec ex{s, true};
  double *hd = B.hh_dev;
  volatile double *hh = B.hh;
  // The host-mapped slots a phase writes are armed with a signalling-NaN pattern no
  // kernel stores before its launches; the host continues once they all hold values
  // (not at the end of the last kernel), polling the phase event as a fallback: a
  // breakdown in the half step leaves the |s| partials unwritten.
  constexpr uint64_t kUnwritten = 0x7FF4DEADBEEF0001ull;
  volatile uint64_t *hw = reinterpret_cast<volatile uint64_t *>(hh);
  int armed[2][2] = {{0, 0}, {0, 0}};
  bool stream_idle = true;
  auto arm = [&](int a0, int n0, int a1, int n1) {
    armed[0][0] = a0, armed[0][1] = n0, armed[1][0] = a1, armed[1][1] = n1;
    for (int k = 0; k < 2; ++k)
      for (int g = 0; g < armed[k][1]; ++g) hw[armed[k][0] + g] = kUnwritten;
  };
  auto ready = [&]() {
    for (int k = 0; k < 2; ++k)
      for (int g = armed[k][1] - 1; g >= 0; --g)
        if (hw[armed[k][0] + g] == kUnwritten) return false;
    return armed[0][1] + armed[1][1] > 0;
  };
  auto drain = [&]() -> int {
    hipError_t e;
    while ((e = hipEventQuery(c->phase_ev)) == hipErrorNotReady) {
    }
    (void)hipGetLastError();
    HIPCHK(e);
    stream_idle = true;
    return FDG_OK;
  };
  auto wait = [&]() -> int {
    HIPCHK(hipEventRecord(c->phase_ev, s));
    stream_idle = false;
    hipError_t e = hipErrorNotReady;
    for (unsigned k = 1; !ready(); ++k) {
      if ((k & 63) == 0 && (e = hipEventQuery(c->phase_ev)) != hipErrorNotReady) break;
    }
    if (e != hipErrorNotReady) {
      (void)hipGetLastError();
      HIPCHK(e);
      stream_idle = true;
    }
    if (!ready() && !stream_idle) return drain();
    return FDG_OK;
  };
  auto apply = [&](const double *in, double *out) {
    return apply_entries(c, ex, cstrided(in, 0), mstrided(out, 0), 1, mstrided(c->t1, 0), mstrided(c->t2, 0),
                         c->t32a, c->t32b, false);
  };
  auto matvec = [&](const double *in, double *out) {
    return matvec_entries(c, ex, cstrided(in, 0), mstrided(out, 0), 1, mstrided(c->t1, 0), mstrided(c->t2, 0));
  };
  // true residual |b - A x| (into sh, using t), partials to hh[3G ..)
  auto true_res = [&](double &nrm) -> int {
    int e;
    arm(3 * G, G, 0, 0);
    if ((e = matvec(x, B.t)) != FDG_OK) return e;
    {
      TimedLaunch tl(c, 2, s, true);
      launch_residual(s, cstrided(b, 0), cstrided(B.t, 0), mstrided(B.sh, 0), N, 1, G, mstrided(hd + 3 * G, 0),
                      false);
    }
    if ((e = wait()) != FDG_OK) return e;
    nrm = std::sqrt(host_sum(hh + 3 * G, G));
    return FDG_OK;
  };

  fdg_info inf{};
  const bool use_x0 = flags & FDG_SOLVE_USE_X0, fixed = flags & FDG_SOLVE_FIXED_ITERS;
  arm(G, G, 2 * G, G);
  if (use_x0 && (st = matvec(x, B.t)) != FDG_OK) return st;
  {
    TimedLaunch tl(c, 2, s, true);
    hipLaunchKernelGGL(k_bi_init, dim3(G), dim3(kRed), 0, s, b, use_x0 ? (const double *)B.t : nullptr, B.r, B.rh, x,
                       use_x0 ? 0 : 1, N, G, B.Prho[1], hd + 2 * G, hd + G);
  }
  HIPCHK(hipGetLastError());
  if ((st = wait()) != FDG_OK) return st;
  const double bnorm = std::sqrt(host_sum(hh + 2 * G, G));
  const double target = rtol * bnorm;
  double rnorm = std::sqrt(host_sum(hh + G, G));
  int half = 0, full = 0;
  bool conv = false, brk = false;
  if (bnorm == 0.0) {
    if (use_x0) HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * N, s));  // A x = 0 has x = 0
    conv = true;
    rnorm = 0.0;
  } else if (!fixed && rnorm <= target) {
    conv = true;
  }
  for (int i = 1; !conv && !brk && i <= maxit; ++i) {
    const int a = i & 1, o = a ^ 1;
    arm(0, G, 4 * G, 2);
    {
      TimedLaunch tl(c, 2, s, true);
      hipLaunchKernelGGL(k_bi_dir, dim3(cdiv(N, kStream)), dim3(kStream), 0, s, B.r, B.p, B.v, N, i == 1 ? 1 : 0, G,
                         B.Prho[a], B.Prho[o], B.Pv[o], B.Pts[o], B.Ptt[o]);
    }
    if ((st = apply(B.p, B.ph)) != FDG_OK) return st;
    if ((st = matvec(B.ph, B.v)) != FDG_OK) return st;
    {
      TimedLaunch tl(c, 2, s, true);
      hipLaunchKernelGGL(k_bi_dot, dim3(G), dim3(kRed), 0, s, B.rh, B.v, N, G, B.Pv[a]);
      hipLaunchKernelGGL(k_bi_half, dim3(G), dim3(kRed), 0, s, B.r, B.v, B.ph, x, B.s, N, G, B.Prho[a], B.Pv[a],
                         hd, hd + 4 * G);
    }
    HIPCHK(hipGetLastError());
    if ((st = wait()) != FDG_OK) return st;
    if (hh[4 * G] == 0.0 || hh[4 * G + 1] == 0.0) {  // rho or r~.v vanished: x untouched
      brk = true;
      break;
    }
    ++half;
    const double snorm = std::sqrt(host_sum(hh, G));
    if (!fixed && snorm <= target) {
      double tr;
      if ((st = true_res(tr)) != FDG_OK) return st;
      if (tr <= target) {
        conv = true;
        rnorm = tr;
        break;
      }
    }
    arm(G, G, 4 * G + 2, 1);
    if ((st = apply(B.s, B.sh)) != FDG_OK) return st;
    if ((st = matvec(B.sh, B.t)) != FDG_OK) return st;
    {
      TimedLaunch tl(c, 2, s, true);
      hipLaunchKernelGGL(k_bi_dot_ts, dim3(G), dim3(kRed), 0, s, B.t, B.s, N, G, B.Pts[a], B.Ptt[a]);
      hipLaunchKernelGGL(k_bi_update, dim3(G), dim3(kRed), 0, s, B.s, B.t, B.sh, B.rh, x, B.r, N, G, B.Pts[a],
                         B.Ptt[a], hd + G, B.Prho[o], hd + 4 * G);
    }
    HIPCHK(hipGetLastError());
    if ((st = wait()) != FDG_OK) return st;
    ++half;
    full = i;
    rnorm = std::sqrt(host_sum(hh + G, G));
    if (!fixed && rnorm <= target) {
      double tr;
      if ((st = true_res(tr)) != FDG_OK) return st;
      if (tr <= target) {
        conv = true;
        rnorm = tr;
        break;
      }
    }
    if (hh[4 * G + 2] == 0.0) brk = true;  // omega = 0: no further progress possible
  }
  double tr = 0.0;
  if (bnorm > 0.0 && (st = true_res(tr)) != FDG_OK) return st;
  if (!stream_idle || (bnorm == 0.0 && use_x0)) {  // x is the caller's once the stream is done
    HIPCHK(hipEventRecord(c->phase_ev, s));
    if ((st = drain()) != FDG_OK) return st;
  }
  inf.iterations = full;
  inf.half_steps = half;
  inf.restarts = 0;
  inf.breakdown = brk ? 1 : 0;
  inf.rel_res_est = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  inf.rel_res_true = bnorm > 0.0 ? tr / bnorm : 0.0;
  inf.converged = bnorm == 0.0 || tr <= target;
  const int status = inf.converged ? FDG_OK : FDG_NOT_CONVERGED;
  inf.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}
