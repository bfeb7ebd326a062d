// Operator matvecs: the unit-domain collocation matrix of eq. 2.9 / 2.7 applied from its
// banded univariate factors, and a slot-major ELL matvec for an assembled matrix.
//
// Unit domain, 3D: y = (K3 x M2 x M1 + M3 x K2 x M1 + M3 x M2 x K1) x, sum-factorised:
// per plane j3 the direction-1 band sums sM = M1 x, sK = K1 x, then the direction-2 sums
//     a(j3) = sum_j2 M2 sM,      c(j3) = sum_j2 (K2 sM + M2 sK),
// and the output y(i3) = sum_j3 K3 a(j3) + M3 c(j3) over the direction-3 band.
// Forms, in order of preference:
//   k_kron3_stream  one pass streaming the planes of a chunk through a register ring
//                   (one band width W in 2..8 in all directions, band starts growing by at
//                   most 1 per row, at least 128 workgroups per entry); no scratch,
//                   gathered batches;
//   k_kron3_wpp     one pass, one wave per plane (bands up to 8 wide whose starts grow by
//                   at most 1 per row in directions 1 and 2); no scratch, gathered batches;
//   k_kron3_planes  two passes through per-plane intermediates a, c (scratch);
//   + k_kron3_mode3
//   k_kron3_lds /   one pass, a thread per output column sweeping i3 with a sliding
//   k_kron3_window  window of planes in registers (contiguous batches only).
// 2D: k_kron2_window, the same sliding window over i2.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_addr.h"
#include "kernels.h"

namespace fdg {

namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 16;  // output rows of the sweep direction per thread

// Shape of the one-pass 3D matvec: i2 rows per tile and i3 outputs per workgroup
// (overridable at build time for tuning sweeps).
#ifndef FDG_MV_T2
#define FDG_MV_T2 2
#endif
#ifndef FDG_MV_C3
#define FDG_MV_C3 16
#endif

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <int WMAX>
__global__ __launch_bounds__(kBlock) void k_kron3_window(const double *__restrict__ x, double *__restrict__ y,
                                                         int n, KronBands bd) {
  const int64_t col = (int64_t)blockIdx.x * kBlock + threadIdx.x;  // i2 * n + i1
  const int64_t n2 = (int64_t)n * n;
  if (col >= n2) return;
  const int s = blockIdx.y * kChunk;
  const int e = s + kChunk < n ? s + kChunk : n;
  const int64_t b = blockIdx.z;
  const int i1 = (int)(col % n), i2 = (int)(col / n);
  const double *xb = x + b * n2 * n;
  double *yb = y + b * n2 * n;
  const int w1 = bd.w[0], w2 = bd.w[1], w3 = bd.w[2];
  double m1[WMAX], k1[WMAX], m2[WMAX], k2[WMAX];
#pragma unroll
  for (int t = 0; t < WMAX; ++t) {
    m1[t] = t < w1 ? bd.M[0][(size_t)i1 * w1 + t] : 0.0;
    k1[t] = t < w1 ? bd.K[0][(size_t)i1 * w1 + t] : 0.0;
    m2[t] = t < w2 ? bd.M[1][(size_t)i2 * w2 + t] : 0.0;
    k2[t] = t < w2 ? bd.K[1][(size_t)i2 * w2 + t] : 0.0;
  }
  const int lo1 = bd.lo[0][i1], lo2 = bd.lo[1][i2];
  auto plane = [&](int j3, double &a, double &c) {
    a = 0.0;
    c = 0.0;
    const double *xp = xb + (int64_t)j3 * n2 + (int64_t)lo2 * n + lo1;
#pragma unroll
    for (int t2 = 0; t2 < WMAX; ++t2) {
      if (t2 < w2) {
        const double *xr = xp + (int64_t)t2 * n;
        double sm = 0.0, sk = 0.0;
#pragma unroll
        for (int t1 = 0; t1 < WMAX; ++t1) {
          if (t1 < w1) {
            const double v = xr[t1];
            sm = fma(m1[t1], v, sm);
            sk = fma(k1[t1], v, sk);
          }
        }
        a = fma(m2[t2], sm, a);
        c = fma(k2[t2], sm, c);
        c = fma(m2[t2], sk, c);
      }
    }
  };
  // window: slots WMAX-w3 .. WMAX-1 hold planes base .. base+w3-1
  double A[WMAX], C[WMAX];
  int base = bd.lo[2][s];
#pragma unroll
  for (int u = 0; u < WMAX; ++u) {
    const int t = u - (WMAX - w3);
    if (t >= 0) {
      plane(base + t, A[u], C[u]);
    } else {
      A[u] = 0.0;
      C[u] = 0.0;
    }
  }
  for (int i3 = s; i3 < e; ++i3) {
    const int target = bd.lo[2][i3];
    while (base < target) {
#pragma unroll
      for (int u = 0; u < WMAX - 1; ++u) {
        A[u] = A[u + 1];
        C[u] = C[u + 1];
      }
      plane(base + w3, A[WMAX - 1], C[WMAX - 1]);
      ++base;
    }
    const double *m3 = bd.M[2] + (size_t)i3 * w3;
    const double *k3 = bd.K[2] + (size_t)i3 * w3;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < WMAX; ++u) {
      const int t = u - (WMAX - w3);
      if (t >= 0) {
        acc = fma(k3[t], A[u], acc);
        acc = fma(m3[t], C[u], acc);
      }
    }
    yb[(int64_t)i3 * n2 + col] = acc;
  }
}

// 3D, LDS-tiled: a workgroup owns 64 consecutive i1 (the lanes) x 4 consecutive i2 (the
// waves) and sweeps a chunk of i3.  For each plane j3 the direction-1 band sums of the
// rows j2 that the 4 rows i2 need are formed once into LDS (double-buffered by plane
// parity, so one barrier per plane suffices); every thread then combines its w2 rows
// into a(j3), c(j3) and keeps the sliding window of planes in registers.
constexpr int kRowsMax = 12;  // rows j2 a tile of 4 rows i2 may need: 3 + w2 (checked on the host)

template <int WMAX>
__global__ __launch_bounds__(kBlock) void k_kron3_lds(const double *__restrict__ x, double *__restrict__ y, int n,
                                                      int nchunk, KronBands bd) {
  __shared__ double sm[2][kRowsMax][64];
  __shared__ double sk[2][kRowsMax][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i1 = blockIdx.x * 64 + lane;
  const int i2a = blockIdx.y * 4;
  const int i2 = i2a + wave;
  const int chunk = blockIdx.z % nchunk;
  const int64_t b = blockIdx.z / nchunk;
  const int s = chunk * kChunk;
  const int e = s + kChunk < n ? s + kChunk : n;
  const int64_t n2 = (int64_t)n * n;
  const double *xb = x + b * n2 * n;
  double *yb = y + b * n2 * n;
  const int w1 = bd.w[0], w2 = bd.w[1], w3 = bd.w[2];
  const bool act1 = i1 < n, act = act1 && i2 < n;
  const int i1c = act1 ? i1 : n - 1;
  const int i2c = i2 < n ? i2 : n - 1;
  const int i2b = i2a + 3 < n ? i2a + 3 : n - 1;
  const int R0 = bd.lo[1][i2a];
  const int NR = bd.lo[1][i2b] + w2 - R0;  // <= kRowsMax
  double m1[WMAX], k1[WMAX], m2[WMAX], k2[WMAX];
#pragma unroll
  for (int t = 0; t < WMAX; ++t) {
    m1[t] = t < w1 ? bd.M[0][(size_t)i1c * w1 + t] : 0.0;
    k1[t] = t < w1 ? bd.K[0][(size_t)i1c * w1 + t] : 0.0;
    m2[t] = t < w2 ? bd.M[1][(size_t)i2c * w2 + t] : 0.0;
    k2[t] = t < w2 ? bd.K[1][(size_t)i2c * w2 + t] : 0.0;
  }
  const int lo1 = bd.lo[0][i1c];
  const int r2 = bd.lo[1][i2c] - R0;  // first LDS row of this thread's band
  int parity = 0;
  auto plane = [&](int j3, double &a, double &c) {
    // phase 1: rows R0 .. R0+NR-1 of plane j3, direction-1 band sums (wave w takes rows w, w+4, ...)
    const double *xp = xb + (int64_t)j3 * n2 + lo1;
    for (int r = wave; r < NR; r += 4) {
      const double *xr = xp + (int64_t)(R0 + r) * n;
      double vm = 0.0, vk = 0.0;
#pragma unroll
      for (int t1 = 0; t1 < WMAX; ++t1)
        if (t1 < w1) {
          const double v = xr[t1];
          vm = fma(m1[t1], v, vm);
          vk = fma(k1[t1], v, vk);
        }
      sm[parity][r][lane] = vm;
      sk[parity][r][lane] = vk;
    }
    __syncthreads();
    // phase 2: direction-2 band of this thread's row i2
    a = 0.0;
    c = 0.0;
#pragma unroll
    for (int t2 = 0; t2 < WMAX; ++t2)
      if (t2 < w2) {
        const double vm = sm[parity][r2 + t2][lane], vk = sk[parity][r2 + t2][lane];
        a = fma(m2[t2], vm, a);
        c = fma(k2[t2], vm, c);
        c = fma(m2[t2], vk, c);
      }
    parity ^= 1;
  };
  double A[WMAX], C[WMAX];
  int base = bd.lo[2][s];
#pragma unroll
  for (int u = 0; u < WMAX; ++u) {
    const int t = u - (WMAX - w3);
    if (t >= 0) {
      plane(base + t, A[u], C[u]);
    } else {
      A[u] = 0.0;
      C[u] = 0.0;
    }
  }
  for (int i3 = s; i3 < e; ++i3) {
    const int target = bd.lo[2][i3];
    while (base < target) {
#pragma unroll
      for (int u = 0; u < WMAX - 1; ++u) {
        A[u] = A[u + 1];
        C[u] = C[u + 1];
      }
      plane(base + w3, A[WMAX - 1], C[WMAX - 1]);
      ++base;
    }
    if (act) {
      const double *m3 = bd.M[2] + (size_t)i3 * w3;
      const double *k3 = bd.K[2] + (size_t)i3 * w3;
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < WMAX; ++u) {
        const int t = u - (WMAX - w3);
        if (t >= 0) {
          acc = fma(k3[t], A[u], acc);
          acc = fma(m3[t], C[u], acc);
        }
      }
      yb[(int64_t)i3 * n2 + (int64_t)i2 * n + i1] = acc;
    }
  }
}

// 3D in two passes, both fully parallel:
//   pass 1, per plane j3 and tile of 64 i1 x 16 i2: the direction-1 band sums of the rows
//   j2 the tile needs go to LDS once; each thread combines its w2 rows into
//       a[j3][i2][i1] = sum_j2 M2 sM,   c[j3][i2][i1] = sum_j2 (K2 sM + M2 sK)
//   pass 2, per output: y[i3] = sum_t3 K3[i3][t3] a[lo3 + t3] + M3[i3][t3] c[lo3 + t3];
//   a thread produces 4 consecutive i3 and loads the union of their plane bands once.
constexpr int kPlaneRows = 16;                 // i2 rows per pass-1 tile
constexpr int kPlaneRowsMax = kPlaneRows + 15; // rows j2 the tile may need (w2 <= 16)

template <int WMAX>
__global__ __launch_bounds__(kBlock) void k_kron3_planes(CBatch x, MBatch ao, MBatch co, int n,
                                                         KronBands bd) {
  __shared__ double sm[kPlaneRowsMax][64];
  __shared__ double sk[kPlaneRowsMax][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i1 = blockIdx.x * 64 + lane;
  const int i2a = blockIdx.y * kPlaneRows;
  const int64_t pl = blockIdx.z;  // b * n + j3
  const int64_t n2 = (int64_t)n * n;
  const int64_t ent = pl / n;
  const int64_t j3 = pl - ent * n;
  gptr<const double> __restrict__ xp = x.gat(ent) + j3 * n2;
  gptr<double> __restrict__ ap = ao.gat(ent) + j3 * n2;
  gptr<double> __restrict__ cp = co.gat(ent) + j3 * n2;
  const int w1 = bd.w[0], w2 = bd.w[1];
  const bool act1 = i1 < n;
  const int i1c = act1 ? i1 : n - 1;
  const int i2b = i2a + kPlaneRows - 1 < n ? i2a + kPlaneRows - 1 : n - 1;
  const int R0 = bd.lo[1][i2a];
  const int NR = bd.lo[1][i2b] + w2 - R0;  // <= kPlaneRowsMax, checked on the host
  const int lo1 = bd.lo[0][i1c];
  double m1[WMAX], k1[WMAX];
#pragma unroll
  for (int t = 0; t < WMAX; ++t) {
    m1[t] = t < w1 ? bd.M[0][(size_t)i1c * w1 + t] : 0.0;
    k1[t] = t < w1 ? bd.K[0][(size_t)i1c * w1 + t] : 0.0;
  }
  // rows r = wave + 4 u, u < kRowsPerWave: every load of the tile is issued before use
  constexpr int kRowsPerWave = (kPlaneRowsMax + 3) / 4;
  double xv[kRowsPerWave][WMAX];
#pragma unroll
  for (int u = 0; u < kRowsPerWave; ++u) {
    const int r = wave + 4 * u;
    gptr<const double> xr = xp + (int64_t)(R0 + (r < NR ? r : 0)) * n + lo1;
#pragma unroll
    for (int t1 = 0; t1 < WMAX; ++t1) xv[u][t1] = (r < NR && t1 < w1) ? xr[t1] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kRowsPerWave; ++u) {
    const int r = wave + 4 * u;
    if (r < NR) {
      double vm = 0.0, vk = 0.0;
#pragma unroll
      for (int t1 = 0; t1 < WMAX; ++t1) {
        vm = fma(m1[t1], xv[u][t1], vm);
        vk = fma(k1[t1], xv[u][t1], vk);
      }
      sm[r][lane] = vm;
      sk[r][lane] = vk;
    }
  }
  __syncthreads();
  if (!act1) return;
#pragma unroll
  for (int u = 0; u < kPlaneRows / 4; ++u) {
    const int i2 = i2a + wave + 4 * u;
    if (i2 > i2b) break;
    const int r2 = bd.lo[1][i2] - R0;
    const double *m2 = bd.M[1] + (size_t)i2 * w2;
    const double *k2 = bd.K[1] + (size_t)i2 * w2;
    double a = 0.0, c = 0.0;
#pragma unroll
    for (int t2 = 0; t2 < WMAX; ++t2)
      if (t2 < w2) {
        const double vm = sm[r2 + t2][lane], vk = sk[r2 + t2][lane];
        a = fma(m2[t2], vm, a);
        c = fma(k2[t2], vm, c);
        c = fma(m2[t2], vk, c);
      }
    const int64_t o = (int64_t)i2 * n + i1;
    ap[o] = a;
    cp[o] = c;
  }
}

constexpr int kRowsPerThread = 4;  // consecutive i3 outputs per thread in pass 2

template <int WMAX>
__global__ __launch_bounds__(kBlock) void k_kron3_mode3(CBatch ai, CBatch ci, MBatch y, int n, int ngroups,
                                                        KronBands bd) {
  const int64_t n2 = (int64_t)n * n;
  const int64_t col = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (col >= n2) return;
  const int grp = blockIdx.y % ngroups;
  const int64_t b = blockIdx.y / ngroups;
  const int s = grp * kRowsPerThread;
  const int e = s + kRowsPerThread < n ? s + kRowsPerThread : n;
  const int w3 = bd.w[2];
  const int P0 = bd.lo[2][s];
  const int np = bd.lo[2][e - 1] + w3 - P0;  // planes needed, <= kRowsPerThread - 1 + WMAX
  gptr<const double> ab = ai.gat(b) + col, cb = ci.gat(b) + col;
  constexpr int NPMAX = kRowsPerThread - 1 + WMAX;
  double av[NPMAX], cv[NPMAX];
#pragma unroll
  for (int q = 0; q < NPMAX; ++q) {
    const bool ok = q < np;
    av[q] = ok ? ab[(int64_t)(P0 + q) * n2] : 0.0;
    cv[q] = ok ? cb[(int64_t)(P0 + q) * n2] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const int i3 = s + r;
    if (i3 >= e) break;
    const int off = bd.lo[2][i3] - P0;
    const double *m3 = bd.M[2] + (size_t)i3 * w3;
    const double *k3 = bd.K[2] + (size_t)i3 * w3;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < NPMAX; ++q) {
      const int t = q - off;
      if (t >= 0 && t < w3) {
        acc = fma(k3[t], av[q], acc);
        acc = fma(m3[t], cv[q], acc);
      }
    }
    y.gat(b)[(int64_t)i3 * n2 + col] = acc;
  }
}

// 2D: one thread owns column i1 and sweeps a chunk of i2; window of direction-1 band sums.
template <int WMAX>
__global__ __launch_bounds__(kBlock) void k_kron2_window(CBatch x, MBatch y, int n, KronBands bd) {
  const int i1 = blockIdx.x * kBlock + threadIdx.x;
  if (i1 >= n) return;
  const int s = blockIdx.y * kChunk;
  const int e = s + kChunk < n ? s + kChunk : n;
  const int64_t b = blockIdx.z;
  gptr<const double> __restrict__ xb = x.gat(b);
  gptr<double> __restrict__ yb = y.gat(b);
  const int w1 = bd.w[0], w2 = bd.w[1];
  double m1[WMAX], k1[WMAX];
#pragma unroll
  for (int t = 0; t < WMAX; ++t) {
    m1[t] = t < w1 ? bd.M[0][(size_t)i1 * w1 + t] : 0.0;
    k1[t] = t < w1 ? bd.K[0][(size_t)i1 * w1 + t] : 0.0;
  }
  const int lo1 = bd.lo[0][i1];
  auto row = [&](int j2, double &sm, double &sk) {
    sm = 0.0;
    sk = 0.0;
    gptr<const double> xr = xb + (int64_t)j2 * n + lo1;
#pragma unroll
    for (int t1 = 0; t1 < WMAX; ++t1)
      if (t1 < w1) {
        const double v = xr[t1];
        sm = fma(m1[t1], v, sm);
        sk = fma(k1[t1], v, sk);
      }
  };
  double SM[WMAX], SK[WMAX];
  int base = bd.lo[1][s];
#pragma unroll
  for (int u = 0; u < WMAX; ++u) {
    const int t = u - (WMAX - w2);
    if (t >= 0) {
      row(base + t, SM[u], SK[u]);
    } else {
      SM[u] = 0.0;
      SK[u] = 0.0;
    }
  }
  for (int i2 = s; i2 < e; ++i2) {
    const int target = bd.lo[1][i2];
    while (base < target) {
#pragma unroll
      for (int u = 0; u < WMAX - 1; ++u) {
        SM[u] = SM[u + 1];
        SK[u] = SK[u + 1];
      }
      row(base + w2, SM[WMAX - 1], SK[WMAX - 1]);
      ++base;
    }
    const double *m2 = bd.M[1] + (size_t)i2 * w2;
    const double *k2 = bd.K[1] + (size_t)i2 * w2;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < WMAX; ++u) {
      const int t = u - (WMAX - w2);
      if (t >= 0) {
        acc = fma(k2[t], SM[u], acc);
        acc = fma(m2[t], SK[u], acc);
      }
    }
    yb[(int64_t)i2 * n + i1] = acc;
  }
}

// ELL (slot-major: slot t of row r at t * ld + r).  S lanes share a row: a wave covers
// R = 64 / S consecutive rows, lane group g (lanes g R .. g R + R - 1) takes slots
// g, g + S, ..., so every group reads R consecutive entries of a slot; the S partial
// sums of a row are then added by a butterfly over the groups.  Wide rows (the Galerkin
// (2p+1)^3 stencil) need S > 1 to keep enough loads in flight; the order of the sum is
// fixed for a given width and S.
template <int S>
__global__ __launch_bounds__(kBlock) void k_ell_f64(CBatch x, MBatch y, int64_t nrows, int64_t ld, int width,
                                                    const int32_t *__restrict__ col,
                                                    const double *__restrict__ val) {
  constexpr int R = 64 / S;
  const int lane = threadIdx.x & 63;
  const int g = lane / R;
  const int64_t row = ((int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63)) / S + (lane % R);
  const bool ok = row < nrows;
  const int64_t b = blockIdx.y;
  gptr<const double> __restrict__ xb = x.gat(b);
  double acc = 0.0;
  if (ok)
    for (int t = g; t < width; t += S) {
      const int64_t e = (int64_t)t * ld + row;
      acc = fma(val[e], xb[col[e]], acc);
    }
#pragma unroll
  for (int m = R; m < 64; m <<= 1) acc += __shfl_xor(acc, m);
  if (ok && g == 0) y.gat(b)[row] = acc;
}

// One-pass 3D form, one wave per plane.  A workgroup of 8 waves owns a tile of 64
// columns i1 x T2 rows i2 and a chunk of C3 outputs i3.  Each wave takes planes j3 of
// the chunk's band: it loads the plane's rows (all issued at once), forms the
// direction-1 band sums per row through a one-row LDS buffer of its own (no workgroup
// barrier) and the direction-2 sums a = M2 sM, c = K2 sM + M2 sK in registers, and
// stores a and c of its T2 x 64 tile to LDS.  After one barrier every wave forms outputs
// y = sum K3 a + M3 c over the direction-3 band.  Two workgroup barriers in all.
// Requires band starts that grow by at most 1 per row in directions 1 and 2.
// RES: store r = b - A x instead of A x, and one partial of |r|^2 per workgroup.
template <int WMAX, int T2, int C3, bool RES>
__global__ __launch_bounds__(512) void k_kron3_wpp(CBatch x, MBatch y, int n, int ntx, int nty, int nchunk,
                                                   KronBands bd, CBatch rhs, MBatch part) {
  constexpr int NWV = 8;
  constexpr int RMAX = T2 + WMAX - 1;    // rows j2 a tile may need
  constexpr int CW = 64 + WMAX;          // staged columns j1 per row
  constexpr int NPLMAX = C3 + WMAX - 1;  // planes j3 a chunk may need
  __shared__ double xrow[NWV][CW];
  __shared__ double cm2[T2][RMAX], ck2[T2][RMAX];  // direction-2 coefficient of staged row r for output u
  __shared__ double c3k[C3][WMAX], c3m[C3][WMAX];
  __shared__ int lo3s[C3];
  __shared__ double As[NPLMAX][T2][64], Cs[NPLMAX][T2][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nb = (int64_t)gridDim.x;
  int64_t t = blockIdx.x;
  if ((nb & 7) == 0) t = (t & 7) * (nb >> 3) + (t >> 3);
  const int tx = (int)(t % ntx);
  int64_t rest = t / ntx;
  const int ty = (int)(rest % nty);
  rest /= nty;
  const int64_t ent = rest / nchunk;
  const int s3 = (int)(rest - ent * nchunk) * C3;
  const int i1a = tx * 64;
  const int i1 = i1a + lane;
  const int i2a = ty * T2;
  const int e3 = s3 + C3 < n ? s3 + C3 : n;
  const int64_t n2 = (int64_t)n * n;
  gptr<const double> __restrict__ xb = x.gat(ent);
  gptr<double> __restrict__ yb = y.gat(ent);
  const int w1 = bd.w[0], w2 = bd.w[1], w3 = bd.w[2];
  const bool act1 = i1 < n;
  const int i1c = act1 ? i1 : n - 1;
  const int L0 = bd.lo[0][i1a];
  const int off1 = bd.lo[0][i1c] - L0;  // in [0, 63]
  const int i2b = i2a + T2 - 1 < n ? i2a + T2 - 1 : n - 1;
  const int R0 = bd.lo[1][i2a];
  const int NR = bd.lo[1][i2b] + w2 - R0;  // <= RMAX
  const int P0 = bd.lo[2][s3];
  const int NPL = bd.lo[2][e3 - 1] + w3 - P0;  // <= NPLMAX
  const int ncols = n - L0;
  double m1[WMAX], k1[WMAX];
#pragma unroll
  for (int q = 0; q < WMAX; ++q) {
    m1[q] = q < w1 ? bd.M[0][(size_t)i1c * w1 + q] : 0.0;
    k1[q] = q < w1 ? bd.K[0][(size_t)i1c * w1 + q] : 0.0;
  }
  // coefficient tables (read from global memory before any LDS store)
  double vm2 = 0.0, vk2 = 0.0, vm3 = 0.0, vk3 = 0.0;
  int vlo3 = 1 << 30;
  if (threadIdx.x < T2 * RMAX) {
    const int u = threadIdx.x / RMAX, r = threadIdx.x - u * RMAX;
    const int i2 = i2a + u;
    if (i2 <= i2b) {
      const int tt = R0 + r - bd.lo[1][i2];
      if (tt >= 0 && tt < w2) {
        vm2 = bd.M[1][(size_t)i2 * w2 + tt];
        vk2 = bd.K[1][(size_t)i2 * w2 + tt];
      }
    }
  }
  if (threadIdx.x < C3 * WMAX) {
    const int q = threadIdx.x / WMAX, tt = threadIdx.x - q * WMAX;
    if (s3 + q < e3 && tt < w3) {
      vm3 = bd.M[2][(size_t)(s3 + q) * w3 + tt];
      vk3 = bd.K[2][(size_t)(s3 + q) * w3 + tt];
    }
  }
  if (threadIdx.x < C3 && s3 + (int)threadIdx.x < e3) vlo3 = bd.lo[2][s3 + threadIdx.x];
  if (threadIdx.x < T2 * RMAX) {
    const int u = threadIdx.x / RMAX, r = threadIdx.x - u * RMAX;
    cm2[u][r] = vm2;
    ck2[u][r] = vk2;
  }
  if (threadIdx.x < C3 * WMAX) {
    const int q = threadIdx.x / WMAX, tt = threadIdx.x - q * WMAX;
    c3m[q][tt] = vm3;
    c3k[q][tt] = vk3;
  }
  if (threadIdx.x < C3) lo3s[threadIdx.x] = vlo3;
  __syncthreads();
  for (int pl = wave; pl < NPL; pl += NWV) {
    gptr<const double> xp = xb + (int64_t)(P0 + pl) * n2 + (int64_t)R0 * n + L0;
    double xr[RMAX], xh[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      xr[r] = (r < NR && lane < ncols) ? xp[(int64_t)r * n + lane] : 0.0;
      xh[r] = (r < NR && lane < WMAX && 64 + lane < ncols) ? xp[(int64_t)r * n + 64 + lane] : 0.0;
    }
    double hm[RMAX], hk[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      xrow[wave][lane] = xr[r];
      if (lane < WMAX) xrow[wave][64 + lane] = xh[r];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double vm = 0.0, vk = 0.0;
#pragma unroll
      for (int q = 0; q < WMAX; ++q)
        if (q < w1) {
          const double v = xrow[wave][off1 + q];
          vm = fma(m1[q], v, vm);
          vk = fma(k1[q], v, vk);
        }
      hm[r] = vm;
      hk[r] = vk;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int u = 0; u < T2; ++u) {
      double a = 0.0, c = 0.0;
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const double cm = cm2[u][r], ck = ck2[u][r];
        a = fma(cm, hm[r], a);
        c = fma(ck, hm[r], c);
        c = fma(cm, hk[r], c);
      }
      As[pl][u][lane] = a;
      Cs[pl][u][lane] = c;
    }
  }
  __syncthreads();
  double rr = 0.0;  // RES: this thread's part of |b - A x|^2
  if (act1) {
    gptr<const double> rb = RES ? rhs.gat(ent) : nullptr;
    for (int idx = wave; idx < C3 * T2; idx += NWV) {
      const int q = idx / T2, u = idx - q * T2;
      const int i2 = i2a + u;
      if (s3 + q >= e3 || i2 > i2b) continue;
      const int b3 = lo3s[q] - P0;
      double acc = 0.0;
#pragma unroll
      for (int tt = 0; tt < WMAX; ++tt)
        if (tt < w3) {
          acc = fma(c3k[q][tt], As[b3 + tt][u][lane], acc);
          acc = fma(c3m[q][tt], Cs[b3 + tt][u][lane], acc);
        }
      const int64_t o = (int64_t)(s3 + q) * n2 + (int64_t)i2 * n + i1;
      if (RES) {
        const double r = rb[o] - acc;
        yb[o] = r;
        rr = fma(r, r, rr);
      } else {
        yb[o] = acc;
      }
    }
  }
  if (RES) {  // one partial per workgroup, waves in index order
    __shared__ double red[NWV];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) rr += __shfl_xor(rr, off, 64);
    if (lane == 0) red[wave] = rr;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = red[0];
      for (int k = 1; k < NWV; ++k) sum += red[k];
      part.gat(ent)[t - ent * (int64_t)ntx * nty * nchunk] = sum;
    }
  }
}


// Workgroup barrier that orders LDS accesses only: __syncthreads() also orders global
// memory, which makes every wave wait for all of its outstanding loads (the prefetched
// planes) at each barrier.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The same between the lanes of one wave.
__device__ inline void lds_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// One-pass 3D form streaming direction 3 through registers.  A workgroup of 8 waves owns
// a tile of 64 columns i1 x T2 rows i2 and a chunk of outputs i3 in [s3, e3).  Waves
// 0..6 load and compute, wave 7 only stores (and, for the residual, loads b): a wave
// keeps its prefetched planes in flight only while it issues no global stores and no
// loads that may or may not execute, and its barriers order LDS only (lds_barrier).
// The tile's windows are at most 64 + w1 - 1 staged columns j1 (lanes, plus w1 - 1 halo
// lanes) and 7 RPW staged rows j2 (T2 = 7 RPW - w2 + 1 with band starts growing by at
// most 1 per row); compute wave w stages rows j2 = R0 + w + 7 k, k < RPW.  The chunk's
// input planes j3 are visited in order, loaded D planes ahead into registers (every load
// is issued, at a clamped address where it lies outside the tensor, and masked when
// used).  Per plane, each compute wave passes its rows through a wave-private LDS row
// buffer and forms the direction-1 band sums sM = M1 x and sK = K1 x, which enter a
// register ring holding the last WMAX planes.  When the ring holds the direction-3 band
// of an output plane i3, each compute wave forms
//     f = K3 sM + M3 sK,   g = M3 sM          (band sums over the ring)
// for its rows and stores them to LDS; after one workgroup barrier it forms the outputs
// of its rows i2 = i2a + w + 7 k,  y = M2 f + K2 g  (band sums over staged rows), into an
// LDS output tile that the store wave writes out after the next barrier.  Coefficients
// are staged in LDS once.
// RES: the store wave writes r = b - A x (b loaded one output ahead) and the workgroup
// writes one partial sum of |r|^2.
template <int W, int RPW, int D, int C3MAX, bool RES>
__global__ __launch_bounds__(512) void k_kron3_stream(CBatch x, MBatch y, int n, int ntx, int nty, int nchunk,
                                                      int c3len, int64_t ntiles, KronBands bd, CBatch rhs,
                                                      MBatch part) {
  constexpr int NWC = 7;               // compute waves; wave 7 stores
  constexpr int NR = NWC * RPW;        // staged rows j2
  constexpr int NPLMAX = C3MAX + W - 1;  // planes j3 of a chunk (band starts growing by <= 1)
  constexpr int KO = (NR + NWC - 1) / NWC;  // output rows i2 per compute wave (T2 <= NR)
  __shared__ double xrow[NWC][RPW][64 + 8];
  __shared__ double zf[2][NR][64], zg[2][NR][64], ob[2][NR][64];
  // Band coefficients of directions 2 and 3 and the direction-3 band starts are uniform
  // per wave: they are read through the constant address space (scalar loads, scalar
  // registers, their own completion counter), so reading them never makes a wave wait
  // for its prefetched planes.
  typedef const __attribute__((address_space(4))) double cdbl;
  typedef const __attribute__((address_space(4))) int32_t cint;
  cdbl *M2c = (cdbl *)bd.M[1], *K2c = (cdbl *)bd.K[1], *M3c = (cdbl *)bd.M[2], *K3c = (cdbl *)bd.K[2];
  cint *lo2c = (cint *)bd.lo[1], *lo3c = (cint *)bd.lo[2];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // XCD-aware order: consecutive linear tiles (neighbours in i1, then i2, then i3) share
  // an XCD, so their halos meet in one L2; the grid is padded to a multiple of 8
  const int64_t nb = (int64_t)gridDim.x;
  const int64_t bid = blockIdx.x;
  const int64_t lin = (bid & 7) * (nb >> 3) + (bid >> 3);
  if (lin >= ntiles) return;
  const int tx = (int)(lin % ntx);
  int64_t rest = lin / ntx;
  const int ty = (int)(rest % nty);
  rest /= nty;
  const int64_t ent = rest / nchunk;
  const int64_t tile_in_ent = lin - ent * (int64_t)ntx * nty * nchunk;
  const int s3 = (int)(rest - ent * nchunk) * c3len;
  const int e3 = s3 + c3len < n ? s3 + c3len : n;
  const int nq = e3 - s3;
  const int64_t n2 = (int64_t)n * n;
  constexpr int w1 = W, w2 = W, w3 = W;  // the launcher checks that every band is W wide
  const int T2 = NR - w2 + 1;
  const int i1a = tx * 64, i2a = ty * T2;
  const int i1 = i1a + lane;
  const bool act1 = i1 < n;
  const int i1c = act1 ? i1 : n - 1;
  const int L0 = bd.lo[0][i1a];
  const int R0 = bd.lo[1][i2a];
  const int P0 = bd.lo[2][s3];
  const int NPL = bd.lo[2][e3 - 1] + w3 - P0;
  auto plane_of = [&](int q) { return lo3c[s3 + q] + w3 - 1 - P0; };  // plane completing output q
  double rr = 0.0;  // RES: this thread's part of |b - A x|^2
  if (wave == NWC) {
    // the store wave: output q - 1 after the barrier of output q, the last one after the
    // final barrier
    gptr<double> __restrict__ yb = y.gat(ent);
    gptr<const double> __restrict__ bbase = RES ? rhs.gat(ent) : nullptr;
    int offo[NR];  // this lane's output offsets within a plane (clamped; masked on store)
    bool oko[NR];
#pragma unroll
    for (int u2 = 0; u2 < NR; ++u2) {
      const int i2 = i2a + u2;
      oko[u2] = act1 && u2 < T2 && i2 < n;
      offo[u2] = oko[u2] ? i2 * n + i1 : 0;
    }
    double bn[NR];
    if (RES) {
#pragma unroll
      for (int u2 = 0; u2 < NR; ++u2) bn[u2] = bbase[(int64_t)s3 * n2 + offo[u2]];
    }
    for (int q = 0; q <= nq; ++q) {
      lds_barrier();
      if (q == 0) continue;
      const int i3 = s3 + q - 1, buf = (q - 1) & 1;
      gptr<double> yp = yb + (int64_t)i3 * n2;
      // every row of the output tile is read before any store is issued, so the LDS reads
      // are in flight together
      double v[NR];
#pragma unroll
      for (int u2 = 0; u2 < NR; ++u2) v[u2] = ob[buf][u2][lane];
      // keep the reads here (the compiler would otherwise sink each into its store's branch
      // and wait for them one at a time)
#pragma unroll
      for (int u2 = 0; u2 < NR; ++u2) asm volatile("" ::"v"(v[u2]));
      if (RES) {
        double bc[NR];
#pragma unroll
        for (int u2 = 0; u2 < NR; ++u2) bc[u2] = bn[u2];
        const int inext = q < nq ? s3 + q : i3;
#pragma unroll
        for (int u2 = 0; u2 < NR; ++u2) bn[u2] = bbase[(int64_t)inext * n2 + offo[u2]];
#pragma unroll
        for (int u2 = 0; u2 < NR; ++u2) {
          const double r = bc[u2] - v[u2];
          v[u2] = r;
          if (oko[u2]) rr = fma(r, r, rr);
        }
      }
#pragma unroll
      for (int u2 = 0; u2 < NR; ++u2)
        if (oko[u2]) yp[offo[u2]] = v[u2];
    }
  } else {
    gptr<const double> __restrict__ xb = x.gat(ent);
    const int off1 = bd.lo[0][i1c] - L0;  // in [0, 63]
    double m1[W], k1[W];  // direction-1 coefficients of this lane's column
#pragma unroll
    for (int t = 0; t < W; ++t) {
      m1[t] = bd.M[0][(size_t)i1c * w1 + t];
      k1[t] = bd.K[0][(size_t)i1c * w1 + t];
    }
    // window offsets of this wave's output rows (their coefficients are read per output)
    int b2[KO];
#pragma unroll
    for (int kk = 0; kk < KO; ++kk) {
      const int u2 = wave + NWC * kk, i2 = i2a + u2;
      b2[kk] = (u2 < T2 && i2 < n) ? lo2c[i2] - R0 : 0;
    }
    // this lane's elements of a plane: row R0 + wave + 7 k, column L0 + lane (and the halo
    // column L0 + 64 + lane for lane < w1 - 1), as offsets within a plane; outside the
    // tensor the offset is clamped to 0: such values only reach outputs beyond the tensor,
    // which are never stored, and every load is issued on every path
    int offm[RPW], offh[RPW];  // n^2 <= 2^20
#pragma unroll
    for (int k = 0; k < RPW; ++k) {
      const int r = R0 + wave + NWC * k;
      const bool rok = r < n;
      offm[k] = (rok && L0 + lane < n) ? r * n + L0 + lane : 0;
      offh[k] = (rok && lane < w1 - 1 && L0 + 64 + lane < n) ? r * n + L0 + 64 + lane : 0;
    }
    double pm[D][RPW], ph[D][RPW];  // prefetched planes (ring of D)
    auto issue = [&](int u, int pl) {
      gptr<const double> xp = xb + (int64_t)(P0 + (pl < NPL ? pl : NPL - 1)) * n2;
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        pm[u][k] = xp[offm[k]];
        ph[u][k] = xp[offh[k]];
      }
    };
#pragma unroll
    for (int u = 0; u < D; ++u) issue(u, u);
    double rm[RPW][W], rk[RPW][W];  // ring: sM, sK of plane pl in slot pl % W
#pragma unroll
    for (int k = 0; k < RPW; ++k)
#pragma unroll
      for (int t = 0; t < W; ++t) {
        rm[k][t] = 0.0;
        rk[k][t] = 0.0;
      }
    int q = 0;      // next output of the chunk
    // every plane step is unrolled: the prefetch ring is indexed statically and every load
    // is issued on every path, so each use waits for exactly the loads it needs
#pragma clang loop unroll(full)
    for (int pl = 0; pl < NPLMAX; ++pl) {
      const int u = pl % D;
      double vm[RPW], vh[RPW];
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        vm[k] = pm[u][k];
        vh[k] = ph[u][k];
      }
      if (pl + D < NPLMAX) issue(u, pl + D);
      if (pl < NPL) {
        // direction 1 on the wave's rows of plane pl
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
          xrow[wave][k][lane] = vm[k];
          if (lane < 8) xrow[wave][k][64 + lane] = vh[k];
        }
        lds_wave_sync();
#pragma unroll
        for (int k = 0; k < RPW; ++k) {
          double sm = 0.0, sk = 0.0;
#pragma unroll
          for (int t = 0; t < W; ++t) {
            const double v = xrow[wave][k][off1 + t];
            sm = fma(m1[t], v, sm);
            sk = fma(k1[t], v, sk);
          }
          rm[k][pl % W] = sm;
          rk[k][pl % W] = sk;
        }
        lds_wave_sync();
        // outputs whose direction-3 band ends at this plane
        while (q < nq && plane_of(q) == pl) {
          const int buf = q & 1;
          double k3[W], m3[W];
#pragma unroll
          for (int t = 0; t < W; ++t) {
            k3[t] = K3c[(size_t)(s3 + q) * W + t];
            m3[t] = M3c[(size_t)(s3 + q) * W + t];
          }
#pragma unroll
          for (int k = 0; k < RPW; ++k) {
            double f = 0.0, g = 0.0;
#pragma unroll
            for (int t = 0; t < W; ++t) {
              const int sl = (pl + 1 + t) % W;  // plane pl - W + 1 + t
              f = fma(k3[t], rm[k][sl], f);
              f = fma(m3[t], rk[k][sl], f);
              g = fma(m3[t], rm[k][sl], g);
            }
            zf[buf][wave + NWC * k][lane] = f;
            zg[buf][wave + NWC * k][lane] = g;
          }
          lds_barrier();
#pragma unroll
          for (int k = 0; k < KO; ++k) {
            const int u2 = wave + NWC * k;
            const int i2 = i2a + u2;
            if (u2 < T2 && i2 < n) {
              double acc = 0.0;
#pragma unroll
              for (int t = 0; t < W; ++t) {
                acc = fma(M2c[(size_t)i2 * W + t], zf[buf][b2[k] + t][lane], acc);
                acc = fma(K2c[(size_t)i2 * W + t], zg[buf][b2[k] + t][lane], acc);
              }
              ob[buf][u2][lane] = acc;
            }
          }
          ++q;
        }
      }
    }
    lds_barrier();  // the last output tile is complete
  }
  if (RES) {  // one partial per workgroup: the store wave's lanes in a fixed order
    if (wave == NWC) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) rr += __shfl_xor(rr, off, 64);
      if (lane == 0) part.gat(ent)[tile_in_ent] = rr;
    }
  }
}

}  // namespace

int kron_window_max() { return 16; }

bool kron_fused_ok(int n, int64_t nbatch, const KronBands &bd) {
#ifdef FDG_MV_NOFUSED  // tuning builds only: compare against the two-pass form
  return false;
#endif
  int w = 0;
  for (int l = 0; l < 3; ++l) w = bd.w[l] > w ? bd.w[l] : w;
  return w <= 8 && bd.step[0] <= 1 && bd.step[1] <= 1 && bd.step[2] <= 1 &&
         (int64_t)n * n * nbatch < ((int64_t)1 << 31);
}

bool kron_two_pass_ok(int d, int n, int64_t nbatch, const KronBands &bd) {
  if (d != 3) return true;
  int w = 0;
  for (int l = 0; l < d; ++l) w = bd.w[l] > w ? bd.w[l] : w;
  return bd.rows16 <= kPlaneRowsMax && bd.step3 <= 1 && w <= 8 && (int64_t)n * nbatch <= 65535;
}

namespace {

// Shape of the streaming one-pass form: D = 2 planes loaded ahead (the measured best at
// n = 128 and 192; deeper rings cost occupancy), and per band width w the staged rows j2
// per compute wave (RPW) and the outputs i3 per chunk.  Measured on MI355X (us per
// product, RPW in {2, 3, 4} x chunk in {4, 6, 8}): wide bands want tall tiles, whose
// halo share 1 - T2 / (7 RPW) is smaller (p = 6, w = 7: 192^3 92.8 -> 74.2 with RPW 4,
// 128^3 28.7 -> 26.9); narrow bands want more, shorter chunks (w <= 4: 96^3 p = 3
// 11.3 -> 9.9, 128^3 p = 2 16.1 -> 14.5 with chunks of 6); w = 5, 6 keep RPW 2 and
// chunks of 8 (128^3 p = 4: 19.2, every other shape 19.1-33.9).
#ifndef FDG_MV_D
#define FDG_MV_D 2
#endif
constexpr int kStreamD = FDG_MV_D;
constexpr int stream_rpw(int w) { return w >= 7 ? 4 : 2; }
constexpr int stream_chunk(int w) { return w <= 4 ? 6 : 8; }

struct StreamShape {
  int ntx, nty, nchunk, c3len;
  int64_t tiles() const { return (int64_t)ntx * nty * nchunk; }
};

StreamShape stream_shape(int n, const KronBands &bd) {
  StreamShape sh;
  const int w = bd.w[1];
  const int T2 = 7 * stream_rpw(w) - w + 1;
  sh.ntx = (int)cdiv(n, 64);
  sh.nty = (int)cdiv(n, T2);
  sh.c3len = stream_chunk(w);
  sh.nchunk = (int)cdiv(n, sh.c3len);
  return sh;
}

// The streaming form needs one band width W in [2, 8] for all three directions, and it
// is taken when it has at least 128 workgroups per entry: each of its workgroups walks
// its planes one after the other, so on small grids the one-wave-per-plane form, which
// spreads the planes over more waves, finishes first (measured on MI355X: 64^3 p = 2
// 8.1 against 10.4 us, 48^3 p = 3 7.9 against 10.2; from 80^3 p = 4 on the streaming form
// is faster).  The choice depends on n and the bands only.
bool stream_ok(int n, const KronBands &bd) {
  return bd.w[0] == bd.w[1] && bd.w[1] == bd.w[2] && bd.w[0] >= 2 && bd.w[0] <= 8 &&
         stream_shape(n, bd).tiles() >= 128;
}

constexpr int kWppT2 = FDG_MV_T2, kWppC3 = FDG_MV_C3;

int64_t wpp_tiles(int n, const KronBands &bd) {
  if (stream_ok(n, bd)) return stream_shape(n, bd).tiles();
  return (int64_t)cdiv(n, 64) * cdiv(n, kWppT2) * cdiv(n, kWppC3);
}

template <bool RES>
void launch_wpp(hipStream_t s, CBatch x, MBatch y, int n, int64_t nbatch, const KronBands &bd, CBatch rhs,
                MBatch part) {
  int w = 0;
  for (int l = 0; l < 3; ++l) w = bd.w[l] > w ? bd.w[l] : w;
  if (stream_ok(n, bd)) {
    const StreamShape sh = stream_shape(n, bd);
    const int64_t ntiles = sh.tiles() * nbatch;
    const dim3 grid((unsigned)((ntiles + 7) / 8 * 8));
#define FDG_STREAM(WW, C3)                                                                                   \
  hipLaunchKernelGGL((k_kron3_stream<WW, stream_rpw(WW), kStreamD, C3, RES>), grid, dim3(512), 0, s, x, y, n, sh.ntx, \
                     sh.nty, sh.nchunk, sh.c3len, ntiles, bd, rhs, part)
    switch (w) {
      case 2: FDG_STREAM(2, 8); break;
      case 3: FDG_STREAM(3, 8); break;
      case 4: FDG_STREAM(4, 8); break;
      case 5: FDG_STREAM(5, 8); break;
      case 6: FDG_STREAM(6, 8); break;
      case 7: FDG_STREAM(7, 8); break;
      default: FDG_STREAM(8, 8); break;
    }
#undef FDG_STREAM
    return;
  }
  const int ntx = (int)cdiv(n, 64), nty = (int)cdiv(n, kWppT2), nchunk = (int)cdiv(n, kWppC3);
  const dim3 grid((unsigned)((int64_t)ntx * nty * nchunk * nbatch));
  if (w <= 4)
    hipLaunchKernelGGL((k_kron3_wpp<4, kWppT2, kWppC3, RES>), grid, dim3(512), 0, s, x, y, n, ntx, nty, nchunk, bd,
                       rhs, part);
  else if (w <= 6)
    hipLaunchKernelGGL((k_kron3_wpp<6, kWppT2, kWppC3, RES>), grid, dim3(512), 0, s, x, y, n, ntx, nty, nchunk, bd,
                       rhs, part);
  else
    hipLaunchKernelGGL((k_kron3_wpp<8, kWppT2, kWppC3, RES>), grid, dim3(512), 0, s, x, y, n, ntx, nty, nchunk, bd,
                       rhs, part);
}

}  // namespace

int kron_residual_partials(int d, int n, const KronBands &bd) {
  if (d != 3 || !kron_fused_ok(n, 1, bd)) return 0;
  return (int)wpp_tiles(n, bd);
}

bool launch_kron_residual_f64(hipStream_t s, CBatch x, CBatch rhs, MBatch r, int d, int n, int64_t nbatch,
                              const KronBands &bd, MBatch part) {
  if (d != 3 || !kron_fused_ok(n, nbatch, bd)) return false;
  launch_wpp<true>(s, x, r, n, nbatch, bd, rhs, part);
  return true;
}

bool launch_kron_matvec_f64(hipStream_t s, CBatch x, MBatch y, int d, int n, int64_t nbatch, const KronBands &bd,
                            MBatch tmp_a, MBatch tmp_c) {
  int w = 0;
  for (int l = 0; l < d; ++l) w = bd.w[l] > w ? bd.w[l] : w;
  const dim3 blk(kBlock);
  if (d == 3 && kron_fused_ok(n, nbatch, bd)) {
    launch_wpp<false>(s, x, y, n, nbatch, bd, CBatch{}, MBatch{});
    return true;
  }
  if (d == 3) {
    if (tmp_a.valid() && tmp_c.valid() && kron_two_pass_ok(d, n, nbatch, bd)) {
      const dim3 g1(cdiv(n, 64), cdiv(n, kPlaneRows), (unsigned)(n * nbatch));
      const int ngroups = (int)cdiv(n, kRowsPerThread);
      const dim3 g2(cdiv((int64_t)n * n, kBlock), (unsigned)(ngroups * nbatch));
      if (w <= 4) {
        hipLaunchKernelGGL(k_kron3_planes<4>, g1, blk, 0, s, x, tmp_a, tmp_c, n, bd);
        hipLaunchKernelGGL(k_kron3_mode3<4>, g2, blk, 0, s, as_const(tmp_a), as_const(tmp_c), y, n, ngroups, bd);
      } else {
        hipLaunchKernelGGL(k_kron3_planes<8>, g1, blk, 0, s, x, tmp_a, tmp_c, n, bd);
        hipLaunchKernelGGL(k_kron3_mode3<8>, g2, blk, 0, s, as_const(tmp_a), as_const(tmp_c), y, n, ngroups, bd);
      }
      return true;
    }
    if (x.ptrs || y.ptrs) return false;  // the one-pass forms take contiguous batches only
    const double *xc = x.base;
    double *yc = y.base;
    if (bd.rows4 <= kRowsMax && w <= 8) {
      const int nchunk = (int)cdiv(n, kChunk);
      const dim3 grid(cdiv(n, 64), cdiv(n, 4), (unsigned)(nchunk * nbatch));
      if (w <= 4)
        hipLaunchKernelGGL(k_kron3_lds<4>, grid, blk, 0, s, xc, yc, n, nchunk, bd);
      else
        hipLaunchKernelGGL(k_kron3_lds<8>, grid, blk, 0, s, xc, yc, n, nchunk, bd);
      return true;
    }
    const dim3 grid(cdiv((int64_t)n * n, kBlock), cdiv(n, kChunk), (unsigned)nbatch);
    if (w <= 4)
      hipLaunchKernelGGL(k_kron3_window<4>, grid, blk, 0, s, xc, yc, n, bd);
    else if (w <= 8)
      hipLaunchKernelGGL(k_kron3_window<8>, grid, blk, 0, s, xc, yc, n, bd);
    else
      hipLaunchKernelGGL(k_kron3_window<16>, grid, blk, 0, s, xc, yc, n, bd);
  } else {
    const dim3 grid(cdiv(n, kBlock), cdiv(n, kChunk), (unsigned)nbatch);
    if (w <= 4)
      hipLaunchKernelGGL(k_kron2_window<4>, grid, blk, 0, s, x, y, n, bd);
    else if (w <= 8)
      hipLaunchKernelGGL(k_kron2_window<8>, grid, blk, 0, s, x, y, n, bd);
    else
      hipLaunchKernelGGL(k_kron2_window<16>, grid, blk, 0, s, x, y, n, bd);
  }
  return true;
}

// The same with implicit columns: row r = (i1, i2, i3) reads x along the rows of its
// window, w1 consecutive elements at a time; lane group g takes window rows
// q = t3 w2 + t2 = g, g + S, ...  lo holds lo1 (n), lo2 (n), lo3 (n) back to back.
template <int S>
__global__ __launch_bounds__(kBlock) void k_ell_tensor_f64(CBatch x, MBatch y, int n, int64_t nrows, int w1,
                                                           int w2, int w3, const int32_t *__restrict__ lo,
                                                           const double *__restrict__ val) {
  constexpr int R = 64 / S;
  const int lane = threadIdx.x & 63;
  const int g = lane / R;
  const int64_t row = ((int64_t)blockIdx.x * kBlock + (threadIdx.x & ~63)) / S + (lane % R);
  const bool ok = row < nrows;
  const int64_t b = blockIdx.y;
  gptr<const double> __restrict__ xb = x.gat(b);
  const int64_t n2 = (int64_t)n * n;
  double acc = 0.0;
  if (ok) {
    const int i1 = (int)(row % n), i2 = (int)((row / n) % n), i3 = (int)(row / n2);
    gptr<const double> __restrict__ x0 = xb + lo[i1] + (int64_t)n * lo[n + i2] + n2 * lo[2 * n + i3];
    const int nq = w2 * w3;
    for (int q = g; q < nq; q += S) {
      const int t3 = q / w2, t2 = q - t3 * w2;
      gptr<const double> __restrict__ xr = x0 + (int64_t)n * t2 + n2 * t3;
      const double *__restrict__ vr = val + (int64_t)q * w1 * nrows + row;
      for (int t1 = 0; t1 < w1; ++t1) acc = fma(vr[(int64_t)t1 * nrows], xr[t1], acc);
    }
  }
#pragma unroll
  for (int m = R; m < 64; m <<= 1) acc += __shfl_xor(acc, m);
  if (ok && g == 0) y.gat(b)[row] = acc;
}

// The same for the common cube stencils w1 = w2 = w3 = W (3: collocation p = 2, 3 at
// exact Greville points; 7: Galerkin p = 3 and the literal (2p+1)^3 stencil; 4 as well):
// the window row unrolled, FDG_ELL_QU window rows per step and 32-bit row arithmetic
// (nrows * 8 < 2^32, checked by the launcher).  Same fma order as the generic form, so the
// result is bitwise the same.  Measured on MI355X (back-to-back products): 27-wide rows at
// N = 96^3 36.5 -> 31.8 us (6.5 TB/s); 343-wide rows at 96^3 529 -> 443 us (5.5 TB/s), at
// 48^3 with 4 lanes per row 66.8 -> 58.0 us.  With 2 lanes per row (343 wide at 64^3) it
// measured 5% slower than the generic form, which keeps that case.
#ifndef FDG_ELL_FIXED
#define FDG_ELL_FIXED 1  // 0: generic form only (tuning builds)
#endif
#ifndef FDG_ELL_QU
#define FDG_ELL_QU 3  // window rows per unrolled step (1 measured 7% slower at 96^3, 27 wide)
#endif
template <int S, int W>
__global__ __launch_bounds__(kBlock) void k_ell_tensor_w_f64(CBatch x, MBatch y, int n, int64_t nrows,
                                                             const int32_t *__restrict__ lo,
                                                             const double *__restrict__ val) {
  constexpr int R = 64 / S;
  constexpr int NQ = W * W;
  const int lane = threadIdx.x & 63;
  const int g = lane / R;
  const unsigned row = ((unsigned)blockIdx.x * kBlock + (threadIdx.x & ~63)) / S + (lane % R);
  const bool ok = row < (unsigned)nrows;
  const int64_t b = blockIdx.y;
  gptr<const double> __restrict__ xb = x.gat(b);
  const unsigned un = (unsigned)n;
  const int64_t n2 = (int64_t)n * n;
  double acc = 0.0;
  if (ok) {
    const unsigned rq = row / un;
    const int i1 = (int)(row - rq * un), i2 = (int)(rq % un), i3 = (int)(rq / un);
    gptr<const double> __restrict__ x0 = xb + lo[i1] + (int64_t)n * lo[n + i2] + n2 * lo[2 * n + i3];
#pragma unroll FDG_ELL_QU
    for (int qq = 0; qq < NQ; qq += S) {
      const int q = qq + g;
      if (S > 1 && q >= NQ) break;
      const int t3 = q / W, t2 = q - t3 * W;
      gptr<const double> __restrict__ xr = x0 + (int64_t)n * t2 + n2 * t3;
#pragma unroll
      for (int t1 = 0; t1 < W; ++t1) {
        acc = fma(val[(int64_t)(q * W + t1) * nrows + row], xr[t1], acc);
      }
    }
  }
#pragma unroll
  for (int m = R; m < 64; m <<= 1) acc += __shfl_xor(acc, m);
  if (ok && g == 0) y.gat(b)[row] = acc;
}

// Lanes per row: doubled (up to 4) while the launch has fewer than ~400K lanes and each
// lane keeps at least 16 slots.  Measured on MI355X: the 27-wide collocation rows at
// N = 96^3 run best with 1 lane per row (4.8 TB/s); the 343-wide Galerkin rows with 4 at
// N = 48^3 (4.4 TB/s against 1.7 with 1) and 2 at N = 64^3 (4.8 TB/s).
#ifndef FDG_ELL_SPLIT
#define FDG_ELL_SPLIT 0
#endif
int ell_split(int64_t nrows, int width) {
  if (FDG_ELL_SPLIT > 0) return FDG_ELL_SPLIT;
  int S = 1;
  while (S < 4 && nrows * S < 400000 && width >= 32 * S) S *= 2;
  return S;
}

void launch_ell_matvec_f64(hipStream_t s, CBatch x, MBatch y, int64_t nrows, int64_t ld, int width,
                           const int32_t *col, const double *val, int64_t nbatch) {
  const int S = ell_split(nrows, width);
  const dim3 grid(cdiv(nrows * S, kBlock), (unsigned)nbatch), blk(kBlock);
  switch (S) {
    case 1: hipLaunchKernelGGL(k_ell_f64<1>, grid, blk, 0, s, x, y, nrows, ld, width, col, val); break;
    case 2: hipLaunchKernelGGL(k_ell_f64<2>, grid, blk, 0, s, x, y, nrows, ld, width, col, val); break;
    case 4: hipLaunchKernelGGL(k_ell_f64<4>, grid, blk, 0, s, x, y, nrows, ld, width, col, val); break;
    default: hipLaunchKernelGGL(k_ell_f64<8>, grid, blk, 0, s, x, y, nrows, ld, width, col, val); break;
  }
}

void launch_ell_tensor_f64(hipStream_t s, CBatch x, MBatch y, int n, int d, const int w[3], const int32_t *lo,
                           const double *val, int64_t nbatch) {
  const int64_t nrows = d == 3 ? (int64_t)n * n * n : (int64_t)n * n;
  const int width = w[0] * w[1] * w[2];
  const int S = ell_split(nrows, width);
  const dim3 grid(cdiv(nrows * S, kBlock), (unsigned)nbatch), blk(kBlock);
  const int W = (w[0] == w[1] && w[1] == w[2]) ? w[0] : 0;
  if (FDG_ELL_FIXED > 0 && d == 3 && nrows * 8 < (int64_t(1) << 32) && (W == 3 || W == 4 || W == 7)) {
#define FDG_ELLW(SS, WW) \
  if (S == SS && W == WW) {  \
    hipLaunchKernelGGL((k_ell_tensor_w_f64<SS, WW>), grid, blk, 0, s, x, y, n, nrows, lo, val); \
    return;                  \
  }
    FDG_ELLW(1, 3) FDG_ELLW(4, 3) FDG_ELLW(1, 4) FDG_ELLW(4, 4) FDG_ELLW(1, 7) FDG_ELLW(4, 7)
#undef FDG_ELLW
  }
  switch (S) {
    case 1: hipLaunchKernelGGL(k_ell_tensor_f64<1>, grid, blk, 0, s, x, y, n, nrows, w[0], w[1], w[2], lo, val); break;
    case 2: hipLaunchKernelGGL(k_ell_tensor_f64<2>, grid, blk, 0, s, x, y, n, nrows, w[0], w[1], w[2], lo, val); break;
    case 4: hipLaunchKernelGGL(k_ell_tensor_f64<4>, grid, blk, 0, s, x, y, n, nrows, w[0], w[1], w[2], lo, val); break;
    default: hipLaunchKernelGGL(k_ell_tensor_f64<8>, grid, blk, 0, s, x, y, n, nrows, w[0], w[1], w[2], lo, val); break;
  }
}

}  // namespace fdg
