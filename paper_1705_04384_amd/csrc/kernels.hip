// Device kernels of the FD-preconditioned flexible GMRES path (gfx950, wave64).
//
//  * FD mode products (eq. 4.7 / 4.9): every mode product of the fast-diagonalization
//    solve is a small dense contraction Y = W x_l X with a zero-padded n x n factor W,
//    run on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//  * The diagonal solve of eq. 4.9 (divide by the sum of univariate eigenvalues).
//  * The unit-domain operator of eq. 2.9 / 2.7 applied from the banded univariate factors.
//  * A slot-major ELL sparse matvec for an assembled operator.
//  * Krylov vector kernels with fixed-order (deterministic) block reductions.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace fdg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;

int reduction_blocks(int64_t N) {
  int64_t g = (N + 4095) / 4096;
  if (g < 1) g = 1;
  if (g > 256) g = 256;
  return (int)g;
}

static inline unsigned grid1(int64_t work, int per_block) {
  return (unsigned)((work + per_block - 1) / per_block);
}

// ------------------------------------------------------------------------------------
// Mode product, FP64 MFMA.  One workgroup (4 waves) computes a 64 (k) x 64 (c) output
// tile; wave w owns a 32 x 32 quarter = 2 x 2 MFMA tiles of 16 x 16.
// v_mfma_f64_16x16x4_f64 operand layout (lane l, li = l % 16, lg = l / 16):
//   A[m = li][k = lg],  B[k = lg][n = li],  D[m = lg + 4*r][n = li] in register r
// (the FP32 16x16x4 form instead returns D[m = 4*lg + r][n = li]).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_modeprod_f64(const double *__restrict__ X,
                                                         double *__restrict__ Y,
                                                         const double *__restrict__ W, int ldw, int n,
                                                         int64_t ncols, int64_t sO, int64_t sJ,
                                                         int64_t sC) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t c0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
  const int k0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int64_t o = blockIdx.z;
  const double *Xo = X + o * sO;
  double *Yo = Y + o * sO;
  dbl4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  const double *Wr0 = W + (size_t)(k0 + li) * ldw;
  const double *Wr1 = W + (size_t)(k0 + 16 + li) * ldw;
  const int64_t cA = c0 + li, cB = c0 + 16 + li;
  const bool okA = cA < ncols, okB = cB < ncols;
  for (int j0 = 0; j0 < n; j0 += 4) {
    const int j = j0 + lg;
    const double a0 = Wr0[j], a1 = Wr1[j];
    const bool jok = j < n;
    const double b0 = (jok && okA) ? Xo[j * sJ + cA * sC] : 0.0;
    const double b1 = (jok && okB) ? Xo[j * sJ + cB * sC] : 0.0;
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  for (int ti = 0; ti < 2; ++ti)
    for (int tj = 0; tj < 2; ++tj) {
      const int64_t c = c0 + 16 * tj + li;
      if (c >= ncols) continue;
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + 16 * ti + lg + 4 * r;
        if (k < n) Yo[k * sJ + c * sC] = acc[ti][tj][r];
      }
    }
}

void launch_modeprod_f64(hipStream_t s, const double *X, double *Y, const double *W, int ldw, int n,
                         int64_t ncols, int64_t sO, int64_t sJ, int64_t sC, int64_t nbatch) {
  for (int64_t o0 = 0; o0 < nbatch; o0 += 65535) {
    const int64_t nb = nbatch - o0 < 65535 ? nbatch - o0 : 65535;
    dim3 grid(grid1(ncols, 64), (unsigned)((n + 63) / 64), (unsigned)nb);
    hipLaunchKernelGGL(k_modeprod_f64, grid, dim3(kBlock), 0, s, X + o0 * sO, Y + o0 * sO, W, ldw, n,
                       ncols, sO, sJ, sC);
  }
}

__global__ __launch_bounds__(kBlock) void k_divide_f64(double *__restrict__ t, int d, int n,
                                                       int64_t total, const double *__restrict__ l1,
                                                       const double *__restrict__ l2,
                                                       const double *__restrict__ l3) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int i1 = (int)(idx % n);
  const int i2 = (int)((idx / n) % n);
  double den = l1[i1] + l2[i2];
  if (d == 3) den += l3[(idx / ((int64_t)n * n)) % n];
  t[idx] = t[idx] / den;
}

void launch_divide_f64(hipStream_t s, double *t, int d, int n, int64_t nbatch, const double *lam1,
                       const double *lam2, const double *lam3) {
  int64_t N = (int64_t)n * n * (d == 3 ? n : 1);
  const int64_t total = N * nbatch;
  hipLaunchKernelGGL(k_divide_f64, dim3(grid1(total, kBlock)), dim3(kBlock), 0, s, t, d, n, total, lam1,
                     lam2, lam3);
}

// ------------------------------------------------------------------------------------
// Unit-domain operator from banded factors, one output per thread; the innermost band
// sum is shared by the M_1 and K_1 terms:
//   3D: y = sum_{j3,j2} [(K3 M2 + M3 K2) (M1 x) + M3 M2 (K1 x)]
//   2D: y = sum_{j2} [K2 (M1 x) + M2 (K1 x)]
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_kron3_f64(const double *__restrict__ x, double *__restrict__ y,
                                                      int n, int64_t total, KronBands bd) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int64_t N = (int64_t)n * n * n;
  const int64_t b = idx / N, r = idx - b * N;
  const int i1 = (int)(r % n), i2 = (int)((r / n) % n), i3 = (int)(r / ((int64_t)n * n));
  const double *xb = x + b * N;
  const int w1 = bd.w[0], w2 = bd.w[1], w3 = bd.w[2];
  const int lo1 = bd.lo[0][i1], lo2 = bd.lo[1][i2], lo3 = bd.lo[2][i3];
  const double *M1 = bd.M[0] + (size_t)i1 * w1, *K1 = bd.K[0] + (size_t)i1 * w1;
  const double *M2 = bd.M[1] + (size_t)i2 * w2, *K2 = bd.K[1] + (size_t)i2 * w2;
  const double *M3 = bd.M[2] + (size_t)i3 * w3, *K3 = bd.K[2] + (size_t)i3 * w3;
  double acc = 0.0;
  for (int t3 = 0; t3 < w3; ++t3) {
    const double m3 = M3[t3], k3 = K3[t3];
    if (m3 == 0.0 && k3 == 0.0) continue;
    const double *xp = xb + (int64_t)(lo3 + t3) * n * n;
    for (int t2 = 0; t2 < w2; ++t2) {
      const double m2 = M2[t2], k2 = K2[t2];
      if (m2 == 0.0 && k2 == 0.0) continue;
      const double *xr = xp + (int64_t)(lo2 + t2) * n + lo1;
      double sm = 0.0, sk = 0.0;
      for (int t1 = 0; t1 < w1; ++t1) {
        const double v = xr[t1];
        sm = fma(M1[t1], v, sm);
        sk = fma(K1[t1], v, sk);
      }
      acc = fma(k3 * m2 + m3 * k2, sm, acc);
      acc = fma(m3 * m2, sk, acc);
    }
  }
  y[idx] = acc;
}

__global__ __launch_bounds__(kBlock) void k_kron2_f64(const double *__restrict__ x, double *__restrict__ y,
                                                      int n, int64_t total, KronBands bd) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int64_t N = (int64_t)n * n;
  const int64_t b = idx / N, r = idx - b * N;
  const int i1 = (int)(r % n), i2 = (int)(r / n);
  const double *xb = x + b * N;
  const int w1 = bd.w[0], w2 = bd.w[1];
  const int lo1 = bd.lo[0][i1], lo2 = bd.lo[1][i2];
  const double *M1 = bd.M[0] + (size_t)i1 * w1, *K1 = bd.K[0] + (size_t)i1 * w1;
  const double *M2 = bd.M[1] + (size_t)i2 * w2, *K2 = bd.K[1] + (size_t)i2 * w2;
  double acc = 0.0;
  for (int t2 = 0; t2 < w2; ++t2) {
    const double m2 = M2[t2], k2 = K2[t2];
    const double *xr = xb + (int64_t)(lo2 + t2) * n + lo1;
    double sm = 0.0, sk = 0.0;
    for (int t1 = 0; t1 < w1; ++t1) {
      const double v = xr[t1];
      sm = fma(M1[t1], v, sm);
      sk = fma(K1[t1], v, sk);
    }
    acc = fma(k2, sm, acc);
    acc = fma(m2, sk, acc);
  }
  y[idx] = acc;
}

void launch_kron_matvec_f64(hipStream_t s, const double *x, double *y, int d, int n, int64_t nbatch,
                            const KronBands &bands) {
  const int64_t N = (int64_t)n * n * (d == 3 ? n : 1);
  const int64_t total = N * nbatch;
  if (d == 3)
    hipLaunchKernelGGL(k_kron3_f64, dim3(grid1(total, kBlock)), dim3(kBlock), 0, s, x, y, n, total, bands);
  else
    hipLaunchKernelGGL(k_kron2_f64, dim3(grid1(total, kBlock)), dim3(kBlock), 0, s, x, y, n, total, bands);
}

__global__ __launch_bounds__(kBlock) void k_ell_f64(const double *__restrict__ x, double *__restrict__ y,
                                                    int64_t nrows, int64_t ld, int width,
                                                    const int32_t *__restrict__ col,
                                                    const double *__restrict__ val, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int64_t b = idx / nrows, row = idx - b * nrows;
  const double *xb = x + b * nrows;
  double acc = 0.0;
  for (int t = 0; t < width; ++t) {
    const int64_t e = (int64_t)t * ld + row;
    acc = fma(val[e], xb[col[e]], acc);
  }
  y[idx] = acc;
}

void launch_ell_matvec_f64(hipStream_t s, const double *x, double *y, int64_t nrows, int64_t ld, int width,
                           const int32_t *col, const double *val, int64_t nbatch) {
  const int64_t total = nrows * nbatch;
  hipLaunchKernelGGL(k_ell_f64, dim3(grid1(total, kBlock)), dim3(kBlock), 0, s, x, y, nrows, ld, width, col,
                     val, total);
}

// ------------------------------------------------------------------------------------
// Krylov vector kernels.  Block g of batch entry b handles the contiguous chunk
// [g*chunk, min(N, (g+1)*chunk)) with chunk = ceil(N / G); sums are reduced in a fixed
// order (thread-strided accumulation, a butterfly within the wave, then the four waves
// in order), so results are bitwise reproducible for a given N.
// ------------------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int kQB = 8;  // basis vectors per register batch

__global__ __launch_bounds__(kBlock) void k_dots(const double *__restrict__ V, int64_t ldv, int nv,
                                                 const double *__restrict__ w, int64_t N, int G,
                                                 double *__restrict__ P) {
  __shared__ double red[kBlock / 64][kQB];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int64_t chunk = (N + G - 1) / G;
  const int64_t beg = (int64_t)g * chunk;
  const int64_t end = beg + chunk < N ? beg + chunk : N;
  const double *wb = w + b * N;
  const double *Vb = V + b * N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q0 = 0; q0 < nv; q0 += kQB) {
    double acc[kQB];
#pragma unroll
    for (int t = 0; t < kQB; ++t) acc[t] = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
      const double wi = wb[i];
#pragma unroll
      for (int t = 0; t < kQB; ++t)
        if (q0 + t < nv) acc[t] = fma(Vb[(int64_t)(q0 + t) * ldv + i], wi, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < kQB; ++t) {
      const double v = wave_sum(acc[t]);
      if (lane == 0) red[wave][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < kQB && q0 + (int)threadIdx.x < nv) {
      const int t = threadIdx.x;
      double s = red[0][t];
      for (int k = 1; k < kBlock / 64; ++k) s += red[k][t];
      P[((int64_t)b * G + g) * nv + q0 + t] = s;
    }
    __syncthreads();
  }
}

void launch_dots(hipStream_t s, const double *V, int64_t ldv, int nv, const double *w, int64_t N,
                 int64_t nbatch, int G, double *P) {
  hipLaunchKernelGGL(k_dots, dim3(G, (unsigned)nbatch), dim3(kBlock), 0, s, V, ldv, nv, w, N, G, P);
}

constexpr int kMaxBasis = 256;

__global__ __launch_bounds__(kBlock) void k_update(const double *__restrict__ V, int64_t ldv, int nv,
                                                   const double *__restrict__ Pin, int G,
                                                   double *__restrict__ w, int64_t N,
                                                   double *__restrict__ Pnorm) {
  __shared__ double h[kMaxBasis];
  __shared__ double red[kBlock / 64];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  for (int q = threadIdx.x; q < nv; q += kBlock) {
    const double *p = Pin + (int64_t)b * G * nv + q;
    double s = 0.0;
    for (int k = 0; k < G; ++k) s += p[(int64_t)k * nv];
    h[q] = s;
  }
  __syncthreads();
  const int64_t chunk = (N + G - 1) / G;
  const int64_t beg = (int64_t)g * chunk;
  const int64_t end = beg + chunk < N ? beg + chunk : N;
  double *wb = w + b * N;
  const double *Vb = V + b * N;
  double nrm = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    double wi = wb[i];
    for (int q = 0; q < nv; ++q) wi = fma(-Vb[(int64_t)q * ldv + i], h[q], wi);
    wb[i] = wi;
    nrm = fma(wi, wi, nrm);
  }
  if (Pnorm) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double v = wave_sum(nrm);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = red[0];
      for (int k = 1; k < kBlock / 64; ++k) s += red[k];
      Pnorm[(int64_t)b * G + g] = s;
    }
  }
}

void launch_update(hipStream_t s, const double *V, int64_t ldv, int nv, const double *Pin, int G, double *w,
                   int64_t N, int64_t nbatch, double *Pnorm) {
  hipLaunchKernelGGL(k_update, dim3(G, (unsigned)nbatch), dim3(kBlock), 0, s, V, ldv, nv, Pin, G, w, N, Pnorm);
}

__global__ void k_finalize_h(const double *__restrict__ P1, const double *__restrict__ P2,
                             const double *__restrict__ P3, int G, int nv, double *__restrict__ Hcol) {
  const int64_t b = blockIdx.x;
  for (int q = threadIdx.x; q <= nv; q += blockDim.x) {
    double s;
    if (q < nv) {
      // the same fixed-order sums as k_update forms for h1 and h2
      double s1 = 0.0, s2 = 0.0;
      for (int k = 0; k < G; ++k) s1 += P1[(b * G + k) * nv + q];
      for (int k = 0; k < G; ++k) s2 += P2[(b * G + k) * nv + q];
      s = s1 + s2;
    } else {
      double s3 = 0.0;
      for (int k = 0; k < G; ++k) s3 += P3[b * G + k];
      s = sqrt(s3);
    }
    Hcol[b * (nv + 1) + q] = s;
  }
}

void launch_finalize_h(hipStream_t s, const double *P1, const double *P2, const double *P3, int G, int nv,
                       int64_t nbatch, double *Hcol) {
  hipLaunchKernelGGL(k_finalize_h, dim3((unsigned)nbatch), dim3(64), 0, s, P1, P2, P3, G, nv, Hcol);
}

__global__ void k_finalize_norm(const double *__restrict__ P, int G, double *__restrict__ out) {
  const int64_t b = blockIdx.x;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int k = 0; k < G; ++k) s += P[b * G + k];
    out[b] = sqrt(s);
  }
}

void launch_finalize_norm(hipStream_t s, const double *P, int G, int64_t nbatch, double *out) {
  hipLaunchKernelGGL(k_finalize_norm, dim3((unsigned)nbatch), dim3(64), 0, s, P, G, out);
}

__global__ __launch_bounds__(kBlock) void k_scale(const double *__restrict__ w, double *__restrict__ v,
                                                  const double *__restrict__ nrm, int nstride, int64_t N,
                                                  int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const double d = nrm[(idx / N) * nstride];
  v[idx] = d != 0.0 ? w[idx] / d : 0.0;
}

void launch_scale(hipStream_t s, const double *w, double *v, const double *nrm, int nstride, int64_t N,
                  int64_t nbatch) {
  const int64_t total = N * nbatch;
  hipLaunchKernelGGL(k_scale, dim3(grid1(total, kBlock)), dim3(kBlock), 0, s, w, v, nrm, nstride, N, total);
}

__global__ __launch_bounds__(kBlock) void k_lincomb(double *__restrict__ x, const double *__restrict__ Z,
                                                    int64_t ldz, int k, const double *__restrict__ y,
                                                    int ystride, int64_t N, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const int64_t b = idx / N;
  const double *yb = y + b * ystride;
  double acc = x[idx];
  for (int q = 0; q < k; ++q) acc = fma(Z[(int64_t)q * ldz + idx], yb[q], acc);
  x[idx] = acc;
}

void launch_lincomb(hipStream_t s, double *x, const double *Z, int64_t ldz, int k, const double *y,
                    int ystride, int64_t N, int64_t nbatch) {
  const int64_t total = N * nbatch;
  hipLaunchKernelGGL(k_lincomb, dim3(grid1(total, kBlock)), dim3(kBlock), 0, s, x, Z, ldz, k, y, ystride, N,
                     total);
}

__global__ __launch_bounds__(kBlock) void k_residual(const double *__restrict__ bv,
                                                     const double *__restrict__ Ax, double *__restrict__ r,
                                                     int64_t N, int G, double *__restrict__ P) {
  __shared__ double red[kBlock / 64];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int64_t chunk = (N + G - 1) / G;
  const int64_t beg = (int64_t)g * chunk;
  const int64_t end = beg + chunk < N ? beg + chunk : N;
  double nrm = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    const int64_t e = b * N + i;
    const double v = bv[e] - Ax[e];
    r[e] = v;
    nrm = fma(v, v, nrm);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double v = wave_sum(nrm);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = red[0];
    for (int k = 1; k < kBlock / 64; ++k) s += red[k];
    P[b * G + g] = s;
  }
}

void launch_residual(hipStream_t s, const double *b, const double *Ax, double *r, int64_t N, int64_t nbatch,
                     int G, double *P) {
  hipLaunchKernelGGL(k_residual, dim3(G, (unsigned)nbatch), dim3(kBlock), 0, s, b, Ax, r, N, G, P);
}

}  // namespace fdg
