// Krylov vector kernels of flexible GMRES: multi-dot products, Gram-Schmidt updates,
// norms, scaling and the final linear combination x += Z y.
//
// Reductions are deterministic: block g of batch entry b sums the contiguous chunk
// [g*chunk, min(N, (g+1)*chunk)) in a fixed order (thread-strided accumulation, an xor
// butterfly inside each wave, then the waves in index order) and writes one partial
// sum; a one-block reduce kernel then sums the G partials (lane t takes g = t, t+64, ...
// in increasing order, then an xor butterfly, which leaves the same bits in every lane).
// G depends on N only, so a solve gives the same bits alone or inside a batch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace fdg {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kQB = 8;  // basis vectors per register batch

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline void chunk_of(int64_t N, int G, int g, int64_t &beg, int64_t &end) {
  const int64_t chunk = (N + G - 1) / G;
  beg = (int64_t)g * chunk;
  end = beg + chunk < N ? beg + chunk : N;
}

__global__ __launch_bounds__(kBlock) void k_dots(const double *__restrict__ V, int64_t ldv, int nv,
                                                 const double *__restrict__ w, int64_t N, int G,
                                                 double *__restrict__ P) {
  __shared__ double red[kWaves][kQB];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  int64_t beg, end;
  chunk_of(N, G, g, beg, end);
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
      for (int k = 1; k < kWaves; ++k) s += red[k][t];
      P[((int64_t)b * G + g) * nv + q0 + t] = s;
    }
    __syncthreads();
  }
}

// out[b*ostride + q] = f(sum_g P[(b*G + g)*ncomp + q]) for q < ncomp, f = sqrt if do_sqrt;
// with add != NULL also out2[b*o2stride + q] = sum + add[b*astride + q].
__global__ __launch_bounds__(kBlock) void k_reduce(const double *__restrict__ P, int G, int ncomp,
                                                   double *__restrict__ out, int ostride, int do_sqrt,
                                                   const double *__restrict__ add, int astride,
                                                   double *__restrict__ out2, int o2stride) {
  const int64_t b = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = wave; q < ncomp; q += kWaves) {
    double s = 0.0;
    for (int g = lane; g < G; g += 64) s += P[((int64_t)b * G + g) * ncomp + q];
    s = wave_sum(s);
    if (lane == 0) {
      out[b * ostride + q] = do_sqrt ? sqrt(s) : s;
      if (add) out2[b * o2stride + q] = s + add[b * astride + q];
    }
  }
}

// w -= sum_q V_q h_q (h from a device array); optional partial sums of |w|^2.
__global__ __launch_bounds__(kBlock) void k_update(const double *__restrict__ V, int64_t ldv, int nv,
                                                   const double *__restrict__ h, int hstride,
                                                   double *__restrict__ w, int64_t N, int G,
                                                   double *__restrict__ Pnorm) {
  __shared__ double hs[256];
  __shared__ double red[kWaves];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  for (int q = threadIdx.x; q < nv; q += kBlock) hs[q] = h[b * hstride + q];
  __syncthreads();
  int64_t beg, end;
  chunk_of(N, G, g, beg, end);
  double *wb = w + b * N;
  const double *Vb = V + b * N;
  double nrm = 0.0;
  for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
    double wi = wb[i];
    for (int q = 0; q < nv; ++q) wi = fma(-Vb[(int64_t)q * ldv + i], hs[q], wi);
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
      for (int k = 1; k < kWaves; ++k) s += red[k];
      Pnorm[(int64_t)b * G + g] = s;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_scale(const double *__restrict__ w, double *__restrict__ v,
                                                  const double *__restrict__ nrm, int nstride, int64_t N,
                                                  int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= total) return;
  const double d = nrm[(idx / N) * nstride];
  v[idx] = d != 0.0 ? w[idx] / d : 0.0;
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

__global__ __launch_bounds__(kBlock) void k_residual(const double *__restrict__ bv, const double *__restrict__ Ax,
                                                     double *__restrict__ r, int64_t N, int G,
                                                     double *__restrict__ P) {
  __shared__ double red[kWaves];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  int64_t beg, end;
  chunk_of(N, G, g, beg, end);
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
    for (int k = 1; k < kWaves; ++k) s += red[k];
    P[b * G + g] = s;
  }
}

}  // namespace

int reduction_blocks(int64_t N) {
  int64_t g = (N + 2047) / 2048;
  if (g < 1) g = 1;
  if (g > 1024) g = 1024;
  return (int)g;
}

void launch_dots(hipStream_t s, const double *V, int64_t ldv, int nv, const double *w, int64_t N, int64_t nbatch,
                 int G, double *P) {
  hipLaunchKernelGGL(k_dots, dim3(G, (unsigned)nbatch), dim3(kBlock), 0, s, V, ldv, nv, w, N, G, P);
}

void launch_reduce(hipStream_t s, const double *P, int G, int ncomp, int64_t nbatch, double *out, int ostride,
                   bool do_sqrt, const double *add, int astride, double *out2, int o2stride) {
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)nbatch), dim3(kBlock), 0, s, P, G, ncomp, out, ostride,
                     do_sqrt ? 1 : 0, add, astride, out2, o2stride);
}

void launch_update(hipStream_t s, const double *V, int64_t ldv, int nv, const double *h, int hstride, double *w,
                   int64_t N, int64_t nbatch, int G, double *Pnorm) {
  hipLaunchKernelGGL(k_update, dim3(G, (unsigned)nbatch), dim3(kBlock), 0, s, V, ldv, nv, h, hstride, w, N, G,
                     Pnorm);
}

void launch_scale(hipStream_t s, const double *w, double *v, const double *nrm, int nstride, int64_t N,
                  int64_t nbatch) {
  const int64_t total = N * nbatch;
  hipLaunchKernelGGL(k_scale, dim3(cdiv(total, kBlock)), dim3(kBlock), 0, s, w, v, nrm, nstride, N, total);
}

void launch_lincomb(hipStream_t s, double *x, const double *Z, int64_t ldz, int k, const double *y, int ystride,
                    int64_t N, int64_t nbatch) {
  const int64_t total = N * nbatch;
  hipLaunchKernelGGL(k_lincomb, dim3(cdiv(total, kBlock)), dim3(kBlock), 0, s, x, Z, ldz, k, y, ystride, N,
                     total);
}

void launch_residual(hipStream_t s, const double *b, const double *Ax, double *r, int64_t N, int64_t nbatch, int G,
                     double *P) {
  hipLaunchKernelGGL(k_residual, dim3(G, (unsigned)nbatch), dim3(kBlock), 0, s, b, Ax, r, N, G, P);
}

}  // namespace fdg
