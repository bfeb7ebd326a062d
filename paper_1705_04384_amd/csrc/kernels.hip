// Device kernels of the FD-preconditioned flexible GMRES path (gfx950, wave64).
//
//  * FD mode products (eq. 4.7 / 4.9): every mode product of the fast-diagonalization
//    solve is a small dense contraction Y = W x_l X with a zero-padded n x n factor W,
//    run on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//  * The diagonal solve of eq. 4.9 (divide by the sum of univariate eigenvalues), and its
//    block form when some pencils have complex eigenvalue pairs (2 x 2 real blocks in D).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace fdg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;

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

// Solve of sum_l I x D_l x I for block-diagonal D_l (1 x 1 blocks lam, 2 x 2 blocks
// [[a, b], [-b, a]] of a pair a +- ib).  The operator decouples into cells, one block
// per direction (at most 2 x 2 x 2 entries); one thread per cell, consecutive threads
// taking consecutive blocks of direction 1.  In every paired direction the pair (x0, x1)
// goes to the eigen-coordinates ((x0 - i x1) / 2, (x0 + i x1) / 2) of a + ib and a - ib,
// each entry is divided by the complex sum of its eigenvalues (one reciprocal of |sum|^2
// per entry), and the transform is undone (x0 = z+ + z-, x1 = i (z+ - z-)).
struct Cplx {
  double re, im;
};

__device__ inline void pair_fwd(Cplx &z0, Cplx &z1) {  // (z0 - i z1) / 2, (z0 + i z1) / 2
  const Cplx p{0.5 * (z0.re + z1.im), 0.5 * (z0.im - z1.re)};
  const Cplx q{0.5 * (z0.re - z1.im), 0.5 * (z0.im + z1.re)};
  z0 = p;
  z1 = q;
}

__device__ inline void pair_inv(Cplx &z0, Cplx &z1) {  // z0 + z1, i (z0 - z1)
  const Cplx p{z0.re + z1.re, z0.im + z1.im};
  const Cplx q{-(z0.im - z1.im), z0.re - z1.re};
  z0 = p;
  z1 = q;
}

// Block k of one direction: first index, size and (a, b).
__device__ inline int cell_dir(const BlockEig &e, int k, int &sz, double &a, double &b) {
  const int i = e.start[k];
  const bool pr = e.role[i] == 1;
  sz = pr ? 2 : 1;
  a = e.lam[i];
  b = pr ? e.mu[i] : 0.0;
  return i;
}

__global__ __launch_bounds__(kBlock) void k_blockdiv_f64(const double *__restrict__ t, double *__restrict__ y, int d,
                                                         int n, int64_t cells, BlockEig e1, BlockEig e2,
                                                         BlockEig e3) {
  const int64_t id = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (id >= cells) return;
  const int64_t nb12 = (int64_t)e1.nb * e2.nb;
  const int64_t nb123 = d == 3 ? nb12 * e3.nb : nb12;
  const int64_t ent = id / nb123, r = id - ent * nb123;
  const int k1 = (int)(r % e1.nb), k2 = (int)((r / e1.nb) % e2.nb), k3 = d == 3 ? (int)(r / nb12) : 0;
  int sz[3] = {1, 1, 1};
  double a[3] = {0.0, 0.0, 0.0}, b[3] = {0.0, 0.0, 0.0};
  const int i1 = cell_dir(e1, k1, sz[0], a[0], b[0]);
  const int i2 = cell_dir(e2, k2, sz[1], a[1], b[1]);
  const int i3 = d == 3 ? cell_dir(e3, k3, sz[2], a[2], b[2]) : 0;
  const int64_t n2 = (int64_t)n * n;
  const int64_t st[3] = {1, n, n2};
  const int64_t base = ent * (d == 3 ? n2 * n : n2) + i1 + (int64_t)n * i2 + n2 * i3;
  Cplx z[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int t1 = c & 1, t2 = (c >> 1) & 1, t3 = c >> 2;
    const bool in = t1 < sz[0] && t2 < sz[1] && t3 < sz[2];
    z[c] = Cplx{in ? t[base + t1 * st[0] + t2 * st[1] + t3 * st[2]] : 0.0, 0.0};
  }
  // eigen-coordinates in every paired direction (entries c and c + 2^l form a pair)
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (sz[l] != 2) continue;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (!((c >> l) & 1)) pair_fwd(z[c], z[c | (1 << l)]);
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int t1 = c & 1, t2 = (c >> 1) & 1, t3 = c >> 2;
    if (!(t1 < sz[0] && t2 < sz[1] && t3 < sz[2])) continue;
    double lr = 0.0, li = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      lr += a[l];
      li += ((c >> l) & 1) ? -b[l] : b[l];
    }
    const double inv = 1.0 / (lr * lr + li * li);  // z / (lr + i li)
    const Cplx q{(z[c].re * lr + z[c].im * li) * inv, (z[c].im * lr - z[c].re * li) * inv};
    z[c] = q;
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (sz[l] != 2) continue;
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (!((c >> l) & 1)) pair_inv(z[c], z[c | (1 << l)]);
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int t1 = c & 1, t2 = (c >> 1) & 1, t3 = c >> 2;
    if (t1 < sz[0] && t2 < sz[1] && t3 < sz[2]) y[base + t1 * st[0] + t2 * st[1] + t3 * st[2]] = z[c].re;
  }
}

void launch_blockdiv_f64(hipStream_t s, const double *t, double *y, int d, int n, int64_t nbatch,
                         const BlockEig &e1, const BlockEig &e2, const BlockEig &e3) {
  const int64_t cells = (int64_t)e1.nb * e2.nb * (d == 3 ? e3.nb : 1) * nbatch;
  hipLaunchKernelGGL(k_blockdiv_f64, dim3(grid1(cells, kBlock)), dim3(kBlock), 0, s, t, y, d, n, cells, e1, e2, e3);
}

void launch_divide_f64(hipStream_t s, double *t, int d, int n, int64_t nbatch, const double *lam1,
                       const double *lam2, const double *lam3) {
  int64_t N = (int64_t)n * n * (d == 3 ? n : 1);
  const int64_t total = N * nbatch;
  hipLaunchKernelGGL(k_divide_f64, dim3(grid1(total, kBlock)), dim3(kBlock), 0, s, t, d, n, total, lam1,
                     lam2, lam3);
}

}  // namespace fdg
