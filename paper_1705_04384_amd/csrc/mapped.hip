// Matrix-free collocation operator of a mapped 3D domain (Sec. 2.2 with K = I on
// F([0,1]^3)):
//   (A x)_i = -sum_k C_kk d_k^2 u - sum_{k<l} 2 C_kl d_k d_l u - sum_k g_k d_k u   at tau_i,
// u = sum_j x_j B_j.  Every derivative is a Kronecker product of univariate factors
// {M, D, E = -K} (values, first and second derivatives at the collocation points), so it
// is applied by sum factorization:
//   direction 1 (per row):   hm = M1 x,  hd = D1 x,  hk = K1 x
//   direction 2 (per plane): Fmm = M2 hm, Fmk = M2 hk, Fkm = K2 hm, Fdd = D2 hd,
//                            Fmd = M2 hd, Fdm = D2 hm
//   direction 3 (per point): d11 = -M3 Fmk, d22 = -M3 Fkm, d33 = -K3 Fmm, d12 = M3 Fdd,
//                            d13 = D3 Fmd, d23 = D3 Fdm, d1 = M3 Fmd, d2 = M3 Fdm, d3 = D3 Fmm
// and the nine results are combined with the coefficient fields read at the point.
// The workgroup layout is the one of the unit-cube one-pass matvec: 8 waves own a tile
// of 64 columns i1 x T2 rows i2 and a chunk of C3 outputs i3; each wave takes planes j3
// (direction-1 sums through a one-row LDS buffer of its own, direction-2 sums in
// registers) and writes the six plane intermediates to LDS; after one barrier every wave
// forms outputs.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch_addr.h"
#include "mapped.h"

namespace fdg {

namespace {

constexpr int kT2 = 2;  // i2 rows per tile
constexpr int kC3 = 8;  // i3 outputs per workgroup

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <int WMAX, int T2, int C3>
__global__ __launch_bounds__(512) void k_mapped_wpp(CBatch x, MBatch y, int n, int ntx, int nty, int nchunk,
                                                    MappedOp op) {
  constexpr int NWV = 8;
  constexpr int RMAX = T2 + WMAX - 1;
  constexpr int CW = 64 + WMAX;
  constexpr int NPLMAX = C3 + WMAX - 1;
  __shared__ double xrow[NWV][CW];
  __shared__ double cm2[T2][RMAX], cd2[T2][RMAX], ck2[T2][RMAX];
  __shared__ double c3m[C3][WMAX], c3d[C3][WMAX], c3k[C3][WMAX];
  __shared__ int lo3s[C3];
  __shared__ double F[6][NPLMAX][T2][64];  // Fmm, Fmk, Fkm, Fdd, Fmd, Fdm
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nb = (int64_t)gridDim.x;
  int64_t t = blockIdx.x;
  if ((nb & 7) == 0) t = (t & 7) * (nb >> 3) + (t >> 3);  // neighbouring tiles share an XCD
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
  const int w1 = op.w[0], w2 = op.w[1], w3 = op.w[2];
  const bool act1 = i1 < n;
  const int i1c = act1 ? i1 : n - 1;
  const int L0 = op.lo[0][i1a];
  const int off1 = op.lo[0][i1c] - L0;  // in [0, 63]
  const int i2b = i2a + T2 - 1 < n ? i2a + T2 - 1 : n - 1;
  const int R0 = op.lo[1][i2a];
  const int NR = op.lo[1][i2b] + w2 - R0;  // <= RMAX
  const int P0 = op.lo[2][s3];
  const int NPL = op.lo[2][e3 - 1] + w3 - P0;  // <= NPLMAX
  const int ncols = n - L0;
  double m1[WMAX], d1[WMAX], k1[WMAX];
#pragma unroll
  for (int q = 0; q < WMAX; ++q) {
    const size_t o = (size_t)i1c * w1 + q;
    m1[q] = q < w1 ? op.M[0][o] : 0.0;
    d1[q] = q < w1 ? op.D[0][o] : 0.0;
    k1[q] = q < w1 ? op.K[0][o] : 0.0;
  }
  // coefficient tables (global reads before any LDS store)
  double vm = 0.0, vd = 0.0, vk = 0.0, um = 0.0, ud = 0.0, uk = 0.0;
  int vlo = 1 << 30;
  if (threadIdx.x < T2 * RMAX) {
    const int u = threadIdx.x / RMAX, r = threadIdx.x - u * RMAX;
    const int i2 = i2a + u;
    if (i2 <= i2b) {
      const int tt = R0 + r - op.lo[1][i2];
      if (tt >= 0 && tt < w2) {
        const size_t o = (size_t)i2 * w2 + tt;
        vm = op.M[1][o];
        vd = op.D[1][o];
        vk = op.K[1][o];
      }
    }
  }
  if (threadIdx.x < C3 * WMAX) {
    const int q = threadIdx.x / WMAX, tt = threadIdx.x - q * WMAX;
    if (s3 + q < e3 && tt < w3) {
      const size_t o = (size_t)(s3 + q) * w3 + tt;
      um = op.M[2][o];
      ud = op.D[2][o];
      uk = op.K[2][o];
    }
  }
  if (threadIdx.x < C3 && s3 + (int)threadIdx.x < e3) vlo = op.lo[2][s3 + threadIdx.x];
  if (threadIdx.x < T2 * RMAX) {
    const int u = threadIdx.x / RMAX, r = threadIdx.x - u * RMAX;
    cm2[u][r] = vm;
    cd2[u][r] = vd;
    ck2[u][r] = vk;
  }
  if (threadIdx.x < C3 * WMAX) {
    const int q = threadIdx.x / WMAX, tt = threadIdx.x - q * WMAX;
    c3m[q][tt] = um;
    c3d[q][tt] = ud;
    c3k[q][tt] = uk;
  }
  if (threadIdx.x < C3) lo3s[threadIdx.x] = vlo;
  __syncthreads();
  for (int pl = wave; pl < NPL; pl += NWV) {
    gptr<const double> xp = xb + (int64_t)(P0 + pl) * n2 + (int64_t)R0 * n + L0;
    double xr[RMAX], xh[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      xr[r] = (r < NR && lane < ncols) ? xp[(int64_t)r * n + lane] : 0.0;
      xh[r] = (r < NR && lane < WMAX && 64 + lane < ncols) ? xp[(int64_t)r * n + 64 + lane] : 0.0;
    }
    double hm[RMAX], hd[RMAX], hk[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      xrow[wave][lane] = xr[r];
      if (lane < WMAX) xrow[wave][64 + lane] = xh[r];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double sm = 0.0, sd = 0.0, sk = 0.0;
#pragma unroll
      for (int q = 0; q < WMAX; ++q)
        if (q < w1) {
          const double v = xrow[wave][off1 + q];
          sm = fma(m1[q], v, sm);
          sd = fma(d1[q], v, sd);
          sk = fma(k1[q], v, sk);
        }
      hm[r] = sm;
      hd[r] = sd;
      hk[r] = sk;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
#pragma unroll
    for (int u = 0; u < T2; ++u) {
      double fmm = 0.0, fmk = 0.0, fkm = 0.0, fdd = 0.0, fmd = 0.0, fdm = 0.0;
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const double cm = cm2[u][r], cd = cd2[u][r], ck = ck2[u][r];
        fmm = fma(cm, hm[r], fmm);
        fmk = fma(cm, hk[r], fmk);
        fkm = fma(ck, hm[r], fkm);
        fdd = fma(cd, hd[r], fdd);
        fmd = fma(cm, hd[r], fmd);
        fdm = fma(cd, hm[r], fdm);
      }
      F[0][pl][u][lane] = fmm;
      F[1][pl][u][lane] = fmk;
      F[2][pl][u][lane] = fkm;
      F[3][pl][u][lane] = fdd;
      F[4][pl][u][lane] = fmd;
      F[5][pl][u][lane] = fdm;
    }
  }
  __syncthreads();
  if (!act1) return;
  const int64_t N = op.N;
  for (int idx = wave; idx < C3 * T2; idx += NWV) {
    const int q = idx / T2, u = idx - q * T2;
    const int i2 = i2a + u;
    if (s3 + q >= e3 || i2 > i2b) continue;
    const int b3 = lo3s[q] - P0;
    double mk = 0.0, km = 0.0, kmm = 0.0, mdd = 0.0, dmd = 0.0, ddm = 0.0, mmd = 0.0, mdm = 0.0, dmm = 0.0;
#pragma unroll
    for (int tt = 0; tt < WMAX; ++tt)
      if (tt < w3) {
        const double cm = c3m[q][tt], cd = c3d[q][tt], ck = c3k[q][tt];
        const int pl = b3 + tt;
        const double fmm = F[0][pl][u][lane], fmk = F[1][pl][u][lane], fkm = F[2][pl][u][lane];
        const double fdd = F[3][pl][u][lane], fmd = F[4][pl][u][lane], fdm = F[5][pl][u][lane];
        mk = fma(cm, fmk, mk);
        km = fma(cm, fkm, km);
        kmm = fma(ck, fmm, kmm);
        mdd = fma(cm, fdd, mdd);
        dmd = fma(cd, fmd, dmd);
        ddm = fma(cd, fdm, ddm);
        mmd = fma(cm, fmd, mmd);
        mdm = fma(cm, fdm, mdm);
        dmm = fma(cd, fmm, dmm);
      }
    const int64_t o = (int64_t)(s3 + q) * n2 + (int64_t)i2 * n + i1;
    const double *cf = op.coef + o;
    // -sum C d2 u - sum g d u with d11 = -mk, d22 = -km, d33 = -kmm
    double v = cf[0] * mk;
    v = fma(cf[N], km, v);
    v = fma(cf[2 * N], kmm, v);
    v = fma(-cf[3 * N], mdd, v);
    v = fma(-cf[4 * N], dmd, v);
    v = fma(-cf[5 * N], ddm, v);
    v = fma(-cf[6 * N], mmd, v);
    v = fma(-cf[7 * N], mdm, v);
    v = fma(-cf[8 * N], dmm, v);
    yb[o] = v;
  }
}

}  // namespace

bool mapped_matvec_ok(int n, int64_t nbatch, const MappedOp &op) {
  int w = 0;
  for (int l = 0; l < 3; ++l) w = op.w[l] > w ? op.w[l] : w;
  return w <= 8 && op.step[0] <= 1 && op.step[1] <= 1 &&
         (int64_t)cdiv(n, 64) * cdiv(n, kT2) * cdiv(n, kC3) * nbatch < ((int64_t)1 << 31);
}

bool launch_mapped_matvec_f64(hipStream_t s, CBatch x, MBatch y, int n, int64_t nbatch, const MappedOp &op) {
  if (!mapped_matvec_ok(n, nbatch, op)) return false;
  int w = 0;
  for (int l = 0; l < 3; ++l) w = op.w[l] > w ? op.w[l] : w;
  const int ntx = (int)cdiv(n, 64), nty = (int)cdiv(n, kT2), nchunk = (int)cdiv(n, kC3);
  const dim3 grid((unsigned)((int64_t)ntx * nty * nchunk * nbatch));
  if (w <= 4)
    hipLaunchKernelGGL((k_mapped_wpp<4, kT2, kC3>), grid, dim3(512), 0, s, x, y, n, ntx, nty, nchunk, op);
  else if (w <= 6)
    hipLaunchKernelGGL((k_mapped_wpp<6, kT2, kC3>), grid, dim3(512), 0, s, x, y, n, ntx, nty, nchunk, op);
  else
    hipLaunchKernelGGL((k_mapped_wpp<8, kT2, kC3>), grid, dim3(512), 0, s, x, y, n, ntx, nty, nchunk, op);
  return true;
}

}  // namespace fdg
