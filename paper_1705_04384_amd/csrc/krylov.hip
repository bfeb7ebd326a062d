// Krylov vector kernels of flexible GMRES: multi-dot products, classical Gram-Schmidt
// with reorthogonalisation, norms, scaling and the linear combination x += Z y.
//
// Reductions are deterministic.  A producer kernel has G <= 256 blocks (G depends on N
// only); block g sums the contiguous chunk [g*chunk, min(N, (g+1)*chunk)) in a fixed
// order (strided accumulation per thread, an xor butterfly inside each wave, then the
// waves in index order) and stores one partial sum per component.  The consumer kernel
// reduces the G partials itself, again in a fixed order (lane t takes g = t, t + 64, ...,
// then an xor butterfly, which leaves the same bits in every lane), so every block of
// the consumer holds identical values; block 0 publishes them to device memory and to
// host-mapped memory for the host's least-squares update.  Kernel boundaries order the
// two steps; no device-wide fences or atomics are used.  A problem gives the same bits
// alone or inside a batch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "batch_addr.h"
#include "kernels.h"
#include "reduce.h"

namespace fdg {

namespace {

typedef double dbl2 __attribute__((ext_vector_type(2)));

constexpr int kBlock = 256;  // threads of the streaming kernels
#ifndef FDG_DOTS_UNROLL
#define FDG_DOTS_UNROLL 2
#endif
#ifndef FDG_UPD_UNROLL
#define FDG_UPD_UNROLL 2
#endif
constexpr int kQB = 8;       // basis vectors per register batch

__device__ inline dbl2 ld2(gptr<const double> p) { return *(gptr<const dbl2>)p; }
__device__ inline void st2(gptr<double> p, dbl2 v) { *(gptr<dbl2>)p = v; }

// hs[q] = sum of the partials of component q, q < ncomp (all waves of the block help).
__device__ inline void reduce_into(gptr<const double> P, int G, int ldp, int ncomp, double *hs, int nwaves) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q = wave; q < ncomp; q += nwaves) {
    const double s = sum_partials(P, G, ldp, q);
    if (lane == 0) hs[q] = s;
  }
  __syncthreads();
}

// Per-block partial sums of kQB components (acc[t] per thread) -> P[g*ncomp + q0 + t].
__device__ inline void store_partials(double (&acc)[kQB], double (*red)[kQB], gptr<double> Pg, int q0, int nv) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t < kQB; ++t)
    if (q0 + t < nv) {  // valid components only (block-uniform)
      const double v = wave_sum(acc[t]);
      if (lane == 0) red[wave][t] = v;
    }
  __syncthreads();
  if (threadIdx.x < kQB && q0 + (int)threadIdx.x < nv) {
    const int t = threadIdx.x;
    double s = red[0][t];
    for (int k = 1; k < kRedWaves; ++k) s += red[k][t];
    Pg[q0 + t] = s;
  }
  __syncthreads();
}

// acc[t] = V_{q0+t} . w over the block's chunk, thread tid of nthr taking a strided share.
template <bool VEC>
__device__ inline void chunk_dots(gptr<const double> Vb, int64_t ldv, int nv, int q0, gptr<const double> wb, int64_t beg,
                                  int64_t end, double (&acc)[kQB], int tid = threadIdx.x, int nthr = kRed) {
#pragma unroll
  for (int t = 0; t < kQB; ++t) acc[t] = 0.0;
  if (VEC) {
#pragma unroll FDG_DOTS_UNROLL
    for (int64_t i = beg + 2 * tid; i < end; i += 2 * nthr) {
      const dbl2 wi = *(gptr<const dbl2>)(wb + i);
#pragma unroll
      for (int t = 0; t < kQB; ++t)
        if (q0 + t < nv) {
          const dbl2 vi = *(gptr<const dbl2>)(Vb + (int64_t)(q0 + t) * ldv + i);
          acc[t] = fma(vi.x, wi.x, acc[t]);
          acc[t] = fma(vi.y, wi.y, acc[t]);
        }
    }
  } else {
    for (int64_t i = beg + tid; i < end; i += nthr) {
      const double wi = wb[i];
#pragma unroll
      for (int t = 0; t < kQB; ++t)
        if (q0 + t < nv) acc[t] = fma(Vb[(int64_t)(q0 + t) * ldv + i], wi, acc[t]);
    }
  }
}

// acc[t] += V_{q0+t} . w for t < NQ over the thread's 2-wide elements, in the order of
// chunk_dots<true>, with no load under a branch (a load the compiler has to predicate is
// waited for where its branch rejoins, which serialises the loads of a thread): each round
// issues the loads of U elements of w and of every V_q at addresses clamped into
// [beg, end), then masks the sums of the elements beyond end.
template <int NQ, int U>
__device__ inline void dots_batch(gptr<const double> Vb, int64_t ldv, int q0, gptr<const double> wb, int64_t beg,
                                  int64_t end, double (&acc)[kQB], int tid, int nthr) {
  const int64_t step = 2 * (int64_t)nthr;
  for (int64_t i = beg + 2 * (int64_t)tid; i < end; i += U * step) {
    dbl2 wv[U], vv[U][NQ];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = i + u * step;
      ok[u] = e < end;
      const int64_t ec = ok[u] ? e : end - 2;
      wv[u] = ld2(wb + ec);
#pragma unroll
      for (int t = 0; t < NQ; ++t) vv[u][t] = ld2(Vb + (int64_t)(q0 + t) * ldv + ec);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < NQ; ++t) {
        const double a = fma(vv[u][t].y, wv[u].y, fma(vv[u][t].x, wv[u].x, acc[t]));
        acc[t] = ok[u] ? a : acc[t];
      }
  }
}

// acc[t] = V_{q0+t} . w for t < min(kQB, nv - q0) (2-wide elements; zero beyond).
__device__ inline void dots_any(gptr<const double> Vb, int64_t ldv, int nv, int q0, gptr<const double> wb,
                                int64_t beg, int64_t end, double (&acc)[kQB], int tid, int nthr) {
#pragma unroll
  for (int t = 0; t < kQB; ++t) acc[t] = 0.0;
  const int nq = nv - q0 < kQB ? nv - q0 : kQB;
  switch (nq) {
    case 1: dots_batch<1, 4>(Vb, ldv, q0, wb, beg, end, acc, tid, nthr); break;
    case 2: dots_batch<2, 4>(Vb, ldv, q0, wb, beg, end, acc, tid, nthr); break;
    case 3: dots_batch<3, 2>(Vb, ldv, q0, wb, beg, end, acc, tid, nthr); break;
    case 4: dots_batch<4, 2>(Vb, ldv, q0, wb, beg, end, acc, tid, nthr); break;
    case 5: dots_batch<5, 1>(Vb, ldv, q0, wb, beg, end, acc, tid, nthr); break;
    case 6: dots_batch<6, 1>(Vb, ldv, q0, wb, beg, end, acc, tid, nthr); break;
    case 7: dots_batch<7, 1>(Vb, ldv, q0, wb, beg, end, acc, tid, nthr); break;
    default: dots_batch<8, 1>(Vb, ldv, q0, wb, beg, end, acc, tid, nthr); break;
  }
}

// w -= sum_q V_q hs[q] over the block's chunk; returns the thread's part of |w|^2.
template <bool VEC>
__device__ inline double chunk_update(gptr<const double> Vb, int64_t ldv, int nv, const double *hs, gptr<double> wb,
                                      int64_t beg, int64_t end) {
  double nrm = 0.0;
  if (VEC) {
#pragma unroll FDG_UPD_UNROLL
    for (int64_t i = beg + 2 * threadIdx.x; i < end; i += 2 * kRed) {
      dbl2 wi = *(gptr<const dbl2>)(wb + i);
      for (int q = 0; q < nv; ++q) {
        const dbl2 vi = *(gptr<const dbl2>)(Vb + (int64_t)q * ldv + i);
        wi.x = fma(-vi.x, hs[q], wi.x);
        wi.y = fma(-vi.y, hs[q], wi.y);
      }
      *(gptr<dbl2>)(wb + i) = wi;
      nrm = fma(wi.x, wi.x, nrm);
      nrm = fma(wi.y, wi.y, nrm);
    }
  } else {
    for (int64_t i = beg + threadIdx.x; i < end; i += kRed) {
      double wi = wb[i];
      for (int q = 0; q < nv; ++q) wi = fma(-Vb[(int64_t)q * ldv + i], hs[q], wi);
      wb[i] = wi;
      nrm = fma(wi, wi, nrm);
    }
  }
  return nrm;
}

__device__ inline double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    s = red[0];
    for (int k = 1; k < kRedWaves; ++k) s += red[k];
  }
  __syncthreads();
  return s;
}

// The update w -= V hs followed by the dots V^T w of the updated w over the block's
// chunk, reading each basis value from memory once when nv <= kGroupNV (the two-step form
// reads the basis twice, and the second read misses the cache at large N).  The summation
// order of the dots depends on nv only.
//
// nv <= kRegNV: thread-strided elements, all nv basis values of an element in registers,
// per-thread running dots, then butterflies and the waves in index order (store_partials);
// the updated w is bitwise that of chunk_update (the same fma order per element).
// kRegNV < nv <= kGroupNV: 2 (nv <= 16) or 4 lanes per element, 8 basis vectors per lane
// (group_update_dots): every thread of the block loads.  Measured on MI355X at N = 96^3
// (deformed cube, FGMRES(30), 35 calls per solve): 968 -> 739 us per solve against the
// previous form, which staged sub-chunks of the basis in LDS with only the threads of a
// sub-chunk loading (at nv = 30: 55.3 -> 37.6 us per call, 4.1 -> 6.0 TB/s).
// Larger nv: the update and the dots each stream the basis.
#ifndef FDG_REG_NV
#define FDG_REG_NV 8  // 10 measures the same; 12 and more spill registers
#endif
constexpr int kRegNV = FDG_REG_NV;
#ifndef FDG_REG2_UNROLL
#define FDG_REG2_UNROLL 4
#endif
constexpr int kGroupNV = 4 * kQB;

struct PassLds {
  double red[kRedWaves][kQB];
};

template <int NVM, int UNR>
__device__ inline void reg_update_dots(gptr<const double> __restrict__ Vb, int64_t ldv, int nv, const double *hs,
                                       gptr<double> __restrict__ wb, int64_t beg, int64_t end, gptr<double> Pg,
                                       PassLds &L) {
  double acc[NVM];
#pragma unroll
  for (int t = 0; t < NVM; ++t) acc[t] = 0.0;
#pragma unroll UNR
  for (int64_t i = beg + threadIdx.x; i < end; i += kRed) {
    gptr<const double> vcol = Vb + i;
    double v[NVM];
#pragma unroll
    for (int t = 0; t < NVM; ++t) v[t] = t < nv ? vcol[(int64_t)t * ldv] : 0.0;
    double wi = wb[i];
#pragma unroll
    for (int t = 0; t < NVM; ++t)
      if (t < nv) wi = fma(-v[t], hs[t], wi);
    wb[i] = wi;
#pragma unroll
    for (int t = 0; t < NVM; ++t) acc[t] = fma(v[t], wi, acc[t]);
  }
#pragma unroll
  for (int q0 = 0; q0 < NVM; q0 += kQB) {
    if (q0 >= nv) break;
    double part[kQB];
#pragma unroll
    for (int t = 0; t < kQB; ++t) part[t] = q0 + t < NVM ? acc[q0 + t] : 0.0;
    store_partials(part, L.red, Pg, q0, nv);
  }
}

// Lane exchange inside a quad of lanes (quad_perm DPP, both halves of a double).
template <int CTRL>
__device__ inline double quad_dpp(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]

// nv <= LPE QPL: LPE lanes per element (1, 2 or 4 adjacent lanes; 2-wide elements with
// VEC), lane k of the group holding basis vectors q = k QPL + t, t < QPL.  Each lane loads
// its basis values of the element (every load issued, at clamped vector and element
// indices), the group adds its partial sums of V_q h_q by xor exchanges inside the quad
// (commutative adds: the same bits in every lane of the group), and every lane forms
// w' = w - that sum and its dots.  The dots are summed over the lanes that hold the same
// q by an xor butterfly, then over the waves in index order.
template <bool VEC, int LPE, int QPL>
__device__ inline void group_update_dots(gptr<const double> __restrict__ Vb, int64_t ldv, int nv, const double *hs,
                                         gptr<double> __restrict__ wb, int64_t beg, int64_t end, gptr<double> Pg,
                                         double (*red)[4 * kQB]) {
  static_assert(LPE == 1 || LPE == 2 || LPE == 4, "lanes per element");
  static_assert(LPE * QPL <= 4 * kQB, "partials buffer");
  constexpr int EL = VEC ? 2 : 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, k = lane & (LPE - 1);
  const int64_t step = (int64_t)EL * (kRed / LPE);
  double hq[QPL];
  gptr<const double> vq[QPL];
#pragma unroll
  for (int t = 0; t < QPL; ++t) {
    const int q = k * QPL + t;
    hq[t] = q < nv ? hs[q] : 0.0;  // vectors beyond nv: clamped loads, zero weight, dots unused
    vq[t] = Vb + (int64_t)(q < nv ? q : nv - 1) * ldv;
  }
  double acc[QPL];
#pragma unroll
  for (int t = 0; t < QPL; ++t) acc[t] = 0.0;
  for (int64_t i = beg + EL * (int64_t)(tid / LPE); i < end; i += step) {
    double v[QPL][EL], w[EL];
    const int64_t ec = i;
    if constexpr (VEC) {
      const dbl2 ww = ld2(wb + ec);
      w[0] = ww.x;
      w[1] = ww.y;
#pragma unroll
      for (int t = 0; t < QPL; ++t) {
        const dbl2 vv = ld2(vq[t] + ec);
        v[t][0] = vv.x;
        v[t][1] = vv.y;
      }
    } else {
      w[0] = wb[ec];
#pragma unroll
      for (int t = 0; t < QPL; ++t) v[t][0] = vq[t][ec];
    }
    double wn[EL];
#pragma unroll
    for (int el = 0; el < EL; ++el) {
      double part = 0.0;
#pragma unroll
      for (int t = 0; t < QPL; ++t) part = fma(v[t][el], hq[t], part);
      if constexpr (LPE >= 2) part += quad_dpp<kQuadXor1>(part);
      if constexpr (LPE >= 4) part += quad_dpp<kQuadXor2>(part);
      wn[el] = w[el] - part;
    }
    if (k == 0) {
      if constexpr (VEC) {
        dbl2 o;
        o.x = wn[0];
        o.y = wn[1];
        st2(wb + ec, o);
      } else {
        wb[ec] = wn[0];
      }
    }
#pragma unroll
    for (int el = 0; el < EL; ++el)
#pragma unroll
      for (int t = 0; t < QPL; ++t) acc[t] = fma(v[t][el], wn[el], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < QPL; ++t) {
    double a = acc[t];
#pragma unroll
    for (int off = LPE; off < 64; off <<= 1) a += __shfl_xor(a, off, 64);
    if (lane < LPE) red[wave][lane * QPL + t] = a;
  }
  __syncthreads();
  if (tid < nv) {
    double sum = red[0][tid];
    for (int wv = 1; wv < kRedWaves; ++wv) sum += red[wv][tid];
    Pg[tid] = sum;
  }
}

// P = partial dots V^T w.  The nb = ceil(nv / kQB) batches of kQB components are spread
// over ng = 1, 2 or 4 groups of waves that stream the chunk side by side (one batch per
// group per round), so the basis is read in ceil(nb / ng) passes instead of nb.  Group
// gg sums its batch thread-strided, by butterflies, then its waves in index order; ng
// depends on nv only (ng = 1 is the whole block, one batch after another).
#ifndef FDG_DOTS_GROUPS
#define FDG_DOTS_GROUPS 4
#endif
template <bool VEC>
__global__ __launch_bounds__(kRed) void k_dots(CBatch V, int64_t ldv, IBatch nvs, CBatch w, int64_t N, int G,
                                               int ldp, MBatch P) {
  __shared__ double red[kRedWaves][kQB];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int nv = nvs.at(b);
  int64_t beg, end;
  chunk_of(N, G, g, beg, end);
  gptr<const double> __restrict__ wb = w.gat(b);
  gptr<const double> __restrict__ Vb = V.gat(b);
  gptr<double> Pg = P.gat(b) + (int64_t)g * ldp;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nb = (nv + kQB - 1) / kQB;
  const int ng = nb >= 4 && FDG_DOTS_GROUPS >= 4 ? 4 : (nb >= 2 && FDG_DOTS_GROUPS >= 2 ? 2 : 1);
  const int gw = kRedWaves / ng, grp = wave / gw;
  const int gtid = (int)threadIdx.x - grp * gw * 64;
  const int rounds = (nb + ng - 1) / ng;
  for (int rd = 0; rd < rounds; ++rd) {
    const int bq = rd * ng + grp;  // this group's batch (none when bq >= nb)
    double acc[kQB];
    if (bq < nb) {
      if (VEC)  // measured on MI355X: 10.7 -> 9.6 us per call at N = 128^3
        dots_any(Vb, ldv, nv, bq * kQB, wb, beg, end, acc, gtid, gw * 64);
      else
        chunk_dots<VEC>(Vb, ldv, nv, bq * kQB, wb, beg, end, acc, gtid, gw * 64);
    } else {
#pragma unroll
      for (int t = 0; t < kQB; ++t) acc[t] = 0.0;
    }
    // butterflies for this wave's valid components only (a wave-uniform count): with one
    // or two basis vectors the other six or seven would be most of the kernel's LDS work
    const int nval = bq < nb ? (nv - bq * kQB < kQB ? nv - bq * kQB : kQB) : 0;
#pragma unroll
    for (int t = 0; t < kQB; ++t)
      if (t < nval) {
        const double v = wave_sum(acc[t]);
        if (lane == 0) red[wave][t] = v;
      }
    __syncthreads();
    if ((int)threadIdx.x < ng * kQB) {
      const int gg = threadIdx.x / kQB, t = threadIdx.x - gg * kQB;
      const int q = (rd * ng + gg) * kQB + t;
      if (q < nv) {
        double sum = red[gg * gw][t];
        for (int k = 1; k < gw; ++k) sum += red[gg * gw + k][t];
        Pg[q] = sum;
      }
    }
    __syncthreads();
  }
}

// h1 = reduce(Pin); w -= V h1; Pout = partial dots V^T w.  Block 0 stores h1 to hout.
template <bool VEC>
__global__ __launch_bounds__(kRed) void k_update_dots(CBatch V, int64_t ldv, IBatch nvs, CBatch Pin, int G,
                                                      int ldp, MBatch w, int64_t N, MBatch Pout, MBatch hout) {
  __shared__ double hs[256];
  __shared__ PassLds L;
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int nv = nvs.at(b);
  reduce_into(Pin.gat(b), G, ldp, nv, hs, kRedWaves);
  if (g == 0) {
    gptr<double> ho = hout.gat(b);
    for (int q = threadIdx.x; q < nv; q += kRed) ho[q] = hs[q];
  }
  int64_t beg, end;
  chunk_of(N, G, g, beg, end);
  gptr<const double> __restrict__ Vb = V.gat(b);
  gptr<double> __restrict__ wb = w.gat(b);
  gptr<double> Pg = Pout.gat(b) + (int64_t)g * ldp;
  if (nv <= 2) {
    reg_update_dots<2, FDG_REG2_UNROLL>(Vb, ldv, nv, hs, wb, beg, end, Pg, L);
    return;
  }
  if (nv <= kRegNV) {
    reg_update_dots<kRegNV, 1>(Vb, ldv, nv, hs, wb, beg, end, Pg, L);
    return;
  }
  if (nv <= kGroupNV) {
    __shared__ double qred[kRedWaves][4 * kQB];
    if (nv <= 16)
      group_update_dots<VEC, 2, kQB>(Vb, ldv, nv, hs, wb, beg, end, Pg, qred);
    else
      group_update_dots<VEC, 4, kQB>(Vb, ldv, nv, hs, wb, beg, end, Pg, qred);
    return;
  }
  (void)chunk_update<VEC>(Vb, ldv, nv, hs, wb, beg, end);
  __syncthreads();  // the block's own chunk of w is complete before it is re-read
  for (int q0 = 0; q0 < nv; q0 += kQB) {
    double acc[kQB];
    chunk_dots<VEC>(Vb, ldv, nv, q0, wb, beg, end, acc);
    store_partials(acc, L.red, Pg, q0, nv);
  }
}

// h2 = reduce(Pin); w -= V h2; Pnorm = partial |w|^2.  Block 0 stores the Hessenberg
// column Hcol[q] = h1[q] + h2[q] (device and, when given, host-mapped memory).
template <bool VEC>
__global__ __launch_bounds__(kRed) void k_update_norm(CBatch V, int64_t ldv, IBatch nvs, CBatch Pin, int G,
                                                      int ldp, MBatch w, int64_t N, MBatch Pnorm, CBatch h1,
                                                      MBatch Hcol, MBatch host, MBatch Pdev) {
  __shared__ double hs[256];
  __shared__ double red[kRedWaves];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  const int nv = nvs.at(b);
  reduce_into(Pin.gat(b), G, ldp, nv, hs, kRedWaves);
  if (g == 0) {
    gptr<const double> h1b = h1.gat(b);
    gptr<double> hc = Hcol.gat(b);
    gptr<double> hh = host.valid() ? host.gat(b) : nullptr;
    for (int q = threadIdx.x; q < nv; q += kRed) {
      const double v = h1b[q] + hs[q];
      hc[q] = v;
      if (hh) hh[q] = v;
    }
  }
  int64_t beg, end;
  chunk_of(N, G, g, beg, end);
  const double nrm = chunk_update<VEC>(V.gat(b), ldv, nv, hs, w.gat(b), beg, end);
  const double s = block_sum(nrm, red);
  if (threadIdx.x == 0) {
    Pnorm.gat(b)[g] = s;
    if (Pdev.valid()) Pdev.gat(b)[g] = s;
  }
}

// d = sqrt(reduce(Pn)); v = w / d (0 if d = 0).  Block 0 stores d to out and host.
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_scale_reduce(CBatch w, MBatch v, CBatch Pn, int G, int64_t N, MBatch out,
                                                         MBatch host) {
  __shared__ double hs[1];
  const int64_t b = blockIdx.y;
  reduce_into(Pn.gat(b), G, 1, 1, hs, kBlock / 64);
  const double d = sqrt(hs[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (out.valid()) out.gat(b)[0] = d;
    if (host.valid()) host.gat(b)[0] = d;
  }
  gptr<const double> wb = w.gat(b);
  gptr<double> vb = v.gat(b);
  if (VEC) {  // 4 pairs per thread per step, all loads issued before the stores
    const int64_t step = (int64_t)gridDim.x * kBlock * 8;  // elements per step of the grid
    for (int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 2; base < N; base += step) {
      dbl2 xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * kBlock * 2 * gridDim.x;
        xv[u] = i < N ? *(gptr<const dbl2>)(wb + i) : dbl2{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * kBlock * 2 * gridDim.x;
        if (i < N)
          *(gptr<dbl2>)(vb + i) = d != 0.0 ? dbl2{xv[u].x / d, xv[u].y / d} : dbl2{0.0, 0.0};
      }
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock)
      vb[i] = d != 0.0 ? wb[i] / d : 0.0;
  }
}

// v = w / d with d given per entry (table) or shared (value); 0 where d = 0.
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_scale_by(CBatch w, MBatch v, const double *__restrict__ dtab, double dval,
                                                     int64_t N) {
  const int64_t b = blockIdx.y;
  const double d = dtab ? dtab[b] : dval;
  gptr<const double> wb = w.gat(b);
  gptr<double> vb = v.gat(b);
  if (VEC) {
    const int64_t step = (int64_t)gridDim.x * kBlock * 8;
    for (int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 2; base < N; base += step) {
      dbl2 xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * kBlock * 2 * gridDim.x;
        xv[u] = i < N ? *(gptr<const dbl2>)(wb + i) : dbl2{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = base + (int64_t)u * kBlock * 2 * gridDim.x;
        if (i < N)
          *(gptr<dbl2>)(vb + i) = d != 0.0 ? dbl2{xv[u].x / d, xv[u].y / d} : dbl2{0.0, 0.0};
      }
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += (int64_t)gridDim.x * kBlock)
      vb[i] = d != 0.0 ? wb[i] / d : 0.0;
  }
}

// d = sqrt(reduce(Pn)) stored to out and host (one block per batch entry).
__global__ __launch_bounds__(kBlock) void k_norm_reduce(CBatch Pn, int G, MBatch out, MBatch host) {
  __shared__ double hs[1];
  const int64_t b = blockIdx.x;
  reduce_into(Pn.gat(b), G, 1, 1, hs, kBlock / 64);
  if (threadIdx.x == 0) {
    const double d = sqrt(hs[0]);
    if (out.valid()) out.gat(b)[0] = d;
    if (host.valid()) host.gat(b)[0] = d;
  }
}

// acc[u] += sum_{t < NQ} Z_{q0+t} y_{q0+t} over U 2-wide elements (Z_q clamped to q < k,
// terms with q >= k skipped), in the order q = q0, q0 + 1, ...
template <int NQ, int U>
__device__ inline void lincomb_batch(gptr<const double> Zb, int64_t ldz, int q0, int k, const double *yv,
                                     const int64_t (&ec)[U], dbl2 (&acc)[U]) {
  dbl2 z[U][NQ];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int t = 0; t < NQ; ++t) z[u][t] = ld2(Zb + (int64_t)(q0 + t < k ? q0 + t : k - 1) * ldz + ec[u]);
#pragma unroll
  for (int t = 0; t < NQ; ++t) {
    if (q0 + t >= k) break;
    const double yq = yv[q0 + t];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u].x = fma(z[u][t].x, yq, acc[u].x);
      acc[u].y = fma(z[u][t].y, yq, acc[u].y);
    }
  }
}

// x = (overwrite ? 0 : x) + sum_q Z_q y_q, q < k; y from a device table (256 per entry)
// or, without a table, the by-value coefficients shared by every entry.  VEC: 2-wide
// elements, U = 4 per thread per round, the Z_q loaded kQB at a time with every load of a
// batch issued together (measured on MI355X: 8.5 -> 7.7 us per call for k = 1 at
// N = 128^3).
template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_lincomb(MBatch x, CBatch Z, int64_t ldz, IBatch ks, Coeffs y,
                                                    const double *__restrict__ ytab, int64_t N, IBatch overwrite) {
  const int64_t b = blockIdx.y;
  gptr<double> __restrict__ xb = x.gat(b);
  gptr<const double> __restrict__ Zb = Z.gat(b);
  const int k = ks.at(b);
  const bool ow = overwrite.at(b) != 0;
  gptr<const double> yt = ytab ? (gptr<const double>)ytab + b * 256 : nullptr;
  if (VEC) {
    __shared__ double ys[256];
    for (int q = threadIdx.x; q < k; q += kBlock) ys[q] = yt ? yt[q] : y.v[q];
    __syncthreads();
    constexpr int U = 4;
    const int64_t gstep = (int64_t)gridDim.x * kBlock * 2;
    for (int64_t base = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * 2; base < N; base += U * gstep) {
      int64_t ec[U];
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i = base + u * gstep;
        ok[u] = i < N;
        ec[u] = ok[u] ? i : N - 2;
      }
      dbl2 acc[U];
      if (ow) {
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = dbl2{0.0, 0.0};
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = ld2(xb + ec[u]);
      }
      for (int q0 = 0; q0 < k; q0 += kQB) {
        const int nq = k - q0;
        if (nq == 1)
          lincomb_batch<1, U>(Zb, ldz, q0, k, ys, ec, acc);
        else if (nq == 2)
          lincomb_batch<2, U>(Zb, ldz, q0, k, ys, ec, acc);
        else if (nq <= 4)
          lincomb_batch<4, U>(Zb, ldz, q0, k, ys, ec, acc);
        else
          lincomb_batch<kQB, U>(Zb, ldz, q0, k, ys, ec, acc);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (ok[u]) st2(xb + ec[u], acc[u]);
    }
    return;
  }
  // 4 elements per thread per step
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock + threadIdx.x; i0 < N; i0 += 4 * stride) {
    double acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + u * stride;
      acc[u] = (ow || i >= N) ? 0.0 : xb[i];
    }
    for (int q = 0; q < k; ++q) {
      const double yq = yt ? yt[q] : y.v[q];
      gptr<const double> zq = Zb + (int64_t)q * ldz;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t i = i0 + u * stride;
        if (i < N) acc[u] = fma(zq[i], yq, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t i = i0 + u * stride;
      if (i < N) xb[i] = acc[u];
    }
  }
}

template <bool VEC>
__global__ __launch_bounds__(kRed) void k_residual(CBatch bv, CBatch Ax, MBatch r, int64_t N, int G, MBatch P) {
  __shared__ double red[kRedWaves];
  const int g = blockIdx.x;
  const int64_t b = blockIdx.y;
  int64_t beg, end;
  chunk_of(N, G, g, beg, end);
  gptr<const double> bb = bv.gat(b), ab = Ax.gat(b);
  gptr<double> rb = r.gat(b);
  double nrm = 0.0;
  if (VEC) {
#pragma unroll 4
    for (int64_t i = beg + 2 * threadIdx.x; i < end; i += 2 * kRed) {
      const dbl2 x = *(gptr<const dbl2>)(bb + i);
      const dbl2 a = *(gptr<const dbl2>)(ab + i);
      const dbl2 v = {x.x - a.x, x.y - a.y};
      *(gptr<dbl2>)(rb + i) = v;
      nrm = fma(v.x, v.x, nrm);
      nrm = fma(v.y, v.y, nrm);
    }
  } else {
#pragma unroll 4
    for (int64_t i = beg + threadIdx.x; i < end; i += kRed) {
      const double v = bb[i] - ab[i];
      rb[i] = v;
      nrm = fma(v, v, nrm);
    }
  }
  const double s = block_sum(nrm, red);
  if (threadIdx.x == 0) P.gat(b)[g] = s;
}

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

unsigned stream_blocks(int64_t N, int per_thread) {
  int64_t g = (N + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
  if (g > 4096) g = 4096;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

#ifndef FDG_RED_ELEMS
#define FDG_RED_ELEMS 1024
#endif
int reduction_blocks(int64_t N) {
  // one 1024-thread workgroup per FDG_RED_ELEMS elements, up to 256 (the device has 256
  // compute units).  Measured: 1024 (or 512) elements beat 2048 by 5% on the FGMRES solve
  // at N = 48^3 and by 1.5% at 96^3; N >= 256K gives 256 workgroups either way.
  int64_t g = (N + FDG_RED_ELEMS - 1) / FDG_RED_ELEMS;
  if (g < 1) g = 1;
  if (g > kMaxG) g = kMaxG;
  return (int)g;
}

void launch_dots(hipStream_t s, CBatch V, int64_t ldv, IBatch nv, CBatch w, int64_t N, int64_t nbatch, int G,
                 int ldp, MBatch P, bool aligned16_all) {
  const bool vec = N % 2 == 0 && ldv % 2 == 0 && aligned16_all;
  const dim3 grid(G, (unsigned)nbatch), blk(kRed);
  if (vec)
    hipLaunchKernelGGL(k_dots<true>, grid, blk, 0, s, V, ldv, nv, w, N, G, ldp, P);
  else
    hipLaunchKernelGGL(k_dots<false>, grid, blk, 0, s, V, ldv, nv, w, N, G, ldp, P);
}

void launch_update_dots(hipStream_t s, CBatch V, int64_t ldv, IBatch nv, CBatch Pin, int G, int ldp, MBatch w,
                        int64_t N, int64_t nbatch, MBatch Pout, MBatch hout, bool aligned16_all) {
  const bool vec = N % 2 == 0 && ldv % 2 == 0 && aligned16_all;
  const dim3 grid(G, (unsigned)nbatch), blk(kRed);
  if (vec)
    hipLaunchKernelGGL(k_update_dots<true>, grid, blk, 0, s, V, ldv, nv, Pin, G, ldp, w, N, Pout, hout);
  else
    hipLaunchKernelGGL(k_update_dots<false>, grid, blk, 0, s, V, ldv, nv, Pin, G, ldp, w, N, Pout, hout);
}

void launch_update_norm(hipStream_t s, CBatch V, int64_t ldv, IBatch nv, CBatch Pin, int G, int ldp, MBatch w,
                        int64_t N, int64_t nbatch, MBatch Pnorm, CBatch h1, MBatch Hcol, MBatch host,
                        bool aligned16_all, MBatch Pdev) {
  const bool vec = N % 2 == 0 && ldv % 2 == 0 && aligned16_all;
  const dim3 grid(G, (unsigned)nbatch), blk(kRed);
  if (vec)
    hipLaunchKernelGGL(k_update_norm<true>, grid, blk, 0, s, V, ldv, nv, Pin, G, ldp, w, N, Pnorm, h1, Hcol, host,
                       Pdev);
  else
    hipLaunchKernelGGL(k_update_norm<false>, grid, blk, 0, s, V, ldv, nv, Pin, G, ldp, w, N, Pnorm, h1, Hcol, host,
                       Pdev);
}

void launch_scale_reduce(hipStream_t s, CBatch w, MBatch v, CBatch Pn, int G, int64_t N, int64_t nbatch,
                         MBatch out, MBatch host, bool aligned16_all) {
  if (N % 2 == 0 && aligned16_all)
    hipLaunchKernelGGL(k_scale_reduce<true>, dim3(stream_blocks(N, 8), (unsigned)nbatch), dim3(kBlock), 0, s, w, v,
                       Pn, G, N, out, host);
  else
    hipLaunchKernelGGL(k_scale_reduce<false>, dim3(stream_blocks(N, 1), (unsigned)nbatch), dim3(kBlock), 0, s, w, v,
                       Pn, G, N, out, host);
}

void launch_scale_by(hipStream_t s, CBatch w, MBatch v, const double *dtab, double dval, int64_t N, int64_t nbatch,
                     bool aligned16_all) {
  if (N % 2 == 0 && aligned16_all)
    hipLaunchKernelGGL(k_scale_by<true>, dim3(stream_blocks(N, 8), (unsigned)nbatch), dim3(kBlock), 0, s, w, v, dtab,
                       dval, N);
  else
    hipLaunchKernelGGL(k_scale_by<false>, dim3(stream_blocks(N, 1), (unsigned)nbatch), dim3(kBlock), 0, s, w, v, dtab,
                       dval, N);
}

void launch_norm_reduce(hipStream_t s, CBatch Pn, int G, int64_t nbatch, MBatch out, MBatch host) {
  hipLaunchKernelGGL(k_norm_reduce, dim3((unsigned)nbatch), dim3(kBlock), 0, s, Pn, G, out, host);
}

void launch_lincomb(hipStream_t s, MBatch x, CBatch Z, int64_t ldz, IBatch k, const Coeffs &y, const double *ytab,
                    int64_t N, int64_t nbatch, IBatch overwrite, bool aligned16_all) {
  if (N % 2 == 0 && ldz % 2 == 0 && aligned16_all)
    hipLaunchKernelGGL(k_lincomb<true>, dim3(stream_blocks(N, 8), (unsigned)nbatch), dim3(kBlock), 0, s, x, Z, ldz, k,
                       y, ytab, N, overwrite);
  else
    hipLaunchKernelGGL(k_lincomb<false>, dim3(stream_blocks(N, 4), (unsigned)nbatch), dim3(kBlock), 0, s, x, Z, ldz,
                       k, y, ytab, N, overwrite);
}

void launch_residual(hipStream_t s, CBatch b, CBatch Ax, MBatch r, int64_t N, int64_t nbatch, int G, MBatch P,
                     bool aligned16_all) {
  if (N % 2 == 0 && aligned16_all)
    hipLaunchKernelGGL(k_residual<true>, dim3(G, (unsigned)nbatch), dim3(kRed), 0, s, b, Ax, r, N, G, P);
  else
    hipLaunchKernelGGL(k_residual<false>, dim3(G, (unsigned)nbatch), dim3(kRed), 0, s, b, Ax, r, N, G, P);
}

}  // namespace fdg
