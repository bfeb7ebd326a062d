// Host setup for the Galerkin discretization of Sec. 3.2: Gauss quadrature, the
// univariate factors of eq. 3.8 with the convection factor H after eq. 3.9, and the
// Galerkin matrix of -Lap u + w . grad u on the deformed cube (CSR).  No GPU is touched.
//
// Quadrature: p + 1 Gauss-Legendre points on every knot span (the paper assumes
// standard Gaussian quadrature; exact for M, K and for H with an affine wind).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "common.h"
#include "spline_eval.h"

namespace fdg {
namespace {

// Gauss-Legendre nodes and weights on [-1, 1] for k points: Newton's method on the
// Legendre polynomial P_k (three-term recurrence) from the classical starting values
// cos(pi (i + 3/4) / (k + 1/2)); w_i = 2 / ((1 - x_i^2) P_k'(x_i)^2).
void gauss_legendre(int k, double *x, double *w) {
  for (int i = 0; i < k; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (k + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // P_0, P_1
      for (int j = 2; j <= k; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = k * (z * p1 - p0) / (z * z - 1.0);  // P_k'(z)
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) <= 1e-16) break;
    }
    // recompute the derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= k; ++j) {
      const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = k * (z * p1 - p0) / (z * z - 1.0);
    x[k - 1 - i] = z;  // ascending
    w[k - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// The 1D rule of the whole interval: E spans x (p+1) points, ascending, with the values
// and first derivatives of the p+1 B-splines that live on each span.
struct Rule1D {
  int p = 0, n = 0, E = 0, P = 0;     // P = p + 1 points per span
  std::vector<double> x, w;           // E * P
  std::vector<double> val, der;       // [(e*P + k)*P + t]: B_{e+t}, B'_{e+t} at point k of span e
};

int make_rule(int p, int n, Rule1D &r) {
  if (p < 1 || p > 15 || n < 1 || n + 2 - p < 1)
    return set_error(FDG_EINVAL, "galerkin: need 1 <= p <= 15 and n >= p - 1 (p=%d n=%d)", p, n);
  r.p = p;
  r.n = n;
  r.E = n + 2 - p;
  r.P = p + 1;
  const int E = r.E, P = r.P;
  const std::vector<int64_t> kn = open_knots(p, E);
  std::vector<double> xi(kn.size());
  for (size_t i = 0; i < kn.size(); ++i) xi[i] = (double)kn[i] / (double)E;
  double g[16], gw[16];
  gauss_legendre(P, g, gw);
  r.x.resize((size_t)E * P);
  r.w.resize((size_t)E * P);
  r.val.resize((size_t)E * P * P);
  r.der.resize((size_t)E * P * P);
  LocalBasis lb;
  for (int e = 0; e < E; ++e)
    for (int k = 0; k < P; ++k) {
      const double x = (e + 0.5 * (g[k] + 1.0)) / E;
      const size_t q = (size_t)e * P + k;
      r.x[q] = x;
      r.w[q] = 0.5 * gw[k] / E;
      eval_local(xi, p, x, lb);
      if (lb.span != e + p) return set_error(FDG_EINVAL, "galerkin: quadrature point outside its span");
      for (int t = 0; t < P; ++t) {
        r.val[q * P + t] = lb.f[0][t];
        r.der[q * P + t] = lb.f[1][t];
      }
    }
  return FDG_OK;
}

// The deformed cube F_a(xi) = xi_a + amp sin(2 pi xi_{a+1}) sin(2 pi xi_{a+2}) (cyclic):
// F(xi), det J and J^{-1}.
void map_at(const double xi[3], double amp, double F[3], double &det, double Ji[3][3]) {
  const double tp = 2.0 * M_PI;
  double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (int a = 0; a < 3; ++a) {
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    const double s1 = std::sin(tp * xi[b1]), c1 = std::cos(tp * xi[b1]);
    const double s2 = std::sin(tp * xi[b2]), c2 = std::cos(tp * xi[b2]);
    F[a] = xi[a] + amp * s1 * s2;
    J[a][b1] += amp * tp * c1 * s2;
    J[a][b2] += amp * tp * s1 * c2;
  }
  double A[3][3];  // adjugate
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ji[i][j] = A[i][j] / det;
}

// Per-row column window of the Galerkin pattern: |j_l - i_l| <= p in every direction.
inline int win_lo(int i, int p) { return std::max(0, i - p); }
inline int win_len(int i, int p, int n) { return std::min(n - 1, i + p) - win_lo(i, p) + 1; }

struct Assembler {
  const Rule1D *r;
  double amp, c[3], beta;
  int64_t n;
  const int64_t *rowptr;
  double *val;

  // Adds the local matrices of every element of slab e3 into val.
  void slab(int e3) const {
    const int p = r->p, P = r->P, E = r->E;
    const int P2 = P * P, P3 = P2 * P;
    constexpr int kTerms = 12;  // 9 diffusion pairs (a, b), 3 convection components b
    std::vector<double> coef((size_t)kTerms * P3);
    std::vector<double> R1((size_t)P2 * P2), R2((size_t)P2 * P2 * P);
    std::vector<double> loc((size_t)P3 * P3);
    const bool conv = c[0] != 0.0 || c[1] != 0.0 || c[2] != 0.0;
    // test / trial derivative order of direction l for term tm
    auto ord = [](int tm, int l, int &dt, int &du) {
      if (tm < 9) {
        dt = (l == tm / 3);
        du = (l == tm % 3);
      } else {
        dt = 0;
        du = (l == tm - 9);
      }
    };
    for (int e2 = 0; e2 < E; ++e2)
      for (int e1 = 0; e1 < E; ++e1) {
        const int ee[3] = {e1, e2, e3};
        // coefficients at the element's quadrature points, weights folded in
        for (int k3 = 0; k3 < P; ++k3)
          for (int k2 = 0; k2 < P; ++k2)
            for (int k1 = 0; k1 < P; ++k1) {
              const size_t q1 = (size_t)e1 * P + k1, q2 = (size_t)e2 * P + k2, q3 = (size_t)e3 * P + k3;
              const double xi[3] = {r->x[q1], r->x[q2], r->x[q3]};
              const double om = r->w[q1] * r->w[q2] * r->w[q3];
              double F[3], det, Ji[3][3];
              map_at(xi, amp, F, det, Ji);
              const int kk = (k3 * P + k2) * P + k1;
              for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                  double s = 0.0;
                  for (int m = 0; m < 3; ++m) s += Ji[a][m] * Ji[b][m];
                  coef[(size_t)(a * 3 + b) * P3 + kk] = om * det * s;
                }
              if (conv) {
                const double tp = 2.0 * M_PI;
                double wv[3];
                for (int a = 0; a < 3; ++a) {
                  const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
                  wv[a] = c[a] * (1.0 + F[a]) * (1.0 + beta * std::cos(tp * F[b1]) * std::cos(tp * F[b2]));
                }
                for (int a = 0; a < 3; ++a) {
                  double s = 0.0;
                  for (int m = 0; m < 3; ++m) s += Ji[a][m] * wv[m];
                  coef[(size_t)(9 + a) * P3 + kk] = om * det * s;
                }
              }
            }
        std::fill(loc.begin(), loc.end(), 0.0);
        const int nterm = conv ? kTerms : 9;
        for (int tm = 0; tm < nterm; ++tm) {
          const double *C = coef.data() + (size_t)tm * P3;
          int dt[3], du[3];
          for (int l = 0; l < 3; ++l) ord(tm, l, dt[l], du[l]);
          const double *ft[3], *fu[3];
          for (int l = 0; l < 3; ++l) {
            const size_t base = (size_t)ee[l] * P * P;
            ft[l] = (dt[l] ? r->der.data() : r->val.data()) + base;  // [k*P + t]
            fu[l] = (du[l] ? r->der.data() : r->val.data()) + base;
          }
          // R1[(t1*P + u1)][k3*P + k2] = sum_k1 ft1(k1, t1) fu1(k1, u1) C[k3][k2][k1]
          for (int t1 = 0; t1 < P; ++t1)
            for (int u1 = 0; u1 < P; ++u1)
              for (int k32 = 0; k32 < P2; ++k32) {
                double s = 0.0;
                for (int k1 = 0; k1 < P; ++k1) s += ft[0][k1 * P + t1] * fu[0][k1 * P + u1] * C[k32 * P + k1];
                R1[(size_t)(t1 * P + u1) * P2 + k32] = s;
              }
          // R2[(t1 u1)][(t2 u2)][k3] = sum_k2 ft2(k2, t2) fu2(k2, u2) R1[(t1 u1)][k3 k2]
          for (int a = 0; a < P2; ++a)
            for (int t2 = 0; t2 < P; ++t2)
              for (int u2 = 0; u2 < P; ++u2)
                for (int k3 = 0; k3 < P; ++k3) {
                  double s = 0.0;
                  for (int k2 = 0; k2 < P; ++k2)
                    s += ft[1][k2 * P + t2] * fu[1][k2 * P + u2] * R1[(size_t)a * P2 + k3 * P + k2];
                  R2[((size_t)a * P2 + t2 * P + u2) * P + k3] = s;
                }
          // loc[t][u] += sum_k3 ft3(k3, t3) fu3(k3, u3) R2[(t1 u1)][(t2 u2)][k3]
          for (int t1 = 0; t1 < P; ++t1)
            for (int u1 = 0; u1 < P; ++u1)
              for (int t2 = 0; t2 < P; ++t2)
                for (int u2 = 0; u2 < P; ++u2) {
                  const double *r2 = R2.data() + (((size_t)(t1 * P + u1) * P2) + t2 * P + u2) * P;
                  for (int t3 = 0; t3 < P; ++t3)
                    for (int u3 = 0; u3 < P; ++u3) {
                      double s = 0.0;
                      for (int k3 = 0; k3 < P; ++k3) s += ft[2][k3 * P + t3] * fu[2][k3 * P + u3] * r2[k3];
                      loc[(size_t)((t3 * P + t2) * P + t1) * P3 + (u3 * P + u2) * P + u1] += s;
                    }
                }
        }
        // scatter: local function t of direction l is unknown e_l + t - 1 when in [0, n)
        for (int t3 = 0; t3 < P; ++t3)
          for (int t2 = 0; t2 < P; ++t2)
            for (int t1 = 0; t1 < P; ++t1) {
              const int i1 = e1 + t1 - 1, i2 = e2 + t2 - 1, i3 = e3 + t3 - 1;
              if (i1 < 0 || i1 >= n || i2 < 0 || i2 >= n || i3 < 0 || i3 >= n) continue;
              const int64_t row = i1 + n * (i2 + n * (int64_t)i3);
              const int lo1 = win_lo(i1, p), lo2 = win_lo(i2, p), lo3 = win_lo(i3, p);
              const int w1 = win_len(i1, p, (int)n), w2 = win_len(i2, p, (int)n);
              double *rv = val + rowptr[row];
              const double *lr = loc.data() + (size_t)((t3 * P + t2) * P + t1) * P3;
              for (int u3 = 0; u3 < P; ++u3) {
                const int j3 = e3 + u3 - 1;
                if (j3 < 0 || j3 >= n) continue;
                for (int u2 = 0; u2 < P; ++u2) {
                  const int j2 = e2 + u2 - 1;
                  if (j2 < 0 || j2 >= n) continue;
                  for (int u1 = 0; u1 < P; ++u1) {
                    const int j1 = e1 + u1 - 1;
                    if (j1 < 0 || j1 >= n) continue;
                    rv[((int64_t)(j3 - lo3) * w2 + (j2 - lo2)) * w1 + (j1 - lo1)] += lr[(u3 * P + u2) * P + u1];
                  }
                }
              }
            }
      }
  }
};

}  // namespace
}  // namespace fdg

using namespace fdg;

extern "C" int fdg_galerkin_factors(int p, int n, double w0, double w1, double *M, double *K, double *H) {
  clear_error();
  if (!std::isfinite(w0) || !std::isfinite(w1)) return set_error(FDG_EINVAL, "galerkin_factors: wind not finite");
  Rule1D r;
  int st = make_rule(p, n, r);
  if (st != FDG_OK) return st;
  const size_t nn = (size_t)n * n;
  std::vector<double> m(nn, 0.0), k(nn, 0.0), h(nn, 0.0);
  const int P = r.P;
  for (int e = 0; e < r.E; ++e)
    for (int q = 0; q < P; ++q) {
      const size_t g = (size_t)e * P + q;
      const double wt = r.w[g], wind = w0 + w1 * r.x[g];
      for (int t = 0; t < P; ++t) {
        const int i = e + t - 1;  // interior unknown of local function t
        if (i < 0 || i >= n) continue;
        for (int u = 0; u < P; ++u) {
          const int j = e + u - 1;
          if (j < 0 || j >= n) continue;
          const double bt = r.val[g * P + t], bu = r.val[g * P + u];
          const double dt = r.der[g * P + t], du = r.der[g * P + u];
          m[(size_t)i * n + j] += wt * bt * bu;
          k[(size_t)i * n + j] += wt * dt * du;
          h[(size_t)i * n + j] += wt * wind * bt * du;
        }
      }
    }
  if (M) std::memcpy(M, m.data(), nn * sizeof(double));
  if (K) std::memcpy(K, k.data(), nn * sizeof(double));
  if (H) std::memcpy(H, h.data(), nn * sizeof(double));
  return FDG_OK;
}

extern "C" int fdg_galerkin_csr(int p, int n, double amp, const double *wind, double beta, int64_t *nnz,
                                int64_t *rowptr, int32_t *col, double *val) {
  clear_error();
  if (!nnz) return set_error(FDG_EINVAL, "galerkin_csr: nnz is NULL");
  if (!std::isfinite(amp) || !std::isfinite(beta)) return set_error(FDG_EINVAL, "galerkin_csr: amp/beta not finite");
  if (wind)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(wind[a])) return set_error(FDG_EINVAL, "galerkin_csr: wind not finite");
  if ((int64_t)n * n * n > INT32_MAX) return set_error(FDG_EINVAL, "galerkin_csr: n too large");
  Rule1D r;
  int st = make_rule(p, n, r);
  if (st != FDG_OK) return st;
  int64_t total = 0;
  for (int i3 = 0; i3 < n; ++i3)
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1) total += (int64_t)win_len(i1, p, n) * win_len(i2, p, n) * win_len(i3, p, n);
  *nnz = total;
  if (!rowptr && !col && !val) return FDG_OK;
  if (!rowptr || !col || !val) return set_error(FDG_EINVAL, "galerkin_csr: output arrays must all be given");
  const int64_t nl = n;
  int64_t pos = 0;
  rowptr[0] = 0;
  for (int i3 = 0; i3 < n; ++i3)
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1) {
        const int lo1 = win_lo(i1, p), lo2 = win_lo(i2, p), lo3 = win_lo(i3, p);
        const int w1 = win_len(i1, p, n), w2 = win_len(i2, p, n), w3 = win_len(i3, p, n);
        for (int j3 = lo3; j3 < lo3 + w3; ++j3)
          for (int j2 = lo2; j2 < lo2 + w2; ++j2)
            for (int j1 = lo1; j1 < lo1 + w1; ++j1) {
              col[pos] = (int32_t)(j1 + nl * (j2 + nl * j3));
              val[pos] = 0.0;
              ++pos;
            }
        rowptr[i1 + nl * (i2 + nl * i3) + 1] = pos;
      }
  Assembler as;
  as.r = &r;
  as.amp = amp;
  for (int a = 0; a < 3; ++a) as.c[a] = wind ? wind[a] : 0.0;
  as.beta = beta;
  as.n = n;
  as.rowptr = rowptr;
  as.val = val;
  // Slabs e3 and e3 + (p+1) touch disjoint rows (i3 in [e3-1, e3+p-1]), so the slabs of
  // one residue class mod p+1 are assembled concurrently; classes run one after another.
  const int P = r.P;
  int nthr = (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  for (int cls = 0; cls < P; ++cls) {
    std::vector<int> slabs;
    for (int e3 = cls; e3 < r.E; e3 += P) slabs.push_back(e3);
    const int nt = std::min<int>(nthr, (int)slabs.size());
    std::vector<std::thread> pool;
    auto work = [&](int t) {
      for (size_t s = t; s < slabs.size(); s += nt) as.slab(slabs[s]);
    };
    try {
      for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
    } catch (...) {  // no more threads: the calling thread takes the rest
    }
    const int started = (int)pool.size() + 1;
    for (int t = 0; t < nt; ++t)
      if (t == 0 || t >= started) work(t);
    for (auto &th : pool) th.join();
  }
  return FDG_OK;
}
