// Host setup of the library: knot vectors, Greville points, B-spline evaluation,
// univariate collocation factors, the deformed-cube collocation matrix and the
// manufactured right-hand side.  No GPU is touched here.
//
// Paper: Sec. 2.1 (open knot vectors, interior functions i = 1..m-2, n = m - 2),
// eq. 2.4 (Greville abscissae), eq. 2.8 (collocation factors), Sec. 2.2 (collocation
// on a mapped domain; the general matrix is derived from the chain rule).
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "spline_eval.h"

namespace fdg {

std::vector<int64_t> open_knots(int p, int E) {
  std::vector<int64_t> k;
  k.reserve(E + 2 * p + 1);
  for (int i = 0; i <= p; ++i) k.push_back(0);
  for (int i = 1; i < E; ++i) k.push_back(i);
  for (int i = 0; i <= p; ++i) k.push_back(E);
  return k;
}

void eval_local(const std::vector<double> &xi, int p, double x, LocalBasis &out) {
  const int nk = (int)xi.size();
  int s = p;
  // locate the span: largest s with xi_s <= x among the non-empty spans p..nk-p-2
  const int last = nk - p - 2;
  if (x >= xi[last + 1]) {
    s = last;
  } else {
    int lo = p, hi = last + 1;  // invariant: xi_lo <= x < xi_hi
    while (hi - lo > 1) {
      int mid = (lo + hi) / 2;
      if (xi[mid] <= x) lo = mid; else hi = mid;
    }
    s = lo;
  }
  out.span = s;
  // tab[q][t] = B_{s-q+t, q}(x), t = 0..q
  double tab[16][16];
  tab[0][0] = 1.0;
  for (int q = 1; q <= p; ++q) {
    for (int t = 0; t <= q; ++t) {
      const int i = s - q + t;
      double v = 0.0;
      if (t > 0) {  // B_{i, q-1} is non-zero only for i >= s-q+1
        const double den = xi[i + q] - xi[i];
        if (den != 0.0) v += (x - xi[i]) / den * tab[q - 1][t - 1];
      }
      if (t < q) {  // B_{i+1, q-1}
        const double den = xi[i + q + 1] - xi[i + 1];
        if (den != 0.0) v += (xi[i + q + 1] - x) / den * tab[q - 1][t];
      }
      tab[q][t] = v;
    }
  }
  auto val = [&](int q, int i) -> double {  // B_{i,q}(x), zero outside the local window
    const int t = i - (s - q);
    return (t >= 0 && t <= q) ? tab[q][t] : 0.0;
  };
  auto d1 = [&](int q, int i) -> double {   // B'_{i,q}(x)
    if (q == 0) return 0.0;
    double r = 0.0;
    const double a = xi[i + q] - xi[i], c = xi[i + q + 1] - xi[i + 1];
    if (a != 0.0) r += q / a * val(q - 1, i);
    if (c != 0.0) r -= q / c * val(q - 1, i + 1);
    return r;
  };
  for (int t = 0; t <= p; ++t) {
    const int i = s - p + t;
    out.f[0][t] = tab[p][t];
    out.f[1][t] = d1(p, i);
    double r = 0.0;
    if (p >= 1) {
      const double a = xi[i + p] - xi[i], c = xi[i + p + 1] - xi[i + 1];
      if (a != 0.0) r += p / a * d1(p - 1, i);
      if (c != 0.0) r -= p / c * d1(p - 1, i + 1);
    }
    out.f[2][t] = r;
  }
}


// Dense univariate factors; shared by the C entry point and the CSR assembly.
int colloc_factors_impl(int p, int n, std::vector<double> &M, std::vector<double> &K,
                        std::vector<double> &D1, std::vector<double> &tau) {
  if (p < 1 || p > 15 || n < 1 || n + 2 - p < 1)
    return set_error(FDG_EINVAL, "colloc_factors: need 1 <= p <= 15 and n >= p - 1 (p=%d n=%d)", p, n);
  const int E = n + 2 - p;
  const std::vector<int64_t> kn = open_knots(p, E);
  std::vector<double> xi(kn.size());
  for (size_t i = 0; i < kn.size(); ++i) xi[i] = (double)kn[i] / (double)E;
  tau.assign(n, 0.0);
  // eq. 2.4 with 1-based knots: tau_i = (xi_{i+2} + ... + xi_{i+p+1}) / p; 0-based storage
  // puts these at numerators kn[i+1..i+p]; one rational division per point.
  for (int i = 1; i <= n; ++i) {
    int64_t sum = 0;
    for (int j = 1; j <= p; ++j) sum += kn[i + j];
    tau[i - 1] = (double)sum / (double)((int64_t)p * E);
  }
  M.assign((size_t)n * n, 0.0);
  K.assign((size_t)n * n, 0.0);
  D1.assign((size_t)n * n, 0.0);
  LocalBasis lb;
  for (int r = 0; r < n; ++r) {
    eval_local(xi, p, tau[r], lb);
    for (int t = 0; t <= p; ++t) {
      const int j = lb.span - p + t;  // global basis index 0..m-1
      if (j < 1 || j > n) continue;   // B_0 and B_{m-1} are not in the Dirichlet space
      M[(size_t)r * n + (j - 1)] = lb.f[0][t];
      D1[(size_t)r * n + (j - 1)] = lb.f[1][t];
      K[(size_t)r * n + (j - 1)] = -lb.f[2][t];
    }
  }
  return FDG_OK;
}

}  // namespace fdg

using namespace fdg;

extern "C" int fdg_colloc_factors(int p, int n, double *M, double *K, double *D1, double *tau) {
  clear_error();
  std::vector<double> m, k, d1, t;
  int st = colloc_factors_impl(p, n, m, k, d1, t);
  if (st != FDG_OK) return st;
  const size_t nn = (size_t)n * n;
  if (M) std::memcpy(M, m.data(), nn * sizeof(double));
  if (K) std::memcpy(K, k.data(), nn * sizeof(double));
  if (D1) std::memcpy(D1, d1.data(), nn * sizeof(double));
  if (tau) std::memcpy(tau, t.data(), (size_t)n * sizeof(double));
  return FDG_OK;
}

extern "C" int fdg_manufactured_rhs(int d, int n, const double *tau, double *f) {
  clear_error();
  if ((d != 2 && d != 3) || n < 1 || !tau || !f)
    return set_error(FDG_EINVAL, "manufactured_rhs: bad arguments");
  std::vector<double> s(n);
  for (int i = 0; i < n; ++i) s[i] = std::sin(M_PI * tau[i]);
  const double c = d * M_PI * M_PI;
  const int n3 = d == 3 ? n : 1;
  size_t idx = 0;
  for (int i3 = 0; i3 < n3; ++i3)
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1)
        f[idx++] = c * s[i1] * s[i2] * (d == 3 ? s[i3] : 1.0);
  return FDG_OK;
}

// ---------------------------------------------------------------------------------
// Deformed cube F_a(xi) = xi_a + amp sin(2 pi xi_{a+1}) sin(2 pi xi_{a+2}).
// ---------------------------------------------------------------------------------
namespace {

struct Geo {
  double C[3][3];  // J^{-1} J^{-T}
  double g[3];     // -J^{-1} sum_lm (d_l d_m F) C_lm
};

void geometry_at(const double xi[3], double amp, Geo &G) {
  const double w = 2.0 * M_PI;
  double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double Hs[3][3][3];
  std::memset(Hs, 0, sizeof(Hs));
  for (int a = 0; a < 3; ++a) {
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    const double s1 = std::sin(w * xi[b1]), c1 = std::cos(w * xi[b1]);
    const double s2 = std::sin(w * xi[b2]), c2 = std::cos(w * xi[b2]);
    J[a][b1] += amp * w * c1 * s2;
    J[a][b2] += amp * w * s1 * c2;
    Hs[a][b1][b1] = -amp * w * w * s1 * s2;
    Hs[a][b2][b2] = -amp * w * w * s1 * s2;
    Hs[a][b1][b2] = amp * w * w * c1 * c2;
    Hs[a][b2][b1] = amp * w * w * c1 * c2;
  }
  // inverse by the adjugate
  double A[3][3];
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
  double Ji[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Ji[i][j] = A[i][j] / det;
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += Ji[k][a] * Ji[l][a];
      G.C[k][l] = s;
    }
  double t[3];
  for (int a = 0; a < 3; ++a) {
    double s = 0.0;
    for (int l = 0; l < 3; ++l)
      for (int m = 0; m < 3; ++m) s += Hs[a][l][m] * G.C[l][m];
    t[a] = s;
  }
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int a = 0; a < 3; ++a) s += Ji[k][a] * t[a];
    G.g[k] = -s;
  }
}

}  // namespace

extern "C" int fdg_deformed_csr(int p, int n, double amp, int band, int64_t *nnz,
                                int64_t *rowptr, int32_t *col, double *val) {
  clear_error();
  if (!nnz) return set_error(FDG_EINVAL, "deformed_csr: nnz is NULL");
  if (!std::isfinite(amp)) return set_error(FDG_EINVAL, "deformed_csr: amp not finite");
  if ((int64_t)n * n * n > INT32_MAX) return set_error(FDG_EINVAL, "deformed_csr: n too large");
  std::vector<double> M, K, D1, tau;
  int st = colloc_factors_impl(p, n, M, K, D1, tau);
  if (st != FDG_OK) return st;
  // per-row column window of the 1D factors (union of M, D1, K non-zeros, or the band)
  std::vector<int> lo(n), hi(n);
  for (int i = 0; i < n; ++i) {
    if (band) {
      lo[i] = std::max(0, i - p);
      hi[i] = std::min(n - 1, i + p);
    } else {
      int a = n, b = -1;
      for (int j = 0; j < n; ++j) {
        const size_t q = (size_t)i * n + j;
        if (M[q] != 0.0 || K[q] != 0.0 || D1[q] != 0.0) {
          a = std::min(a, j);
          b = std::max(b, j);
        }
      }
      lo[i] = a;
      hi[i] = b;
    }
  }
  const int64_t N = (int64_t)n * n * n;
  int64_t total = 0;
  for (int i3 = 0; i3 < n; ++i3)
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1)
        total += (int64_t)(hi[i1] - lo[i1] + 1) * (hi[i2] - lo[i2] + 1) * (hi[i3] - lo[i3] + 1);
  *nnz = total;
  if (!rowptr && !col && !val) return FDG_OK;
  if (!rowptr || !col || !val) return set_error(FDG_EINVAL, "deformed_csr: output arrays must all be given");
  // 1D factors by derivative order: 0 -> M, 1 -> D1, 2 -> -K
  const double *F[3] = {M.data(), D1.data(), K.data()};
  const double sgn[3] = {1.0, 1.0, -1.0};
  int64_t pos = 0;
  rowptr[0] = 0;
  for (int i3 = 0; i3 < n; ++i3)
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1) {
        const int ii[3] = {i1, i2, i3};
        const double xi[3] = {tau[i1], tau[i2], tau[i3]};
        Geo G;
        geometry_at(xi, amp, G);
        for (int j3 = lo[i3]; j3 <= hi[i3]; ++j3)
          for (int j2 = lo[i2]; j2 <= hi[i2]; ++j2)
            for (int j1 = lo[i1]; j1 <= hi[i1]; ++j1) {
              const int jj[3] = {j1, j2, j3};
              double e[3][3];  // e[q][r]: r-th derivative of B_{j_q} at tau_{i_q}
              for (int q = 0; q < 3; ++q)
                for (int r = 0; r < 3; ++r) e[q][r] = sgn[r] * F[r][(size_t)ii[q] * n + jj[q]];
              double v = 0.0;
              for (int k = 0; k < 3; ++k) {
                for (int l = 0; l < 3; ++l) {
                  int o[3] = {0, 0, 0};
                  o[k] += 1;
                  o[l] += 1;
                  v -= G.C[k][l] * e[0][o[0]] * e[1][o[1]] * e[2][o[2]];
                }
                int o[3] = {0, 0, 0};
                o[k] = 1;
                v -= G.g[k] * e[0][o[0]] * e[1][o[1]] * e[2][o[2]];
              }
              col[pos] = (int32_t)(j1 + (int64_t)n * j2 + (int64_t)n * n * j3);
              val[pos] = v;
              ++pos;
            }
        rowptr[(int64_t)i1 + (int64_t)n * i2 + (int64_t)n * n * i3 + 1] = pos;
      }
  (void)N;
  return FDG_OK;
}

extern "C" int fdg_deformed_coefficients(int p, int n, double amp, double *coef) {
  clear_error();
  if (!coef) return set_error(FDG_EINVAL, "deformed_coefficients: coef is NULL");
  if (!std::isfinite(amp)) return set_error(FDG_EINVAL, "deformed_coefficients: amp not finite");
  std::vector<double> M, K, D1, tau;
  int st = colloc_factors_impl(p, n, M, K, D1, tau);
  if (st != FDG_OK) return st;
  const int64_t N = (int64_t)n * n * n;
  for (int i3 = 0; i3 < n; ++i3)
    for (int i2 = 0; i2 < n; ++i2)
      for (int i1 = 0; i1 < n; ++i1) {
        const double xi[3] = {tau[i1], tau[i2], tau[i3]};
        Geo G;
        geometry_at(xi, amp, G);
        const int64_t o = i1 + (int64_t)n * i2 + (int64_t)n * n * i3;
        coef[0 * N + o] = G.C[0][0];
        coef[1 * N + o] = G.C[1][1];
        coef[2 * N + o] = G.C[2][2];
        coef[3 * N + o] = G.C[0][1] + G.C[1][0];
        coef[4 * N + o] = G.C[0][2] + G.C[2][0];
        coef[5 * N + o] = G.C[1][2] + G.C[2][1];
        coef[6 * N + o] = G.g[0];
        coef[7 * N + o] = G.g[1];
        coef[8 * N + o] = G.g[2];
      }
  return FDG_OK;
}
