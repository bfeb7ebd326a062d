// Host FP64 factorisation of a symmetric-definite pencil for the symmetric FD method.
//
// Sec. 4, after eq. 4.6: when K is symmetric and M symmetric positive definite the
// eigenvectors of M^{-1} K can be chosen M-orthonormal (U^T M U = I), and then
// V = (M U)^{-T} = U, which is the symmetric FD method; eq. 3.7 / 3.8 give such pencils
// (univariate Galerkin factors).
//
// Method: Cholesky M = L L^T, C = L^{-1} K L^{-T} (symmetric), cyclic Jacobi rotations
// C = Q diag(lambda) Q^T (each rotation zeroes one off-diagonal pair, the classical
// symmetric Schur step; a pair is skipped once |c_pq| <= eps sqrt(|c_pp c_qq|), which
// keeps small eigenvalues to high relative accuracy), then U = L^{-T} Q.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"

using namespace fdg;

extern "C" int fdg_factor_pencil_sym(int n, const double *K, const double *M, double *U, double *lambda) {
  clear_error();
  if (n < 1 || n > 4096 || !K || !M || !U || !lambda) return set_error(FDG_EINVAL, "factor_pencil_sym: bad arguments");
  const size_t nn = (size_t)n * n;
  double kmax = 0.0, mmax = 0.0;
  for (size_t i = 0; i < nn; ++i) {
    if (!std::isfinite(K[i]) || !std::isfinite(M[i])) return set_error(FDG_EINVAL, "factor_pencil_sym: non-finite input");
    kmax = std::max(kmax, std::fabs(K[i]));
    mmax = std::max(mmax, std::fabs(M[i]));
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const size_t a = (size_t)i * n + j, b = (size_t)j * n + i;
      if (std::fabs(K[a] - K[b]) > 1e-12 * kmax || std::fabs(M[a] - M[b]) > 1e-12 * mmax)
        return set_error(FDG_EINVAL, "factor_pencil_sym: K or M not symmetric (entry %d,%d)", i, j);
    }
  // Cholesky of the symmetric part of M (lower triangle used)
  std::vector<double> L(nn, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = M[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0.0)) return set_error(FDG_EINVAL, "factor_pencil_sym: M not positive definite");
    const double d = std::sqrt(s);
    L[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / d;
    }
  }
  // Y = L^{-1} Ks (forward substitution, column by column of Ks = sym(K)), C = L^{-1} Y^T
  std::vector<double> Y(nn), C(nn);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Y[(size_t)i * n + j] = 0.5 * (K[(size_t)i * n + j] + K[(size_t)j * n + i]);
  auto forward = [&](std::vector<double> &X) {  // X <- L^{-1} X, all columns
    for (int i = 0; i < n; ++i) {
      double *xi = X.data() + (size_t)i * n;
      for (int k = 0; k < i; ++k) {
        const double l = L[(size_t)i * n + k];
        if (l == 0.0) continue;
        const double *xk = X.data() + (size_t)k * n;
        for (int j = 0; j < n; ++j) xi[j] -= l * xk[j];
      }
      const double d = L[(size_t)i * n + i];
      for (int j = 0; j < n; ++j) xi[j] /= d;
    }
  };
  forward(Y);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[(size_t)i * n + j] = Y[(size_t)j * n + i];
  forward(C);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const double s = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
      C[(size_t)i * n + j] = C[(size_t)j * n + i] = s;
    }
  // cyclic Jacobi; Q accumulated by columns in row-major Qt (Qt[k][i] = Q[i][k])
  std::vector<double> Qt(nn, 0.0);
  for (int i = 0; i < n; ++i) Qt[(size_t)i * n + i] = 1.0;
  const double eps = 2.2e-16;
  double cnorm = 0.0;  // Frobenius norm of C: floor of the skip test for indefinite input
  for (double x : C) cnorm += x * x;
  cnorm = std::sqrt(cnorm);
  const double skip_floor = eps * eps * cnorm + 1e-300;
  bool done = false;
  for (int sweep = 0; sweep < 60 && !done; ++sweep) {
    done = true;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = C[(size_t)p * n + q];
        const double app = C[(size_t)p * n + p], aqq = C[(size_t)q * n + q];
        if (std::fabs(apq) <= eps * std::sqrt(std::fabs(app * aqq)) || std::fabs(apq) <= skip_floor) {
          C[(size_t)p * n + q] = C[(size_t)q * n + p] = 0.0;
          continue;
        }
        done = false;
        const double tau = (aqq - app) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        double *rp = C.data() + (size_t)p * n, *rq = C.data() + (size_t)q * n;
        for (int k = 0; k < n; ++k) {  // rows p and q
          const double x = rp[k], y = rq[k];
          rp[k] = c * x - s * y;
          rq[k] = s * x + c * y;
        }
        for (int k = 0; k < n; ++k) {  // columns p and q
          double *rk = C.data() + (size_t)k * n;
          const double x = rk[p], y = rk[q];
          rk[p] = c * x - s * y;
          rk[q] = s * x + c * y;
        }
        C[(size_t)p * n + q] = C[(size_t)q * n + p] = 0.0;
        double *qp = Qt.data() + (size_t)p * n, *qq = Qt.data() + (size_t)q * n;
        for (int k = 0; k < n; ++k) {
          const double x = qp[k], y = qq[k];
          qp[k] = c * x - s * y;
          qq[k] = s * x + c * y;
        }
      }
  }
  if (!done) return set_error(FDG_ENOCONV, "factor_pencil_sym: Jacobi sweeps did not converge");
  // U = L^{-T} Q: back substitution L^T u_k = q_k for every column (rows of Qt)
  std::vector<double> Ut(Qt);
  for (int k = 0; k < n; ++k) {
    double *u = Ut.data() + (size_t)k * n;
    for (int i = n - 1; i >= 0; --i) {
      double s = u[i];
      for (int j = i + 1; j < n; ++j) s -= L[(size_t)j * n + i] * u[j];
      u[i] = s / L[(size_t)i * n + i];
    }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return C[(size_t)a * n + a] < C[(size_t)b * n + b]; });
  for (int k = 0; k < n; ++k) {
    const int src = order[k];
    lambda[k] = C[(size_t)src * n + src];
    for (int i = 0; i < n; ++i) U[(size_t)i * n + k] = Ut[(size_t)src * n + i];
  }
  if (!(lambda[0] > 0.0)) return set_error(FDG_ECOMPLEX, "factor_pencil_sym: non-positive eigenvalue %g", lambda[0]);
  return FDG_OK;
}
