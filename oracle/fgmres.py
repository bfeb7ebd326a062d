"""Flexible GMRES(m) for the oracle (test infrastructure only; see package header).

Sec. 3 names GMRES as a Krylov method for the nonsymmetric system (eq. 3.1)
with the preconditioner P applied at every iteration; the paper's experiments
use BiCGStab and state no tolerance, starting guess, side or orthogonalisation.
Readings fixed here:
* right preconditioning in the flexible form (the preconditioned vectors z_j are
  kept), x0 = 0 unless given, restart length m;
* classical Gram-Schmidt with one full reorthogonalisation (CGS2);
* Givens rotations r = hypot(a, b), c = a / r, s = b / r on the Hessenberg
  columns, residual estimate |g_{j+1}|;
* a cycle stops when |g_{j+1}| <= rtol ||b||, on lucky breakdown
  (h_{j+1,j} <= 1e-14 ||A z_j||, with ||A z_j|| taken as the 2-norm of the
  Hessenberg column, equal to it because the basis is orthonormal), at the
  restart length, or at maxit;
* at the end of a cycle x += Z y (back-substitution) and the true residual
  ||b - A x|| decides convergence; otherwise the next cycle restarts from x.
"""
import numpy as np


def _givens(a, b):
    if b == 0.0:
        return 1.0, 0.0, a
    r = np.hypot(a, b)
    return a / r, b / r, r


def fgmres(matvec, prec, b, rtol=1e-8, restart=30, maxit=1000, x0=None, iters=None):
    """Solve A x = b.  matvec(v) = A v, prec(v) ~ P^{-1} v.

    If ``iters`` is given the solver runs exactly that many inner iterations in
    total (restarting every ``restart``) and ignores rtol inside a cycle; this is
    the fixed-count mode used to compare two implementations of the same
    iteration.  Returns (x, info) where info holds iterations, restarts, the
    residual-estimate history, the true relative residual and a converged flag."""
    b = np.asarray(b, dtype=np.float64)
    N = b.shape[0]
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    target = rtol * bnorm
    total = 0
    restarts = 0
    hist = []
    limit = maxit if iters is None else iters
    if bnorm == 0.0:                                # A nonsingular: A x = 0 has x = 0
        return np.zeros(N), dict(iterations=0, restarts=0, history=[], rel_res=0.0, converged=True)
    while True:
        r = b - matvec(x) if np.any(x) else b.copy()
        beta = np.linalg.norm(r)
        if (iters is None and beta <= target) or total >= limit:
            return x, dict(iterations=total, restarts=restarts, history=hist,
                           rel_res=beta / bnorm, converged=beta <= target)
        m = restart
        V = np.zeros((m + 1, N))
        Z = np.zeros((m, N))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = matvec(Z[j])
            h1 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h1
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            H[:j + 1, j] = h1 + h2
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            wnorm0 = np.linalg.norm(H[:j + 2, j])    # = ||A z_j|| (V orthonormal)
            for i in range(j):                      # previous rotations
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            cs[j], sn[j], H[j, j] = _givens(H[j, j], H[j + 1, j])
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            breakdown = hn <= 1e-14 * wnorm0
            if not breakdown:
                V[j + 1] = w / hn
            if total >= limit or breakdown:
                break
            if iters is None and abs(g[j + 1]) <= target:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):             # back-substitution R y = g
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        restarts += 1
        if total >= limit:
            r = b - matvec(x)
            rn = np.linalg.norm(r)
            return x, dict(iterations=total, restarts=restarts, history=hist,
                           rel_res=rn / bnorm, converged=rn <= target)


def arnoldi_check(matvec, prec, b, k):
    """Run k FGMRES steps from x0 = 0 and return (V, Z, Hbar) without Givens, for the
    Arnoldi-relation pin A Z_k = V_{k+1} Hbar_k and the orthogonality of V."""
    N = b.shape[0]
    V = np.zeros((k + 1, N))
    Z = np.zeros((k, N))
    H = np.zeros((k + 1, k))
    V[0] = b / np.linalg.norm(b)
    for j in range(k):
        Z[j] = prec(V[j])
        w = matvec(Z[j])
        h1 = V[:j + 1] @ w
        w = w - V[:j + 1].T @ h1
        h2 = V[:j + 1] @ w
        w = w - V[:j + 1].T @ h2
        H[:j + 1, j] = h1 + h2
        H[j + 1, j] = np.linalg.norm(w)
        V[j + 1] = w / H[j + 1, j]
    return V, Z, H
