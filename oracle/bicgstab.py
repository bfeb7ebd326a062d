"""Preconditioned BiCGStab for the oracle (test infrastructure only; see package header).

Sec. 5 solves every system with BiCGStab (van der Vorst, 1992) preconditioned by P
(applied by FD), and recalls that one iteration is a BiCG step followed by one
GMRES step (a one-dimensional minimal-residual correction).  An iteration that
converges between its two halves is reported as k + 0.5.

Readings fixed here (the paper states no tolerance, start, side or shadow vector):
* right preconditioning (the preconditioned directions p^ = P^{-1} p and
  s^ = P^{-1} s update x; residuals are those of the original system), x0 = 0
  unless given, shadow residual r~ = r_0;
* after the BiCG half: s = r - alpha v, x <- x + alpha p^; after the GMRES half:
  x <- x + omega s^, r = s - omega t with omega = (t.s)/(t.t);
* a half step whose recursively updated residual satisfies ||.|| <= rtol ||b||
  is confirmed by the true residual ||b - A x||; convergence is declared only
  when the true residual satisfies it (otherwise the iteration goes on);
* iteration count: k + 0.5 when convergence comes after the BiCG half of the
  (k+1)-th iteration, i.e. k full iterations plus one half -- the convention of
  MATLAB's bicgstab, the tool of Sec. 5; k when it comes after a full iteration;
* breakdown (rho = r~.r = 0, r~.v = 0 or omega = 0 exactly) stops the iteration
  with the current iterate.
"""
import numpy as np


def bicgstab(matvec, prec, b, rtol=1e-8, maxit=1000, x0=None, iters=None, hook=None):
    """Solve A x = b.  matvec(v) = A v, prec(v) ~ P^{-1} v.

    With ``iters`` given, exactly that many full iterations run with no convergence
    test (fixed-count mode for comparing two implementations of the same iteration).
    ``hook(name, value)`` (optional) is called with the intermediate vectors and
    scalars of every half step ('rhat', 's', 'alpha', 't', 'omega', 'r').
    Returns (x, info): iterations (float, k or k + 0.5), half_steps (int),
    converged, breakdown, rel_res_true."""
    b = np.asarray(b, dtype=np.float64)
    N = b.shape[0]
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    info = {"iterations": 0.0, "half_steps": 0, "converged": False, "breakdown": False}
    if bnorm == 0.0:
        x[:] = 0.0
        info.update(converged=True, rel_res_true=0.0)
        return x, info
    target = rtol * bnorm
    fixed = iters is not None
    limit = iters if fixed else maxit
    r = b - matvec(x) if x0 is not None else b.copy()
    if not fixed and np.linalg.norm(r) <= target:
        info.update(converged=True, rel_res_true=np.linalg.norm(r) / bnorm)
        return x, info
    rhat = r.copy()
    if hook:
        hook("rhat", rhat)
    rho_prev = alpha = omega = 1.0
    p = np.zeros(N)
    v = np.zeros(N)

    def true_ok():
        return np.linalg.norm(b - matvec(x)) <= target

    for i in range(1, limit + 1):
        rho = rhat @ r
        if rho == 0.0:
            info["breakdown"] = True
            break
        if i == 1:
            p = r.copy()
        else:
            beta = (rho / rho_prev) * (alpha / omega)
            p = r + beta * (p - omega * v)
        ph = prec(p)
        v = matvec(ph)
        rv = rhat @ v
        if rv == 0.0:
            info["breakdown"] = True
            break
        alpha = rho / rv
        s = r - alpha * v
        x = x + alpha * ph
        info["half_steps"] += 1
        if hook:
            hook("alpha", alpha)
            hook("s", s)
        if not fixed and np.linalg.norm(s) <= target and true_ok():
            info.update(converged=True, iterations=(i - 1) + 0.5)
            break
        sh = prec(s)
        t = matvec(sh)
        tt = t @ t
        omega = (t @ s) / tt if tt != 0.0 else 0.0
        x = x + omega * sh
        r = s - omega * t
        info["half_steps"] += 1
        info["iterations"] = float(i)
        if hook:
            hook("t", t)
            hook("omega", omega)
            hook("r", r)
        if not fixed and np.linalg.norm(r) <= target and true_ok():
            info["converged"] = True
            break
        if omega == 0.0:
            info["breakdown"] = True
            break
        rho_prev = rho
    info["rel_res_true"] = np.linalg.norm(b - matvec(x)) / bnorm
    if fixed:
        info["converged"] = info["rel_res_true"] <= rtol
    return x, info
