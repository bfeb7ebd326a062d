"""Pins of the BiCGStab oracle (Sec. 5: BiCGStab preconditioned by the FD solve of P).

Checked against scipy's BiCGStab (a library routine running the same right-
preconditioned iteration), the exact-preconditioner special case (convergence in half
an iteration, the paper's k + 0.5 count), the orthogonality each half step enforces,
and dense solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import bicgstab, colloc, fd


def _deformed(p, n):
    A = colloc.deformed_operator(p, n, 0.1)
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    prec = lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v)
    return A, prec


def test_exact_preconditioner_converges_in_half_an_iteration():
    # A = P: p^ = P^{-1} b, v = b, alpha = 1, s = 0 after the first BiCG half -> "0.5"
    p, n = 3, 8
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    P = colloc.unit_operator([M] * 3, [K] * 3)
    prec = lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v)
    b = np.random.default_rng(1).standard_normal(n ** 3)
    x, info = bicgstab.bicgstab(lambda v: P @ v, prec, b, rtol=1e-8)
    assert info["converged"] and info["iterations"] == 0.5 and info["half_steps"] == 1
    assert np.linalg.norm(x - prec(b)) <= 1e-13 * np.linalg.norm(x)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_matches_scipy_bicgstab(k):
    # scipy's bicgstab runs the same right-preconditioned iteration (p^ = M p, x += alpha
    # p^ + omega s^); with no tolerance to stop it, k iterations give the same iterate
    A, prec = _deformed(3, 6)
    b = np.random.default_rng(2).uniform(-1, 1, A.shape[0])
    x, info = bicgstab.bicgstab(lambda v: A @ v, prec, b, iters=k)
    Mop = spla.LinearOperator(A.shape, matvec=prec, dtype=np.float64)
    xs, flag = spla.bicgstab(A, b, rtol=1e-300, atol=0.0, maxiter=k, M=Mop)
    assert info["half_steps"] == 2 * k
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


def test_half_steps_enforce_their_orthogonality():
    # BiCG half: rhat . s = rho - alpha rhat . v = 0; GMRES half: t . r = t . s - omega t . t = 0
    A, prec = _deformed(3, 6)
    b = np.random.default_rng(3).uniform(-1, 1, A.shape[0])
    seen = {}
    checks = []

    def hook(name, val):
        seen[name] = val
        if name == "s":
            checks.append(abs(seen["rhat"] @ val) / (np.linalg.norm(seen["rhat"]) * np.linalg.norm(val)))
        if name == "r":
            checks.append(abs(seen["t"] @ val) / (np.linalg.norm(seen["t"]) * np.linalg.norm(val)))

    bicgstab.bicgstab(lambda v: A @ v, prec, b, iters=6, hook=hook)
    assert len(checks) == 12
    assert max(checks) <= 1e-10


@pytest.mark.parametrize("p,n", [(3, 6), (2, 7), (4, 6)])
def test_converges_to_dense_solution(p, n):
    A, prec = _deformed(p, n)
    b = np.random.default_rng(4).uniform(-1, 1, A.shape[0])
    x, info = bicgstab.bicgstab(lambda v: A @ v, prec, b, rtol=1e-12)
    assert info["converged"] and info["rel_res_true"] <= 1e-12
    xd = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert info["half_steps"] == round(2 * info["iterations"])


def test_zero_rhs_and_start_guess():
    A, prec = _deformed(3, 5)
    x, info = bicgstab.bicgstab(lambda v: A @ v, prec, np.zeros(A.shape[0]))
    assert info["converged"] and not np.any(x)
    b = np.random.default_rng(5).uniform(-1, 1, A.shape[0])
    xd = np.linalg.solve(A.toarray(), b)
    x, info = bicgstab.bicgstab(lambda v: A @ v, prec, b, x0=xd)
    assert info["converged"] and info["half_steps"] == 0
