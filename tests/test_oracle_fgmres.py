"""Pins of the oracle's flexible GMRES.

* A = P (unit domain, exact FD preconditioner): converges in one iteration with
  x = P^{-1} b (the preconditioned operator is the identity).
* Arnoldi relation A Z_k = V_{k+1} Hbar_k and orthonormal V (CGS2).
* Deformed cube: the solution agrees with a sparse direct solve (scipy
  spsolve, independent library) to the accuracy the tolerance implies.
* Unpreconditioned small dense systems vs numpy.linalg.solve, including a
  restart length shorter than the iteration count.
* Iteration counts stay nearly flat in h and p (Sec. 5 observation).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import colloc, fd, fgmres


def _fd(p, n, d):
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    return M, K, (lambda v: fd.fd_apply([U] * d, [V] * d, [lam] * d, v))


@pytest.mark.parametrize("d,p,n", [(2, 3, 33), (3, 4, 16)])
def test_unit_domain_one_iteration(d, p, n):
    M, K, prec = _fd(p, n, d)
    P = colloc.unit_operator([M] * d, [K] * d)
    b = colloc.manufactured_rhs(p, n, d)
    x, info = fgmres.fgmres(lambda v: P @ v, prec, b, rtol=1e-8, restart=30)
    assert info["iterations"] == 1 and info["converged"]
    assert info["rel_res"] < 1e-12
    assert np.linalg.norm(x - prec(b)) <= 1e-13 * np.linalg.norm(x)


def test_arnoldi_relation_and_orthogonality():
    p, n = 3, 8
    A = colloc.deformed_operator(p, n, 0.1)
    _, _, prec = _fd(p, n, 3)
    b = np.random.default_rng(4).uniform(-1, 1, n ** 3)
    k = 12
    V, Z, H = fgmres.arnoldi_check(lambda v: A @ v, prec, b, k)
    AZ = np.stack([A @ Z[j] for j in range(k)])
    assert np.linalg.norm(AZ - H.T @ V) <= 1e-12 * np.linalg.norm(AZ)
    assert np.abs(V @ V.T - np.eye(k + 1)).max() <= 1e-13


@pytest.mark.parametrize("n", [8, 12])
def test_deformed_against_direct_solve(n):
    p = 3
    A = colloc.deformed_operator(p, n, 0.1)
    _, _, prec = _fd(p, n, 3)
    b = np.random.default_rng(2).uniform(-1, 1, n ** 3)
    x, info = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-12, restart=30)
    ref = spla.spsolve(A.tocsc(), b)
    assert info["converged"]
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)


def test_dense_unpreconditioned_with_restarts():
    rng = np.random.default_rng(9)
    n = 40
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    x, info = fgmres.fgmres(lambda v: A @ v, lambda v: v.copy(), b, rtol=1e-10, restart=7, maxit=500)
    assert info["converged"] and info["restarts"] > 1
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-8 * np.linalg.norm(x)


def test_fixed_iteration_mode_and_history():
    p, n = 3, 8
    A = colloc.deformed_operator(p, n, 0.1)
    _, _, prec = _fd(p, n, 3)
    b = np.random.default_rng(2).uniform(-1, 1, n ** 3)
    x5, info5 = fgmres.fgmres(lambda v: A @ v, prec, b, iters=5, restart=30)
    assert info5["iterations"] == 5
    # the residual estimate is the true residual of the cycle's iterate
    assert abs(info5["history"][-1] - info5["rel_res"]) <= 1e-10
    # history is non-increasing (GMRES minimises the residual)
    h = np.array(info5["history"])
    assert np.all(np.diff(h) <= 1e-14)


def test_iterations_nearly_flat_in_h_and_p():
    its = {}
    for p in (2, 3, 4):
        for n in (8, 12, 16):
            A = colloc.deformed_operator(p, n, 0.1)
            _, _, prec = _fd(p, n, 3)
            b = np.random.default_rng(2).uniform(-1, 1, n ** 3)
            _, info = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-8, restart=30)
            assert info["converged"]
            its[(p, n)] = info["iterations"]
    assert max(its.values()) <= 40
    assert max(its.values()) <= 2 * min(its.values())


@pytest.mark.parametrize("k,m", [(12, 5), (7, 7), (9, 4), (20, 6)])
def test_fixed_count_iterate_is_the_restarted_minimal_residual_iterate(k, m):
    """The fixed-count mode (iters=k), the reference of every fixed-count GPU comparison,
    against its definition computed another way: each cycle of restarted, right-
    preconditioned GMRES minimises ||b - A x|| over x_c + P^{-1} K_s(A P^{-1}, r_c)
    (s = m, the last cycle shorter), here by a dense least-squares solve over an explicit
    (normalised power) basis of that Krylov space, on a small deformed-cube system."""
    from paper_1705_04384_amd import inputs
    p, n = 3, 6
    A = colloc.deformed_operator(p, n, 0.1).toarray()
    _, _, prec = _fd(p, n, 3)
    b = inputs.rhs_uniform(5, n ** 3)
    xo, info = fgmres.fgmres(lambda v: A @ v, prec, b, restart=m, iters=k)
    assert info["iterations"] == k and info["restarts"] == -(-k // m)
    x = np.zeros(n ** 3)
    done = 0
    while done < k:
        s = min(m, k - done)
        r = b - A @ x
        cols = [r / np.linalg.norm(r)]
        for _ in range(1, s):
            w = A @ prec(cols[-1])
            cols.append(w / np.linalg.norm(w))
        Z = np.column_stack([prec(c) for c in cols])
        c, *_ = np.linalg.lstsq(A @ Z, r, rcond=None)
        x = x + Z @ c
        done += s
    assert np.linalg.norm(x - xo) <= 1e-11 * np.linalg.norm(x)
    assert np.max(np.abs(x - xo)) <= 1e-11 * np.max(np.abs(x))
    # and the agreement is sharp: one step fewer is far further away
    xk1, _ = fgmres.fgmres(lambda v: A @ v, prec, b, restart=m, iters=k - 1)
    assert np.linalg.norm(xk1 - xo) > 100 * np.linalg.norm(x - xo)
