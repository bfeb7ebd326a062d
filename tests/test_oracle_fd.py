"""Pins of the oracle's fast-diagonalization solve (Sec. 4, eq. 4.6-4.9).

* Brute force: the dense Kronecker matrix (numpy.kron of the factors, eq. 2.7 /
  2.9) solved with numpy.linalg.solve, for n <= 8, d = 2, 3.
* The identity P (P^{-1} v) = v at larger sizes.
* Remark 1: real positive eigenvalues, well-conditioned eigenvectors; the
  lowest eigenvalues approach the 1D Dirichlet Laplacian ones, (k pi)^2.
* The symmetric special case (p = 2 collocation: symmetric pencil with SPD M):
  M-orthonormal U gives V = U, and the symmetric FD equals the nonsymmetric one.
* The flop count printed in Sec. 4.1 (8 n^3 in 2D, 12 n^4 in 3D).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import colloc, fd


def _dense_P(Ms, Ks):
    d = len(Ms)
    P = 0
    for l in range(d):
        mats = [Ks[q] if q == l else Ms[q] for q in range(d)]
        T = mats[-1]
        for F in reversed(mats[:-1]):
            T = np.kron(T, F)
        P = P + T
    return P


@pytest.mark.parametrize("d,p,n", [(2, 3, 6), (2, 4, 8), (3, 3, 5), (3, 6, 7), (3, 2, 6), (2, 5, 7)])
def test_fd_equals_dense_solve(d, p, n):
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    b = np.random.default_rng(d + 10 * p + 100 * n).standard_normal(n ** d)
    s = fd.fd_apply([U] * d, [V] * d, [lam] * d, b)
    ref = np.linalg.solve(_dense_P([M] * d, [K] * d), b)
    assert np.linalg.norm(s - ref) <= 1e-12 * np.linalg.norm(ref)


def test_fd_mixed_directions_dense():
    """Different pencils per direction (different n and p) still give P^{-1} exactly."""
    specs = [(3, 5), (4, 6), (2, 4)]
    Ms, Ks, Us, Vs, lams = [], [], [], [], []
    for p, n in specs:
        M, K, _, _ = colloc.colloc_factors(p, n)
        U, V, lam = fd.factor_pencil(K, M)
        Ms.append(M); Ks.append(K); Us.append(U); Vs.append(V); lams.append(lam)
    N = int(np.prod([n for _, n in specs]))
    b = np.random.default_rng(5).standard_normal(N)
    s = fd.fd_apply(Us, Vs, lams, b)
    ref = np.linalg.solve(_dense_P(Ms, Ks), b)
    assert np.linalg.norm(s - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("d,p,n", [(3, 4, 24), (2, 3, 64), (3, 6, 20)])
def test_kronecker_identity(d, p, n):
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    P = colloc.unit_operator([M] * d, [K] * d)
    v = np.random.default_rng(1).standard_normal(n ** d)
    s = fd.fd_apply([U] * d, [V] * d, [lam] * d, v)
    assert np.linalg.norm(P @ s - v) <= 1e-12 * np.linalg.norm(v)


@pytest.mark.parametrize("p,n", [(2, 16), (3, 33), (4, 64), (5, 40), (6, 48), (3, 96), (4, 128), (6, 192), (5, 47), (6, 47)])
def test_remark1_real_positive_wellconditioned(p, n):
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    assert np.all(lam > 0)
    assert np.linalg.cond(U) < 100
    # K U = M U D
    assert np.linalg.norm(K @ U - M @ U * lam) <= 1e-10 * np.linalg.norm(K)
    # V^T M U = I by construction of V
    assert np.allclose(V.T @ M @ U, np.eye(n), atol=1e-10)


def test_low_eigenvalues_approach_dirichlet_laplacian():
    M, K, _, _ = colloc.colloc_factors(4, 128)
    _, _, lam = fd.factor_pencil(K, M)
    for k in range(1, 4):
        assert abs(lam[k - 1] - (k * np.pi) ** 2) <= 1e-6 * (k * np.pi) ** 2


@pytest.mark.parametrize("p,n", [(3, 96), (4, 128)])
def test_double_outlier_kronecker_identity(p, n):
    """Where the two outlier eigenvalues coincide to rounding, P^{-1} is still exact (2D)."""
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    assert lam[-1] - lam[-2] <= 1e-12 * lam[-1]
    P = colloc.unit_operator([M] * 2, [K] * 2)
    v = np.random.default_rng(3).standard_normal(n * n)
    s = fd.fd_apply([U] * 2, [V] * 2, [lam] * 2, v)
    assert np.linalg.norm(P @ s - v) <= 1e-12 * np.linalg.norm(v)


def test_outlier_eigenvalue_pair():
    """Remark 1: the top of the spectrum holds an outlier of algebraic multiplicity two."""
    M, K, _, _ = colloc.colloc_factors(3, 33)
    _, _, lam = fd.factor_pencil(K, M)
    assert abs(lam[-1] - lam[-2]) <= 1e-6 * lam[-1]
    assert lam[-2] - lam[-3] > 0.1 * lam[-1]


def test_symmetric_case_recovers_symmetric_fd():
    p, n, d = 2, 9, 3
    M, K, _, _ = colloc.colloc_factors(p, n)
    assert np.allclose(M, M.T, atol=1e-15) and np.allclose(K, K.T, atol=1e-12)
    lam_s, Us = sla.eigh(K, M)                  # M-orthonormal eigenvectors
    Vs = np.linalg.inv(M @ Us).T
    assert np.allclose(Vs, Us, atol=1e-12)
    U, V, lam = fd.factor_pencil(K, M)
    b = np.random.default_rng(2).standard_normal(n ** d)
    s1 = fd.fd_apply([Us] * d, [Us] * d, [lam_s] * d, b)
    s2 = fd.fd_apply([U] * d, [V] * d, [lam] * d, b)
    assert np.linalg.norm(s1 - s2) <= 1e-12 * np.linalg.norm(s1)


def test_complex_pencil_rejected():
    rng = np.random.default_rng(0)
    K = rng.standard_normal((8, 8))
    M = np.eye(8)
    with pytest.raises(fd.ComplexPencilError):
        fd.factor_pencil(K, M)


def test_flop_count_from_section_4_1():
    n = 37
    assert fd.fd_flops(2, n) == 8 * n ** 3
    assert fd.fd_flops(3, n) == 12 * n ** 4
