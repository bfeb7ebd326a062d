"""GPU: the Galerkin preconditioners of Sec. 3.2 -- the symmetric FD of eq. 3.7 / 3.8
(V = U) and the nonsymmetric FD of the convection pencils of eq. 3.9 (K_l + H_l) -- and
FGMRES on the Galerkin convection-diffusion matrix, against the oracle."""
import functools

import numpy as np
import pytest

from oracle import colloc, fd, fgmres
from oracle import galerkin as G
from paper_1705_04384_amd import inputs
from tests.gpu_helpers import relerr, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

WIND = (10.0, 10.0, 10.0)
BETA = 0.5
AMP = 0.1


@functools.lru_cache(maxsize=4)
def _oracle_operator(p, n, amp, wind, beta):
    return G.galerkin_operator(p, n, amp, wind, beta)


def _fdg():
    torch_cuda()
    from paper_1705_04384_amd import fdgmres
    fdgmres.lib()
    return fdgmres


def _sym_context(fdg, d, p, n, prec=0):
    M, K, _ = fdg.galerkin_factors(p, n)
    U, lam = fdg.factor_pencil_sym(K, M)
    ctx = fdg.Context(d, n)
    for l in range(d):
        ctx.set_prec_factors_sym(l, U, lam)
        ctx.set_operator_kron(l, M, K)
    ctx.set_precision(prec)
    return ctx


def _oracle_sym(d, p, n):
    M, K, _ = G.galerkin_factors(p, n)
    U, lam = G.factor_pencil_sym(K, M)
    P = colloc.unit_operator([M] * d, [K] * d)
    return P, lambda v: fd.fd_apply([U] * d, [U] * d, [lam] * d, v)


def _oracle_wind(p, n, winds):
    facs = [G.galerkin_factors(p, n, G.affine_wind(c)) for c in winds]
    Ms = [f[0] for f in facs]
    KHs = [f[1] + f[2] for f in facs]
    fac = [fd.factor_pencil(KH, M) for KH, M in zip(KHs, Ms)]
    P = colloc.unit_operator(Ms, KHs)
    return P, lambda v: fd.fd_apply([f[0] for f in fac], [f[1] for f in fac], [f[2] for f in fac], v)


@pytest.mark.parametrize("d,p,n", [(3, 3, 20), (3, 2, 33), (3, 4, 37), (2, 3, 47), (2, 6, 70)])
def test_symmetric_fd_apply_matches_oracle(d, p, n):
    fdg = _fdg()
    torch = torch_cuda()
    ctx = _sym_context(fdg, d, p, n)
    b = inputs.rhs_normal(11, n ** d)
    s = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    P, prec = _oracle_sym(d, p, n)
    assert relerr(s.cpu().numpy(), prec(b)) <= 1e-12
    # the Kronecker operator of the same factors on the device inverts it
    y = torch.empty_like(s)
    ctx.matvec(s, y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), b) <= 1e-12
    ctx.close()


def test_symmetric_fd_apply_fp32():
    fdg = _fdg()
    torch = torch_cuda()
    d, p, n = 3, 3, 40
    ctx = _sym_context(fdg, d, p, n, prec=fdg.PREC_FP32)
    b = inputs.rhs_normal(12, n ** d)
    s = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    P, prec = _oracle_sym(d, p, n)
    sg = s.cpu().numpy()
    assert relerr(P @ sg, b) <= 5e-5
    assert relerr(sg, prec(b)) <= 5e-4
    ctx.close()


@pytest.mark.parametrize("p,n,winds", [(3, 24, (2.0, 4.0, 6.0)), (2, 40, (10.0, 5.0, 1.0)), (4, 17, (3.0, 3.0, 3.0))])
def test_convection_fd_apply_matches_oracle(p, n, winds):
    # distinct winds per direction: a direction mix-up changes the result
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.Context(3, n)
    for l in range(3):
        M, K, H = fdg.galerkin_factors(p, n, winds[l], winds[l])
        U, V, lam, _ = fdg.factor_pencil(K + H, M, want_cond=False)
        ctx.set_prec_factors(l, U, V, lam)
        ctx.set_operator_kron(l, M, K + H)
    b = inputs.rhs_uniform(13, n ** 3)
    s = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    P, prec = _oracle_wind(p, n, winds)
    assert relerr(s.cpu().numpy(), prec(b)) <= 1e-12
    y = torch.empty_like(s)
    ctx.matvec(s, y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), b) <= 1e-12
    assert relerr(y.cpu().numpy(), P @ s.cpu().numpy()) <= 1e-13
    ctx.close()


@pytest.mark.parametrize("p,n", [(3, 10), (2, 13)])
def test_galerkin_matvec_matches_oracle(p, n):
    fdg = _fdg()
    torch = torch_cuda()
    # (the preconditioner is not used; the symmetric one exists at any mesh size)
    ctx = fdg.galerkin_problem(p, n, AMP, WIND, BETA, wind_prec=False)
    A = _oracle_operator(p, n, AMP, WIND, BETA)
    x = inputs.rhs_uniform(14, n ** 3)
    y = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    ctx.matvec(to_dev(x), y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), A @ x) <= 1e-13
    ctx.close()


@pytest.mark.parametrize("wind_prec", [True, False])
def test_galerkin_solve_matches_oracle(wind_prec):
    # same iterations free-running; same iterate after the oracle's count (fixed iterations)
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 16
    ctx = fdg.galerkin_problem(p, n, AMP, WIND, BETA, wind_prec=wind_prec)
    A = _oracle_operator(p, n, AMP, WIND, BETA)
    _, prec = _oracle_wind(p, n, WIND) if wind_prec else _oracle_sym(3, p, n)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    xo, io = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-8, restart=30)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-8, restart=30)
    assert info["converged"] and abs(info["iterations"] - io["iterations"]) <= 1
    assert relerr(A @ x.cpu().numpy(), b) <= 1e-8
    k = io["iterations"]
    ctx.solve(to_dev(b), x, rtol=1e-8, restart=30, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
    assert relerr(x.cpu().numpy(), xo) <= 1e-8
    ctx.close()


def test_wind_in_preconditioner_cuts_iterations():
    # Sec. 3.2: putting a univariate approximation of the wind into P (eq. 3.9) makes it
    # more effective than dropping the convection term (eq. 3.7)
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 24
    b = to_dev(inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3))
    x = torch.empty_like(b)
    its = {}
    for wp in (True, False):
        ctx = fdg.galerkin_problem(p, n, 0.0, WIND, BETA, wind_prec=wp)
        info = ctx.solve(b, x, rtol=1e-8, restart=30)
        assert info["converged"]
        its[wp] = info["iterations"]
        ctx.close()
    assert its[True] < its[False], its


def test_galerkin_bench_size_properties():
    # p = 3, n = 48 (the measured configuration): P P^{-1} b = b for both preconditioners
    # through the device Kronecker operator, the ELL matvec of the 343-wide rows against a
    # host product with the same CSR, and a converged solve with an FP64 true residual
    import scipy.sparse as sp
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 48
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    bd = to_dev(b)
    s = torch.empty_like(bd)
    y = torch.empty_like(bd)
    sym = _sym_context(fdg, 3, p, n)
    sym.apply_prec(bd, s)
    sym.matvec(s, y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), b) <= 1e-12
    sym.close()
    ctx = fdg.galerkin_problem(p, n, AMP, WIND, BETA)
    rowptr, col, val = fdg.galerkin_csr(p, n, AMP, WIND, BETA)
    A = sp.csr_matrix((val, col, rowptr), shape=(n ** 3, n ** 3))
    ctx.matvec(bd, y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), A @ b) <= 1e-13
    x = torch.empty_like(bd)
    info = ctx.solve(bd, x, rtol=1e-8, restart=30)
    assert info["converged"]
    assert relerr(A @ x.cpu().numpy(), b) <= 1e-8
    ctx.close()


# ---- pencils with complex eigenvalue pairs (Sec. 4, the remark after eq. 4.7) -----------

def _blocks_context(fdg, d, p, n, winds):
    ctx = fdg.Context(d, n)
    Ms, KHs = [], []
    npairs, cond = 0, 1.0
    for l in range(d):
        M, K, H = fdg.galerkin_factors(p, n, winds[l], winds[l])
        U, V, lam, mu, cu = fdg.factor_pencil_blocks(K + H, M, want_cond=True)
        npairs += int((mu > 0).sum())
        cond = max(cond, cu)
        if mu.any():
            ctx.set_prec_factors_blocks(l, U, V, lam, mu)
        else:   # directions with real eigenvalues set through the plain entry point
            ctx.set_prec_factors(l, U, V, lam)
        ctx.set_operator_kron(l, M, K + H)
        Ms.append(M)
        KHs.append(K + H)
    return ctx, Ms, KHs, npairs, cond


# winds past the point where the pencils turn complex, with eigenvector bases of moderate
# condition (right after the transition they are nearly defective)
@pytest.mark.parametrize("d,p,n,winds", [(3, 3, 8, (10.0, 20.0, 15.0)), (3, 3, 20, (100.0, 150.0, 80.0)),
                                         (2, 3, 33, (150.0, 150.0)), (2, 2, 17, (150.0, 80.0)),
                                         (3, 4, 24, (150.0, 100.0, 80.0)), (3, 2, 17, (80.0, 100.0, 150.0)),
                                         (3, 2, 17, (150.0, 1.0, 5.0)), (3, 3, 20, (1.0, 100.0, 2.0)),
                                         (2, 2, 17, (1.0, 150.0))])
def test_complex_pencil_fd_apply_matches_oracle(d, p, n, winds):
    # the device keeps D in real 2 x 2 blocks; the oracle runs the FD in complex arithmetic.
    # Tolerance: rounding amplified by the condition of the eigenvector basis
    fdg = _fdg()
    torch = torch_cuda()
    ctx, Ms, KHs, npairs, cond = _blocks_context(fdg, d, p, n, winds)
    assert npairs > 0
    # cond(U) of these cases is 66 .. 1.33e4 (host factorization, deterministic): bounded
    # here so that the tolerance cannot grow loose unnoticed (tol <= 2.1e-9)
    assert cond <= 2e4, cond
    tol = 1e-13 * cond + 1e-10
    b = inputs.rhs_normal(31, n ** d)
    s = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    fac = [fd.factor_pencil(KH, M, allow_complex=True) for KH, M in zip(KHs, Ms)]
    so = fd.fd_apply([f[0] for f in fac], [f[1] for f in fac], [f[2] for f in fac], b)
    assert relerr(s.cpu().numpy(), so) <= tol
    y = torch.empty_like(s)
    ctx.matvec(s, y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), b) <= tol
    ctx.close()


def test_complex_blocks_unfused_beyond_256():
    # n > 256 runs unfused mode products around the block solve.  Synthetic factors: U
    # orthogonal, V = U (M = I), D with 2 x 2 blocks, so P = K_2 x I + I x K_1 with
    # K_l = U D_l U^T, checked by applying P to the result in numpy
    fdg = _fdg()
    torch = torch_cuda()
    n = 300
    rng = np.random.default_rng(41)
    ctx = fdg.Context(2, n)
    Ks = []
    for l in range(2):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = np.sort(rng.uniform(1.0, 50.0, n))
        mu = np.zeros(n)
        for c in range(l, n - 1, 7):
            lam[c + 1] = lam[c]
            mu[c], mu[c + 1] = 3.0 + c % 5, -(3.0 + c % 5)
        D = np.diag(lam)
        for c in range(n - 1):
            if mu[c] > 0:
                D[c, c + 1], D[c + 1, c] = mu[c], mu[c + 1]
        ctx.set_prec_factors_blocks(l, Q, Q, lam, mu)
        Ks.append(Q @ D @ Q.T)
    b = inputs.rhs_normal(32, n * n)
    s = torch.empty(n * n, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    S = s.cpu().numpy().reshape(n, n)           # S[i2][i1]
    Ps = S @ Ks[0].T + Ks[1] @ S
    assert relerr(Ps.ravel(), b) <= 1e-11
    ctx.close()


def test_galerkin_solve_with_complex_pencils():
    # strong wind on a coarse mesh: the eq. 3.9 pencils have complex pairs; FGMRES with the
    # block FD against the oracle (complex FD): same iterations, same iterate
    fdg = _fdg()
    torch = torch_cuda()
    p, n, amp, wind, beta = 3, 10, 0.1, (10.0, 10.0, 10.0), 0.5
    ctx = fdg.galerkin_problem(p, n, amp, wind, beta)
    A = _oracle_operator(p, n, amp, wind, beta)
    facs = [G.galerkin_factors(p, n, G.affine_wind(c)) for c in wind]
    fac = [fd.factor_pencil(f[1] + f[2], f[0], allow_complex=True) for f in facs]
    assert max(np.abs(f[2].imag).max() for f in fac) > 0
    prec = lambda v: fd.fd_apply([f[0] for f in fac], [f[1] for f in fac], [f[2] for f in fac], v)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    xo, io = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-8, restart=30)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-8, restart=30)
    assert info["converged"] and abs(info["iterations"] - io["iterations"]) <= 1
    k = io["iterations"]
    ctx.solve(to_dev(b), x, rtol=1e-8, restart=30, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
    assert relerr(x.cpu().numpy(), xo) <= 1e-8
    # the server runs such a context one request at a time, with the same bits
    srv = fdg.Server(max_slots=4, restart=30, lanes=1, arena_bytes=64 << 20)
    bd = to_dev(b)
    xs = [torch.empty_like(bd) for _ in range(2)]
    for t in range(2):
        assert srv.admit(ctx, bd, xs[t], rtol=1e-8, tag=t)
    while srv.pending() > 0:
        srv.step(wait_us=1000)
    x1 = torch.empty_like(bd)
    ctx.solve(bd, x1, rtol=1e-8, restart=30)
    for t in range(2):
        assert np.array_equal(xs[t].cpu().numpy(), x1.cpu().numpy())
    srv.close()
    # reduced precision needs real eigenvalues
    ctx.set_precision(fdg.PREC_FP32)
    with pytest.raises(fdg.FdgError):
        ctx.apply_prec(bd, x1)
    ctx.close()


def test_block_factor_arguments_are_checked():
    # malformed pairs are rejected before anything is stored
    fdg = _fdg()
    n = 12
    ctx = fdg.Context(2, n)
    M, K, H = fdg.galerkin_factors(3, n, 100.0, 100.0)
    U, V, lam, mu, _ = fdg.factor_pencil_blocks(K + H, M)
    c = int(np.flatnonzero(mu > 0)[0])
    bad1 = mu.copy(); bad1[c + 1] = mu[c]            # second entry not -b
    bad2 = mu.copy(); bad2[c] = -mu[c]; bad2[c + 1] = mu[c]   # pair starting with -b
    bad3 = np.zeros(n); bad3[n - 1] = 1.0            # pair running past n
    for bad in (bad1, bad2, bad3):
        with pytest.raises(fdg.FdgError):
            ctx.set_prec_factors_blocks(0, U, V, lam, bad)
    ctx.set_prec_factors_blocks(0, U, V, lam, mu)
    ctx.close()
