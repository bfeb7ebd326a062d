"""GPU parity at the full workload sizes, in the launch configuration the benchmark times.

- 2D unit square, p = 3, n = 33, manufactured right-hand side, FGMRES(30), FP64.
- 3D unit cube, p = 4, n = 128, manufactured and N(0,1) right-hand sides, FGMRES(30).
- 3D deformed cube, p = 3, n = 96, CSR operator (27 nonzeros per row), U[-1,1] right-hand
  side, FGMRES(30): the library's CSR equals the oracle's assembled operator, the solve
  stops at the oracle's iteration, and a fixed-count solve matches the oracle iterate; the
  literal (2p+1)^3 = 343-wide stencil (explicit zeros) gives the same matvec.
- 3D unit cube, p = 6, n = 192, N(0,1) right-hand side, FGMRES(50) with P^{-1} in FP64,
  FP32 and BF16-in/FP32-accumulate: the iteration count k* at which the solution error
  against the oracle (A = P, so x = P^{-1} b) reaches 1e-8.
"""
import numpy as np
import pytest

from oracle import colloc, fd, fgmres
from paper_1705_04384_amd import inputs
from tests.gpu_helpers import maxrel, relerr, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _fdg():
    torch_cuda()
    from paper_1705_04384_amd import fdgmres
    fdgmres.lib()
    return fdgmres


def _oracle_unit(p, n, d):
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    mv = lambda v: colloc.unit_matvec([M] * d, [K] * d, v)
    pr = lambda v: fd.fd_apply([U] * d, [V] * d, [lam] * d, v)
    return mv, pr


def test_c1_2d_p3_n33():
    fdg = _fdg()
    torch = torch_cuda()
    d, p, n = 2, 3, 33
    ctx = fdg.unit_problem(d, p, n)
    f = colloc.manufactured_rhs(p, n, d)
    x = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(f), x, rtol=1e-8, restart=30)
    mv, pr = _oracle_unit(p, n, d)
    xo, io = fgmres.fgmres(mv, pr, f, rtol=1e-8, restart=30)
    assert info["converged"] and info["iterations"] == io["iterations"]
    assert relerr(x.cpu().numpy(), xo) <= 1e-8 and maxrel(x.cpu().numpy(), xo) <= 1e-8
    ctx.close()


@pytest.mark.parametrize("rhs", ["manufactured", "normal"])
def test_c2_3d_p4_n128(rhs):
    fdg = _fdg()
    torch = torch_cuda()
    d, p, n = 3, 4, 128
    ctx = fdg.unit_problem(d, p, n)
    f = colloc.manufactured_rhs(p, n, d) if rhs == "manufactured" else inputs.rhs_normal(inputs.SEED_NOISE_128,
                                                                                           n ** d)
    x = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(f), x, rtol=1e-8, restart=30)
    mv, pr = _oracle_unit(p, n, d)
    xo, io = fgmres.fgmres(mv, pr, f, rtol=1e-8, restart=30)
    assert info["converged"] and info["iterations"] == io["iterations"] == 1
    assert info["rel_res_true"] <= 1e-8
    assert relerr(x.cpu().numpy(), xo) <= 1e-8 and maxrel(x.cpu().numpy(), xo) <= 1e-8
    ctx.close()


def test_c3_deformed_p3_n96():
    fdg = _fdg()
    torch = torch_cuda()
    p, n, restart = 3, 96, 30
    N = n ** 3
    A = colloc.deformed_operator(p, n, 0.1).tocsr()
    rowptr, col, val = fdg.deformed_csr(p, n, 0.1)
    assert len(col) == 27 * N
    import scipy.sparse as sp
    Al = sp.csr_matrix((val, col, rowptr), shape=(N, N))
    diff = abs(Al - A).max()
    assert diff <= 1e-11 * abs(A).max(), diff
    ctx = fdg.deformed_problem(p, n, 0.1)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, N)
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    pr = lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v)
    xo, io = fgmres.fgmres(lambda v: A @ v, pr, b, rtol=1e-8, restart=restart)
    x = torch.empty(N, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-8, restart=restart)
    assert info["converged"] and io["converged"]
    assert info["iterations"] == io["iterations"] and info["restarts"] == io["restarts"]
    # the residual the library reports, recomputed on the host from the oracle's operator
    xg = x.cpu().numpy()
    assert np.linalg.norm(b - A @ xg) <= 1e-8 * np.linalg.norm(b)
    k = io["iterations"]
    xf = torch.empty(N, dtype=torch.float64, device="cuda")
    ctx.solve(to_dev(b), xf, rtol=1e-8, restart=restart, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
    assert relerr(xf.cpu().numpy(), xo) <= 1e-8 and maxrel(xf.cpu().numpy(), xo) <= 1e-8
    # the free-running solve stops at the same iteration, so it is the same iterate
    assert relerr(xg, xo) <= 1e-8 and maxrel(xg, xo) <= 1e-8
    ctx.close()


def test_c3_literal_343_stencil_same_matvec():
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 96
    N = n ** 3
    a = fdg.deformed_problem(p, n, 0.1)
    bnd = fdg.deformed_problem(p, n, 0.1, band=True)
    # (2p+1)^3 stencil clipped at the boundary: per direction sum_i |[i-p, i+p] & [0, n)|
    width = sum(min(i + p, n - 1) - max(i - p, 0) + 1 for i in range(n))
    assert bnd.nnz == width ** 3
    xv = to_dev(inputs.rhs_uniform(11, N))
    y1 = torch.empty_like(xv)
    y2 = torch.empty_like(xv)
    a.matvec(xv, y1)
    bnd.matvec(xv, y2)
    torch.cuda.synchronize()
    assert np.array_equal(y1.cpu().numpy(), y2.cpu().numpy())
    a.close()
    bnd.close()


def test_c4_precision_sweep_p6_n192():
    fdg = _fdg()
    torch = torch_cuda()
    d, p, n = 3, 6, 192
    N = n ** d
    b = inputs.rhs_normal(inputs.SEED_SWEEP_192, N)
    _, pr = _oracle_unit(p, n, d)
    x_ref = pr(b)  # A = P on the unit cube: the exact discrete solution
    bd = to_dev(b)
    x = torch.empty(N, dtype=torch.float64, device="cuda")
    ctx = fdg.unit_problem(d, p, n)
    info = ctx.solve(bd, x, rtol=1e-8, restart=50)
    assert info["converged"] and info["iterations"] == 1
    assert relerr(x.cpu().numpy(), x_ref) <= 1e-8 and maxrel(x.cpu().numpy(), x_ref) <= 1e-8
    ctx.close()
    for prec, kmax in ((fdg.PREC_FP32, 4), (fdg.PREC_BF16, 10)):
        ctx = fdg.unit_problem(d, p, n, prec=prec)
        errs = []
        for k in range(1, kmax + 1):
            ctx.solve(bd, x, rtol=0.0, restart=50, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
            xk = x.cpu().numpy()
            errs.append(max(relerr(xk, x_ref), maxrel(xk, x_ref)))
            if errs[-1] <= 1e-8:
                break
        assert errs[-1] <= 1e-8, (prec, errs)
        ctx.close()
