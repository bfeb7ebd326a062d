"""GPU: preconditioned BiCGStab (the Krylov method of Sec. 5, counted in half steps,
"k + 0.5") against the BiCGStab oracle, on the unit cube (A = P), the deformed cube
(assembled and matrix-free operators), the Galerkin convection-diffusion matrix and the
full-size deformed workload."""
import numpy as np
import pytest

from oracle import bicgstab as obi
from oracle import colloc, fd
from oracle import galerkin as G
from paper_1705_04384_amd import inputs
from tests.gpu_helpers import oracle_unit, relerr, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _fdg():
    torch_cuda()
    from paper_1705_04384_amd import fdgmres
    fdgmres.lib()
    return fdgmres


def _oracle_deformed(p, n):
    A = colloc.deformed_operator(p, n, 0.1)
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    return A, (lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v))


@pytest.mark.parametrize("d,p,n", [(3, 3, 20), (2, 3, 33), (3, 4, 40)])
def test_exact_preconditioner_half_iteration(d, p, n):
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(d, p, n)
    b = inputs.rhs_normal(21, n ** d)
    x = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    info = ctx.bicgstab(to_dev(b), x, rtol=1e-8)
    assert info["converged"] and info["iterations"] == 0.5 and info["half_steps"] == 1
    _, prec = oracle_unit(p, n, d)
    assert relerr(x.cpu().numpy(), prec(b)) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("kind,p,n", [("csr", 3, 12), ("csr", 2, 10), ("mapped", 3, 12), ("mapped", 4, 9)])
def test_deformed_matches_oracle(kind, p, n):
    # free-running: the same half-step count as the oracle (one either way at the threshold);
    # fixed count: the same iterate
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.deformed_problem(p, n, 0.1) if kind == "csr" else fdg.mapped_problem(p, n, 0.1)
    A, prec = _oracle_deformed(p, n)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    xo, io = obi.bicgstab(lambda v: A @ v, prec, b, rtol=1e-8)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.bicgstab(to_dev(b), x, rtol=1e-8)
    assert info["converged"] and abs(info["half_steps"] - io["half_steps"]) <= 1
    assert relerr(A @ x.cpu().numpy(), b) <= 1e-8
    k = int(io["iterations"])
    xk, _ = obi.bicgstab(lambda v: A @ v, prec, b, iters=k)
    ctx.bicgstab(to_dev(b), x, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
    assert relerr(x.cpu().numpy(), xk) <= 1e-8
    ctx.close()


def test_galerkin_convection_matches_oracle():
    fdg = _fdg()
    torch = torch_cuda()
    p, n, amp, wind, beta = 3, 16, 0.1, (10.0, 10.0, 10.0), 0.5
    ctx = fdg.galerkin_problem(p, n, amp, wind, beta)
    A = G.galerkin_operator(p, n, amp, wind, beta)
    facs = [G.galerkin_factors(p, n, G.affine_wind(c)) for c in wind]
    fac = [fd.factor_pencil(f[1] + f[2], f[0]) for f in facs]
    prec = lambda v: fd.fd_apply([f[0] for f in fac], [f[1] for f in fac], [f[2] for f in fac], v)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    xo, io = obi.bicgstab(lambda v: A @ v, prec, b, rtol=1e-8)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.bicgstab(to_dev(b), x, rtol=1e-8)
    assert info["converged"] and abs(info["half_steps"] - io["half_steps"]) <= 1
    k = int(io["iterations"])
    xk, _ = obi.bicgstab(lambda v: A @ v, prec, b, iters=k)
    ctx.bicgstab(to_dev(b), x, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
    assert relerr(x.cpu().numpy(), xk) <= 1e-8
    ctx.close()


def test_fp32_preconditioner_reaches_fp64_residual():
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 14
    ctx = fdg.deformed_problem(p, n, 0.1, prec=fdg.PREC_FP32)
    A, _ = _oracle_deformed(p, n)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.bicgstab(to_dev(b), x, rtol=1e-10)
    assert info["converged"] and info["rel_res_true"] <= 1e-10
    assert relerr(A @ x.cpu().numpy(), b) <= 1e-10
    ctx.close()


def test_start_guess_zero_rhs_and_budget():
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 10
    ctx = fdg.deformed_problem(p, n, 0.1)
    A, _ = _oracle_deformed(p, n)
    b = inputs.rhs_uniform(5, n ** 3)
    xd = np.linalg.solve(A.toarray(), b)
    x = to_dev(xd)
    info = ctx.bicgstab(to_dev(b), x, rtol=1e-8, flags=fdg.SOLVE_USE_X0)
    assert info["converged"] and info["half_steps"] == 0
    x = to_dev(np.ones(n ** 3))
    info = ctx.bicgstab(to_dev(np.zeros(n ** 3)), x, flags=fdg.SOLVE_USE_X0)
    assert info["converged"] and not np.any(x.cpu().numpy())
    info = ctx.bicgstab(to_dev(b), x, rtol=1e-14, maxit=2)
    assert not info["converged"] and info["full_iterations"] <= 2
    ctx.close()


def test_full_size_deformed_against_fgmres():
    # p = 3, n = 96 (the deformed-cube workload): BiCGStab and FGMRES(30) solve the same
    # system to rtol 1e-8 (true residuals), so their solutions agree to the conditioning
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 96
    ctx = fdg.deformed_problem(p, n, 0.1)
    b = to_dev(inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3))
    xb = torch.empty_like(b)
    xg = torch.empty_like(b)
    ib = ctx.bicgstab(b, xb, rtol=1e-8)
    ig = ctx.solve(b, xg, rtol=1e-8, restart=30)
    assert ib["converged"] and ig["converged"]
    assert ib["rel_res_true"] <= 1e-8
    assert relerr(xb.cpu().numpy(), xg.cpu().numpy()) <= 1e-6
    ctx.close()
