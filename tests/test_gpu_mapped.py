"""GPU: the matrix-free operator of the deformed cube (1D factors M, D1, K and the nine
chain-rule coefficient fields, sum factorization on the device) against the oracle's
assembled collocation matrix, alone, in batches, inside FGMRES and through the server."""
import numpy as np
import pytest

from oracle import colloc, fd, fgmres
from paper_1705_04384_amd import inputs
from tests.gpu_helpers import relerr, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _fdg():
    torch_cuda()
    from paper_1705_04384_amd import fdgmres
    fdgmres.lib()
    return fdgmres


@pytest.mark.parametrize("p,n", [(3, 12), (4, 9), (2, 10), (6, 13), (3, 70), (5, 33)])
def test_mapped_matvec_matches_assembled_oracle(p, n):
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.mapped_problem(p, n, 0.1)
    A = colloc.deformed_operator(p, n, 0.1)
    x = inputs.rhs_uniform(31, n ** 3)
    y = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    ctx.matvec(to_dev(x), y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), A @ x) <= 1e-13
    ctx.close()


def test_mapped_matvec_full_size_p3_n96():
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 96
    ctx = fdg.mapped_problem(p, n, 0.1)
    A = colloc.deformed_operator(p, n, 0.1).tocsr()
    x = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    y = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    ctx.matvec(to_dev(x), y)
    torch.cuda.synchronize()
    assert relerr(y.cpu().numpy(), A @ x) <= 1e-13
    ctx.close()


def test_mapped_batch_entries_equal_single():
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 20
    one = fdg.mapped_problem(p, n, 0.1)
    M, K, D1, _ = fdg.colloc_factors(p, n)
    U, V, lam, _ = fdg.factor_pencil(K, M)
    two = fdg.Context(3, n, batch=2)
    for l in range(3):
        two.set_prec_factors(l, U, V, lam)
        two.set_operator_mapped(l, M, D1, K)
    two.set_operator_fields(fdg.deformed_coefficients(p, n, 0.1))
    xs = [inputs.rhs_uniform(40 + k, n ** 3) for k in range(2)]
    yb = torch.empty(2 * n ** 3, dtype=torch.float64, device="cuda")
    two.matvec(to_dev(np.concatenate(xs)), yb)
    y1 = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    for k in range(2):
        one.matvec(to_dev(xs[k]), y1)
        torch.cuda.synchronize()
        assert np.array_equal(yb.cpu().numpy()[k * n ** 3:(k + 1) * n ** 3], y1.cpu().numpy())
    one.close()
    two.close()


@pytest.mark.parametrize("p,n,restart", [(3, 12, 30), (3, 10, 6)])
def test_mapped_solve_matches_oracle(p, n, restart):
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.mapped_problem(p, n, 0.1)
    A = colloc.deformed_operator(p, n, 0.1)
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    prec = lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    xo, io = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-8, restart=restart)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-8, restart=restart)
    assert info["converged"] and info["iterations"] == io["iterations"]
    k = io["iterations"]
    ctx.solve(to_dev(b), x, rtol=1e-8, restart=restart, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
    assert relerr(x.cpu().numpy(), xo) <= 1e-8
    ctx.close()


def test_mapped_served_mix_equals_solo():
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.mapped_problem(3, 12, 0.1)
    srv = fdg.Server(max_slots=8, restart=10, lanes=1, arena_bytes=128 << 20)
    bs = [to_dev(inputs.rhs_uniform(60 + k, ctx.N)) for k in range(3)]
    xs = [torch.empty_like(b) for b in bs]
    for k in range(3):
        assert srv.admit(ctx, bs[k], xs[k], rtol=1e-8, tag=k)
    res = {}
    while srv.pending() > 0:
        for tag, st, info in srv.step(wait_us=1000):
            res[tag] = info
    assert srv.stats()["max_group"] >= 2
    for k in range(3):
        x1 = torch.empty_like(bs[k])
        info = ctx.solve(bs[k], x1, rtol=1e-8, restart=10)
        assert info["iterations"] == res[k]["iterations"]
        assert np.array_equal(x1.cpu().numpy(), xs[k].cpu().numpy())
    srv.close()
    ctx.close()
