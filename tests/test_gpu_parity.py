"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: the FD apply is exact up to rounding on both sides, so FP64 results agree
to ~1e-13 relative (checked at 1e-11: the two sides use independently computed
eigenvector bases, whose conditioning scales the rounding).  Solves are compared
after the same number of FGMRES iterations at <= 1e-8 relative solution error.
"""
import numpy as np
import pytest

from oracle import colloc, fd, fgmres
from paper_1705_04384_amd import inputs
from tests.gpu_helpers import maxrel, oracle_unit, relerr, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _fdg():
    torch_cuda()
    from paper_1705_04384_amd import fdgmres
    fdgmres.lib()
    return fdgmres


@pytest.mark.parametrize("d,p,n,batch", [
    (2, 3, 33, 1), (3, 4, 16, 1), (3, 3, 33, 2), (2, 5, 47, 3), (3, 6, 20, 1),
    (2, 2, 64, 1), (3, 2, 17, 1), (2, 4, 130, 2), (3, 4, 70, 1),
    (2, 2, 1, 2), (3, 3, 5, 1), (3, 3, 65, 1), (2, 4, 256, 2), (2, 3, 260, 1), (3, 5, 129, 1),
    (3, 4, 128, 1),
])
def test_apply_prec_fp64(d, p, n, batch):
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(d, p, n, batch=batch)
    N = n ** d
    b = np.concatenate([inputs.rhs_normal(100 + k, N) for k in range(batch)])
    s = torch.empty(batch * N, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    got = s.cpu().numpy()
    _, prec = oracle_unit(p, n, d)
    for k in range(batch):
        ref = prec(b[k * N:(k + 1) * N])
        assert relerr(got[k * N:(k + 1) * N], ref) <= 1e-11, (d, p, n, k)
    ctx.close()


@pytest.mark.parametrize("d,p,n,batch", [(2, 3, 33, 1), (3, 4, 16, 2), (3, 6, 21, 1), (2, 5, 40, 1)])
def test_kron_matvec(d, p, n, batch):
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(d, p, n, batch=batch)
    N = n ** d
    x = np.concatenate([inputs.rhs_normal(200 + k, N) for k in range(batch)])
    y = torch.empty(batch * N, dtype=torch.float64, device="cuda")
    ctx.matvec(to_dev(x), y)
    torch.cuda.synchronize()
    P, _ = oracle_unit(p, n, d)
    got = y.cpu().numpy()
    for k in range(batch):
        assert relerr(got[k * N:(k + 1) * N], P @ x[k * N:(k + 1) * N]) <= 1e-13
    ctx.close()

@pytest.mark.parametrize("p,n,batch", [(4, 70, 2), (3, 131, 1), (6, 67, 1), (2, 66, 1), (4, 5, 3)])
def test_kron_matvec_tiles_and_tails(p, n, batch):
    """One-pass 3D matvec over several 64-column tiles, i2 row pairs and i3 chunks with
    ragged tails (n = 70, 131, 67, 66), bands of 3 to 7 taps (p = 2 .. 6) and a tensor
    smaller than one tile; against the oracle's sum-factorised product."""
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(3, p, n, batch=batch)
    N = n ** 3
    x = np.concatenate([inputs.rhs_normal(300 + k, N) for k in range(batch)])
    y = torch.empty(batch * N, dtype=torch.float64, device="cuda")
    ctx.matvec(to_dev(x), y)
    torch.cuda.synchronize()
    M, K, _, _ = colloc.colloc_factors(p, n)
    got = y.cpu().numpy()
    for k in range(batch):
        ref = colloc.unit_matvec([M] * 3, [K] * 3, x[k * N:(k + 1) * N])
        assert relerr(got[k * N:(k + 1) * N], ref) <= 1e-13, (p, n, k)
    ctx.close()



@pytest.mark.parametrize("p,n,batch", [(4, 80, 2), (3, 96, 1), (6, 100, 1), (2, 130, 1), (5, 97, 1), (4, 128, 1),
                                       (6, 133, 1), (7, 110, 1)])
def test_kron_matvec_streaming_form(p, n, batch):
    """Shapes with at least 128 workgroups per entry take the streaming one-pass form (band
    widths w = 3 to 8; 14 staged rows for w <= 6, 28 for w >= 7; chunks of 6 planes for
    w <= 4, else 8; ragged tails in every direction: 80, 100, 130, 97, 133 and 110 are not
    multiples of the 64-column tile, of the T2 = 7 RPW - w + 1 row tile or of the chunk); against
    the oracle's product element by element, and its residual form (r = b - A x with the
    |r|^2 partials) through the true residual a solve reports."""
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(3, p, n, batch=batch)
    N = n ** 3
    x = np.concatenate([inputs.rhs_normal(400 + k, N) for k in range(batch)])
    y = torch.full((batch * N,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.matvec(to_dev(x), y)
    torch.cuda.synchronize()
    M, K, _, _ = colloc.colloc_factors(p, n)
    got = y.cpu().numpy()
    for k in range(batch):
        ref = colloc.unit_matvec([M] * 3, [K] * 3, x[k * N:(k + 1) * N])
        assert relerr(got[k * N:(k + 1) * N], ref) <= 1e-13, (p, n, k)
        assert maxrel(got[k * N:(k + 1) * N], ref) <= 1e-13, (p, n, k)
    ctx.close()
    if batch == 1:
        # residual form: a solve from a start guess x0 reports ||b - A x|| / ||b|| of its
        # iterate, computed by the fused residual kernel; recompute it with the oracle
        ctx = fdg.unit_problem(3, p, n)
        b = inputs.rhs_normal(410, N)
        xd = to_dev(inputs.rhs_normal(411, N) * 1e-3)
        info = ctx.solve(to_dev(b), xd, rtol=0.0, restart=30, maxit=1,
                         flags=fdg.SOLVE_USE_X0 | fdg.SOLVE_FIXED_ITERS)
        xr = xd.cpu().numpy()
        r = b - colloc.unit_matvec([M] * 3, [K] * 3, xr)
        assert abs(info["rel_res_true"] - np.linalg.norm(r) / np.linalg.norm(b)) <= 1e-12 * max(
            1.0, info["rel_res_true"]), (info["rel_res_true"], np.linalg.norm(r) / np.linalg.norm(b))
        ctx.close()


@pytest.mark.parametrize("p,n,band", [(3, 12, False), (4, 9, False), (3, 8, True)])
def test_csr_matvec_deformed(p, n, band):
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.deformed_problem(p, n, 0.1, band=band)
    x = inputs.rhs_uniform(3, n ** 3)
    y = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    ctx.matvec(to_dev(x), y)
    torch.cuda.synchronize()
    A = colloc.deformed_operator(p, n, 0.1)
    assert relerr(y.cpu().numpy(), A @ x) <= 1e-13
    ctx.close()


@pytest.mark.parametrize("d,p,n", [(2, 3, 33), (3, 4, 24), (3, 6, 18)])
def test_solve_unit_domain_one_iteration(d, p, n):
    """A = P on the unit domain: one FGMRES iteration reaches rounding level."""
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(d, p, n)
    f = fdg.manufactured_rhs(d, n, ctx.tau)
    assert np.allclose(f, colloc.manufactured_rhs(p, n, d), rtol=1e-14, atol=1e-12)
    x = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(f), x, rtol=1e-8, restart=30)
    P, prec = oracle_unit(p, n, d)
    xo, io = fgmres.fgmres(lambda v: P @ v, prec, f, rtol=1e-8, restart=30)
    assert info["converged"] and info["iterations"] == io["iterations"] == 1
    assert info["rel_res_true"] <= 1e-12
    assert relerr(x.cpu().numpy(), xo) <= 1e-8
    ctx.close()


@pytest.mark.parametrize("p,n,restart", [(3, 12, 30), (3, 10, 6), (2, 9, 30), (4, 8, 30)])
def test_solve_deformed_matches_oracle(p, n, restart):
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.deformed_problem(p, n, 0.1)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    A = colloc.deformed_operator(p, n, 0.1)
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    prec = lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v)
    xo, io = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-8, restart=restart)
    # free-running: same stopping iteration
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-8, restart=restart)
    assert info["converged"] and io["converged"]
    assert info["iterations"] == io["iterations"], (info, io["iterations"])
    assert info["restarts"] == io["restarts"]
    # fixed count: identical iteration, solutions agree
    xf = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    k = io["iterations"]
    info_f = ctx.solve(to_dev(b), xf, rtol=1e-8, restart=restart, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
    assert info_f["iterations"] == k
    assert relerr(xf.cpu().numpy(), xo) <= 1e-8
    assert abs(info_f["rel_res_true"] - io["rel_res"]) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("k,n", [(6, 20), (20, 20), (44, 20), (20, 21)])
def test_fixed_iterations_span_every_orthogonalization_form(k, n):
    # one restart cycle of 44 steps at N = 20^3 (8 reduction chunks, ragged sub-chunks):
    # the Gram-Schmidt update-and-dots step takes nv = j + 1 basis vectors, so k = 6 uses
    # the register form only, 20 adds the grouped-lane forms (2 lanes per element for
    # nv 9..16, 4 for 17..32) and 44 the two-read form; N = 21^3 is odd, so the basis
    # vectors are not 16-byte aligned and every form takes its one-element path
    fdg = _fdg()
    torch = torch_cuda()
    p, restart = 3, 44
    ctx = fdg.deformed_problem(p, n, 0.1)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    A = colloc.deformed_operator(p, n, 0.1)
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    prec = lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v)
    xo, io = fgmres.fgmres(lambda v: A @ v, prec, b, restart=restart, iters=k)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-8, restart=restart, maxit=k, flags=fdg.SOLVE_FIXED_ITERS)
    assert info["iterations"] == k and info["restarts"] == io["restarts"]
    assert relerr(x.cpu().numpy(), xo) <= 1e-8
    if k <= 20:  # above, both estimates sit at the rounding floor
        assert abs(info["rel_res_est"] - io["history"][-1]) <= 1e-6 * io["history"][-1]
    ctx.close()


@pytest.mark.parametrize("kind,p,n,restart,rtol", [("csr", 3, 12, 30, 1e-8), ("csr", 3, 10, 6, 1e-10),
                                                    ("csr", 2, 9, 3, 1e-9), ("mapped", 3, 12, 30, 1e-8),
                                                    ("mapped", 4, 9, 5, 1e-11)])
def test_steps_queued_ahead_change_nothing(kind, p, n, restart, rtol):
    # the single solve queues the next Arnoldi step before reading the current one; with
    # that turned off the iterates, counts and residuals are the same bits
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.deformed_problem(p, n, 0.1) if kind == "csr" else fdg.mapped_problem(p, n, 0.1)
    b = to_dev(inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3))
    xa = torch.empty_like(b)
    xs = torch.empty_like(b)
    ia = ctx.solve(b, xa, rtol=rtol, restart=restart)
    is_ = ctx.solve(b, xs, rtol=rtol, restart=restart, flags=fdg.SOLVE_NO_AHEAD)
    assert ia["converged"] and is_["converged"]
    assert (ia["iterations"], ia["restarts"]) == (is_["iterations"], is_["restarts"])
    assert ia["rel_res_true"] == is_["rel_res_true"] and ia["rel_res_est"] == is_["rel_res_est"]
    assert np.array_equal(xa.cpu().numpy(), xs.cpu().numpy())
    ctx.close()


def test_solve_use_x0_and_zero_rhs():
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 10
    ctx = fdg.deformed_problem(p, n, 0.1)
    b = inputs.rhs_uniform(9, n ** 3)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-10)
    assert info["converged"]
    # restarting from the converged solution needs no iteration
    info2 = ctx.solve(to_dev(b), x, rtol=1e-8, flags=fdg.SOLVE_USE_X0)
    assert info2["iterations"] == 0 and info2["converged"]
    z = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    info3 = ctx.solve(z, x, rtol=1e-8)
    assert info3["converged"] and info3["iterations"] == 0
    assert float(x.abs().max()) == 0.0
    ctx.close()


@pytest.mark.parametrize("p,n", [(4, 70), (3, 131), (6, 67)])
def test_true_residual_of_a_start_guess(p, n):
    """maxit = 0 from a start guess: the solve only forms r = b - A x0 (the one-pass
    matvec with the residual fused, its per-workgroup partials of |r|^2 summed on the
    host) over several tiles with ragged tails; the reported |r| / |b| against the
    oracle's product, and x0 left as it was."""
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(3, p, n)
    N = n ** 3
    b = inputs.rhs_normal(400, N)
    x0 = inputs.rhs_normal(401, N)
    x = to_dev(x0).clone()
    info = ctx.solve(to_dev(b), x, rtol=1e-8, maxit=0, flags=fdg.SOLVE_USE_X0)
    M, K, _, _ = colloc.colloc_factors(p, n)
    r = b - colloc.unit_matvec([M] * 3, [K] * 3, x0)
    ref = np.linalg.norm(r) / np.linalg.norm(b)
    assert info["iterations"] == 0 and not info["converged"]
    assert abs(info["rel_res_true"] - ref) <= 1e-13 * ref, (info["rel_res_true"], ref)
    assert np.array_equal(x.cpu().numpy(), x0)
    ctx.close()


def test_not_converged_status():
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 10
    ctx = fdg.deformed_problem(p, n, 0.1)
    b = inputs.rhs_uniform(9, n ** 3)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-12, restart=5, maxit=3)
    assert not info["converged"] and info["iterations"] == 3
    ctx.close()


@pytest.mark.parametrize("prec,bound", [(1, 2e-5), (2, 5e-2)])
def test_low_precision_apply_contraction(prec, bound):
    """P P~^{-1} b ~ b with the FP32 / BF16 preconditioner (one-apply contraction)."""
    fdg = _fdg()
    torch = torch_cuda()
    d, p, n = 3, 4, 40
    ctx = fdg.unit_problem(d, p, n, prec=prec)
    b = inputs.rhs_normal(5, n ** d)
    s = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    P, prec64 = oracle_unit(p, n, d)
    sg = s.cpu().numpy()
    contraction = relerr(P @ sg, b)
    assert contraction <= bound, contraction
    assert relerr(sg, prec64(b)) <= 50 * bound
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2])
def test_mixed_precision_solve_reaches_fp64_accuracy(prec):
    fdg = _fdg()
    torch = torch_cuda()
    d, p, n = 3, 6, 24
    ctx = fdg.unit_problem(d, p, n, prec=prec)
    b = inputs.rhs_normal(inputs.SEED_SWEEP_192, n ** d)
    x = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-10, restart=50)
    _, prec64 = oracle_unit(p, n, d)
    xref = prec64(b)
    assert info["converged"]
    assert info["iterations"] <= (3 if prec == 1 else 8)
    assert relerr(x.cpu().numpy(), xref) <= 1e-8
    ctx.close()


def test_errors_through_the_abi():
    fdg = _fdg()
    torch = torch_cuda()
    with pytest.raises(fdg.FdgError):
        fdg.Context(4, 10)
    ctx = fdg.Context(3, 8)
    v = torch.zeros(512, dtype=torch.float64, device="cuda")
    w = torch.zeros(512, dtype=torch.float64, device="cuda")
    with pytest.raises(fdg.FdgError) as ei:
        ctx.apply_prec(v, w)            # no factors yet
    assert ei.value.status == -5
    with pytest.raises(fdg.FdgError) as ei:
        ctx.set_operator_csr(np.array([0, 2, 1] + [1] * 510, dtype=np.int64), np.zeros(1, np.int32), np.zeros(1))
    assert ei.value.status == -1
    rowptr = np.arange(513, dtype=np.int64)
    with pytest.raises(fdg.FdgError):
        ctx.set_operator_csr(rowptr, np.full(512, 600, np.int32), np.ones(512))   # column out of range
    with pytest.raises(fdg.FdgError):
        ctx.set_precision(7)
    ctx.close()


@pytest.mark.parametrize("d,p,n,bound", [(3, 4, 40, 5e-2), (3, 3, 33, 5e-2), (3, 6, 65, 5e-2), (2, 4, 130, 5e-2),
                                         (2, 3, 47, 5e-2), (3, 5, 96, 5e-2), (3, 4, 129, 5e-2), (3, 3, 200, 5e-2),
                                         (2, 2, 260, 0.2)])
def test_bf16_apply_fused_passes(d, p, n, bound):
    """BF16 products with FP32 accumulation (fused passes for n <= 256, mode products
    beyond): the one-apply contraction |b - P P~^{-1} b| / |b| stays at the BF16 rounding
    level times the conditioning of P, which grows like n^2 (0.14 for the 2D p = 2, n = 260
    case, which takes the mode-product form)."""
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(d, p, n, prec=fdg.PREC_BF16)
    b = inputs.rhs_normal(7, n ** d)
    s = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    P, prec64 = oracle_unit(p, n, d)
    sg = s.cpu().numpy()
    assert np.all(np.isfinite(sg))
    assert relerr(P @ sg, b) <= bound
    assert relerr(sg, prec64(b)) <= 0.5
    ctx.close()


@pytest.mark.parametrize("d,p,n", [(3, 4, 40), (3, 3, 33), (3, 6, 65), (2, 4, 130), (2, 3, 47), (3, 5, 96),
                                   (3, 4, 129), (2, 2, 260)])
def test_fp32_apply_fused_passes(d, p, n):
    """FP32 factors and MFMA (fused passes for n <= 256, mode products beyond): the
    contraction |b - P P~^{-1} b| / |b| and the distance to the FP64 oracle stay at the
    FP32 rounding level."""
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(d, p, n, prec=fdg.PREC_FP32)
    b = inputs.rhs_normal(7, n ** d)
    s = torch.empty(n ** d, dtype=torch.float64, device="cuda")
    ctx.apply_prec(to_dev(b), s)
    torch.cuda.synchronize()
    P, prec64 = oracle_unit(p, n, d)
    sg = s.cpu().numpy()
    assert relerr(P @ sg, b) <= 5e-5
    assert relerr(sg, prec64(b)) <= 5e-4
    ctx.close()


def test_fp32_preconditioned_deformed_solve():
    """P != A: the FP32 preconditioner inside FGMRES reaches the FP64 true residual and
    the oracle's FP64 solution."""
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 12
    ctx = fdg.deformed_problem(p, n, 0.1, prec=fdg.PREC_FP32)
    b = inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3)
    A = colloc.deformed_operator(p, n, 0.1)
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    prec = lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v)
    x_ref, _ = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-13, restart=30)
    _, io = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-10, restart=30)
    x = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    info = ctx.solve(to_dev(b), x, rtol=1e-10, restart=30)
    assert info["converged"] and info["rel_res_true"] <= 1e-10
    assert abs(info["iterations"] - io["iterations"]) <= 2, (info["iterations"], io["iterations"])
    assert relerr(x.cpu().numpy(), x_ref) <= 1e-8
    ctx.close()


@pytest.mark.parametrize("d,n", [(3, 9), (2, 40)])
def test_csr_operator_general_and_tensor_patterns(d, n):
    """An assembled operator whose pattern is a product of per-direction windows is stored
    with implicit columns; any other pattern goes through the general ELL.  Both give the
    CSR product: a tensor-pattern matrix, the same with one entry removed (general), and
    a random pattern with empty rows (general)."""
    import scipy.sparse as sp
    fdg = _fdg()
    torch = torch_cuda()
    N = n ** d
    M, K, _, _ = colloc.colloc_factors(3, n)
    A = colloc.unit_operator([M] * d, [K] * d).tocsr()
    A.sort_indices()
    B = A.tolil()
    B[N // 2, A.indices[A.indptr[N // 2]]] = 0.0
    B = B.tocsr()
    B.eliminate_zeros()
    rng = np.random.default_rng(9)
    R = sp.random(N, N, density=8.0 / N, random_state=rng, format="csr")
    R = R.tolil()
    R[3, :] = 0.0
    R = R.tocsr()
    R.eliminate_zeros()
    R.sort_indices()
    x = inputs.rhs_normal(17, N)
    for S in (A, B, R):
        ctx = fdg.Context(d, n)
        ctx.set_operator_csr(S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data)
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        ctx.matvec(to_dev(x), y)
        torch.cuda.synchronize()
        assert relerr(y.cpu().numpy(), S @ x) <= 1e-14
        ctx.close()


def test_solve_time_split():
    """FDG_SOLVE_TIME_SPLIT fills the device time of the applies, matvecs and vector
    kernels (kernel timers), and the host time is always set; the iterate is the same bits
    as without the split, and the caller's timer states are restored."""
    fdg = _fdg()
    torch = torch_cuda()
    p, n = 3, 12
    ctx = fdg.deformed_problem(p, n, 0.1)
    b = to_dev(inputs.rhs_uniform(inputs.SEED_DEFORMED_96, n ** 3))
    x1 = torch.empty_like(b)
    x2 = torch.empty_like(b)
    i1 = ctx.solve(b, x1, rtol=1e-8, restart=30)
    i2 = ctx.solve(b, x2, rtol=1e-8, restart=30, flags=fdg.SOLVE_TIME_SPLIT)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]
    assert i1["t_apply_ms"] == 0.0 and i1["t_matvec_ms"] == 0.0 and i1["t_orth_ms"] == 0.0
    assert i1["t_host_ms"] > 0.0 and i2["t_host_ms"] > 0.0
    assert i2["t_apply_ms"] > 0.0 and i2["t_matvec_ms"] > 0.0 and i2["t_orth_ms"] > 0.0
    assert i2["t_apply_ms"] + i2["t_matvec_ms"] + i2["t_orth_ms"] < i2["ms_total"]
    # timers were off before, so nothing is recorded by a later solve
    ctx.solve(b, x1, rtol=1e-8, restart=30)
    assert ctx.timer_read(fdg.TIMER_APPLY) == (0, 0.0)
    ctx.close()
