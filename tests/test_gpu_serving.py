"""GPU: the request server (continuous batching) through the C ABI.

Each served request must give bit-for-bit the blocking single-solve result for the same
context and right-hand side, whatever it is mixed with (same-context requests are
grouped into shared launches at different Arnoldi indices; different shapes run on
other lanes), and the solve must match the FP64 oracle as the single solve does.
"""
import numpy as np
import pytest

from oracle import colloc, fd, fgmres
from paper_1705_04384_amd import inputs
from tests.gpu_helpers import oracle_unit, relerr, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _fdg():
    torch_cuda()
    from paper_1705_04384_amd import fdgmres
    fdgmres.lib()
    return fdgmres


def _drain(srv, results, limit_steps=200000):
    steps = 0
    while srv.pending() > 0:
        for tag, st, info in srv.step(wait_us=1000):
            results[tag] = (st, info)
        steps += 1
        assert steps < limit_steps, "server made no progress"


def _solo(ctx, b, restart, rtol=1e-8, maxit=1000):
    torch = torch_cuda()
    x = torch.empty_like(b)
    info = ctx.solve(b, x, rtol=rtol, restart=restart, maxit=maxit)
    return x.cpu().numpy(), info


def test_served_mix_is_bitwise_identical_to_solo():
    fdg = _fdg()
    torch = torch_cuda()
    restart = 8
    ctxs = [fdg.deformed_problem(3, 10, 0.1), fdg.deformed_problem(2, 9, 0.1),
            fdg.unit_problem(3, 4, 20), fdg.unit_problem(2, 3, 45), fdg.unit_problem(3, 2, 17)]
    reqs = []
    k = 0
    for ci, ctx in enumerate(ctxs):
        for r in range(4 if ci < 2 else 2):
            b = to_dev(inputs.rhs_uniform(500 + k, ctx.N))
            reqs.append((k, ci, b, torch.full_like(b, np.nan)))
            k += 1
    srv = fdg.Server(max_slots=32, restart=restart, lanes=2, arena_bytes=256 << 20)
    results = {}
    # staggered admission: the second half enters while the first is mid-iteration
    half = len(reqs) // 2
    for tag, ci, b, x in reqs[:half]:
        assert srv.admit(ctxs[ci], b, x, rtol=1e-8, tag=tag)
    for _ in range(3):
        for tag, st, info in srv.step(wait_us=2000):
            results[tag] = (st, info)
    for tag, ci, b, x in reqs[half:]:
        assert srv.admit(ctxs[ci], b, x, rtol=1e-8, tag=tag)
    _drain(srv, results)
    torch.cuda.synchronize()
    stats = srv.stats()
    assert stats["max_group"] >= 2, stats
    assert len(results) == len(reqs)
    for tag, ci, b, x in reqs:
        st, info = results[tag]
        xs, info_s = _solo(ctxs[ci], b, restart)
        assert st == 0 and info["converged"] == 1
        assert info["iterations"] == info_s["iterations"], (tag, info, info_s)
        assert info["restarts"] == info_s["restarts"]
        assert info["rel_res_true"] == info_s["rel_res_true"]
        xg = x.cpu().numpy()
        assert np.array_equal(xg, xs), (tag, relerr(xg, xs))
    srv.close()
    for c in ctxs:
        c.close()


def test_served_deformed_matches_oracle():
    fdg = _fdg()
    torch = torch_cuda()
    p, n, restart = 3, 10, 6
    ctx = fdg.deformed_problem(p, n, 0.1)
    A = colloc.deformed_operator(p, n, 0.1)
    M, K, _, _ = colloc.colloc_factors(p, n)
    U, V, lam = fd.factor_pencil(K, M)
    prec = lambda v: fd.fd_apply([U] * 3, [V] * 3, [lam] * 3, v)
    srv = fdg.Server(max_slots=8, restart=restart, lanes=1, arena_bytes=64 << 20)
    bs = [inputs.rhs_uniform(700 + k, n ** 3) for k in range(3)]
    xs = []
    for k, b in enumerate(bs):
        bd = to_dev(b)
        x = torch.empty_like(bd)
        xs.append((bd, x))
        assert srv.admit(ctx, bd, x, rtol=1e-8, tag=k)
    results = {}
    _drain(srv, results)
    for k, b in enumerate(bs):
        xo, io = fgmres.fgmres(lambda v: A @ v, prec, b, rtol=1e-8, restart=restart)
        st, info = results[k]
        assert info["converged"] and io["converged"]
        assert info["iterations"] == io["iterations"]
        assert relerr(xs[k][1].cpu().numpy(), xo) <= 1e-8
    srv.close()
    ctx.close()


def test_admission_by_footprint_and_slots():
    fdg = _fdg()
    torch = torch_cuda()
    ctx = fdg.unit_problem(3, 3, 24)
    per = fdg.Server(max_slots=1, restart=4, lanes=1, arena_bytes=1 << 20).run_bytes(ctx)
    srv = fdg.Server(max_slots=4, restart=4, lanes=1, arena_bytes=2 * per + 1024)
    bs = [to_dev(inputs.rhs_normal(800 + k, ctx.N)) for k in range(3)]
    xs = [torch.empty_like(b) for b in bs]
    assert srv.admit(ctx, bs[0], xs[0], tag=0)
    assert srv.admit(ctx, bs[1], xs[1], tag=1)
    assert not srv.admit(ctx, bs[2], xs[2], tag=2)   # arena holds two requests
    results = {}
    _drain(srv, results)
    assert srv.admit(ctx, bs[2], xs[2], tag=2)       # space returned on completion
    _drain(srv, results)
    _, prec = oracle_unit(3, 24, 3)
    for k in range(3):
        assert results[k][0] == 0
        assert relerr(xs[k].cpu().numpy(), prec(bs[k].cpu().numpy())) <= 1e-10
    one = fdg.Server(max_slots=1, restart=4, lanes=1, arena_bytes=64 << 20)
    assert one.admit(ctx, bs[0], xs[0], tag=0)
    assert not one.admit(ctx, bs[1], xs[1], tag=1)   # no free slot
    _drain(one, results)
    one.close()
    srv.close()
    ctx.close()


def test_served_low_precision_and_zero_rhs():
    fdg = _fdg()
    torch = torch_cuda()
    ctx32 = fdg.unit_problem(3, 6, 24, prec=fdg.PREC_FP32)
    ctx64 = fdg.unit_problem(2, 4, 33)
    srv = fdg.Server(max_slots=8, restart=20, lanes=2, arena_bytes=128 << 20)
    b32 = to_dev(inputs.rhs_normal(900, ctx32.N))
    x32 = torch.empty_like(b32)
    z = torch.zeros(ctx64.N, dtype=torch.float64, device="cuda")
    xz = torch.full_like(z, 3.0)
    assert srv.admit(ctx32, b32, x32, rtol=1e-10, tag=0)
    assert srv.admit(ctx64, z, xz, rtol=1e-8, tag=1)
    results = {}
    _drain(srv, results)
    xs, info_s = _solo(ctx32, b32, 20, rtol=1e-10)
    assert results[0][1]["iterations"] == info_s["iterations"]
    assert np.array_equal(x32.cpu().numpy(), xs)
    assert results[1][1]["converged"] and results[1][1]["iterations"] == 0
    assert float(xz.abs().max()) == 0.0
    srv.close()
    ctx32.close()
    ctx64.close()
