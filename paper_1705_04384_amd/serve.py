"""Request scheduling over the native server (fdg_server_*): arrival process, factor
cache, admission by device-memory footprint and latency bookkeeping.

The device work and the per-request FGMRES host arithmetic run in the library; this
module only decides *when* a request enters the server:

- Host setup of a request's 1D factors (collocation matrices, generalized eigenproblem
  of eq. 4.6) depends on (p, n) only; it runs in a thread pool (the library releases
  the GIL) the first time a (p, n) arrives, and its device context (d, p, n) is created
  once and kept; the contexts share one blocking-solve workspace.
- Requests are admitted first come, first served among those whose context is ready;
  a request enters when the server has a free slot and arena space for its Krylov
  bases (its footprint), otherwise it and everything behind it wait.
- Latency is measured from arrival to the completion returned by the server, with the
  right-hand sides already resident in device memory.
"""
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import fdgmres, inputs


def _factors(p, n):
    M, K, _, _ = fdgmres.colloc_factors(p, n)
    U, V, lam, _ = fdgmres.factor_pencil(K, M, want_cond=False)
    return M, K, U, V, lam


class FactorCache:
    """(p, n) -> host factors (thread pool); (d, p, n) -> device context.

    The contexts carve their blocking-solve workspace ((2m + 3) N doubles and partials) from
    one shared device buffer sized for the largest of them: the blocking solves run one
    at a time and each returns with its stream drained, so the cache holds one workspace
    instead of one per shape.  Served requests do not use it: their bases live in the
    server's arena, which admission by footprint bounds."""

    def __init__(self, threads=8, restart=30, device="cuda"):
        self.pool = ThreadPoolExecutor(max_workers=threads)
        self.futs = {}
        self.ctxs = {}
        self.restart = restart
        self.device = device
        self.ws_buf = None
        self.ws_grows = 0

    def request(self, p, n):
        if (p, n) not in self.futs:
            self.futs[(p, n)] = self.pool.submit(_factors, p, n)

    def attach(self, key, ctx):
        """Adds a context, attached to the shared workspace (grown, and every context
        re-attached, when this one needs more)."""
        need = fdgmres.workspace_bytes(ctx.d, ctx.n, ctx.batch, self.restart)
        if self.ws_buf is None or self.ws_buf.numel() < need:
            import torch
            buf = torch.empty(need, dtype=torch.uint8, device=self.device)
            for c in self.ctxs.values():
                c.attach_workspace(buf, self.restart)
            self.ws_buf = buf
            self.ws_grows += 1
        ctx.attach_workspace(self.ws_buf, self.restart)
        self.ctxs[key] = ctx

    def context(self, d, p, n):
        """The device context, or None while its factors are still being computed."""
        c = self.ctxs.get((d, p, n))
        if c is not None:
            return c
        f = self.futs.get((p, n))
        if f is None:
            self.request(p, n)
            return None
        if not f.done():
            return None
        M, K, U, V, lam = f.result()
        c = fdgmres.unit_context(d, n, M, K, U, V, lam)
        self.attach((d, p, n), c)
        return c

    def held_bytes(self):
        """Device bytes of the cache: what the contexts own (factors, operator bands) and
        the shared workspace."""
        own = sum(c.device_bytes()[0] for c in self.ctxs.values())
        return own + (0 if self.ws_buf is None else self.ws_buf.numel())

    def warm(self, reqs):
        for r in reqs:
            self.request(r["p"], r["n"])
        for r in reqs:
            self.futs[(r["p"], r["n"])].result()
            self.context(r["d"], r["p"], r["n"])

    def close(self):
        self.pool.shutdown(wait=True)
        for c in self.ctxs.values():
            c.close()
        self.ctxs.clear()
        self.ws_buf = None


def stage(reqs, device="cuda"):
    """Right-hand sides (N(0,1), seed of each request) and solution buffers in device memory."""
    import torch
    bufs = {}
    for r in reqs:
        N = r["n"] ** r["d"]
        b = torch.from_numpy(inputs.rhs_normal(r["seed"], N)).to(device)
        bufs[r["id"]] = (b, torch.empty_like(b))
    torch.cuda.synchronize()
    return bufs


def run_served(server, cache, reqs, bufs, rtol=1e-8, maxit=1000, time_scale=1.0):
    """Replays the arrival times of reqs (seconds, times time_scale) through the server.

    Returns {id: (latency_s, status, info)} and the makespan in seconds."""
    order = sorted(reqs, key=lambda r: r["t"])
    by_id = {r["id"]: r for r in order}
    queue = deque()
    out = {}
    i = 0
    t0 = time.perf_counter()
    while len(out) < len(order):
        now = time.perf_counter() - t0
        while i < len(order) and order[i]["t"] * time_scale <= now:
            cache.request(order[i]["p"], order[i]["n"])
            queue.append(order[i])
            i += 1
        # FCFS among requests whose context is ready; stop at the first that does not fit
        blocked = False
        for r in list(queue):
            ctx = cache.context(r["d"], r["p"], r["n"])
            if ctx is None:
                continue
            b, x = bufs[r["id"]]
            if not server.admit(ctx, b, x, rtol=rtol, maxit=maxit, tag=r["id"]):
                blocked = True
                break
            queue.remove(r)
        wait_us = 0
        if i < len(order) and not blocked:
            wait_us = int(max(0.0, min(200e-6, order[i]["t"] * time_scale - now)) * 1e6)
        elif blocked or not queue:
            wait_us = 200
        for tag, st, info in server.step(wait_us):
            r = by_id[tag]
            out[tag] = (time.perf_counter() - t0 - r["t"] * time_scale, st, info)
    return out, time.perf_counter() - t0


def run_one_by_one(cache, reqs, bufs, rtol=1e-8, restart=None, maxit=1000, time_scale=1.0):
    """The same arrival stream solved one request at a time with the blocking fdg_solve
    (a request starts when it has arrived and the previous one has finished); restart
    defaults to the one the cache's shared workspace is sized for."""
    restart = cache.restart if restart is None else restart
    order = sorted(reqs, key=lambda r: r["t"])
    out = {}
    t0 = time.perf_counter()
    for r in order:
        ctx = cache.context(r["d"], r["p"], r["n"])
        while ctx is None:
            time.sleep(1e-4)
            ctx = cache.context(r["d"], r["p"], r["n"])
        while time.perf_counter() - t0 < r["t"] * time_scale:
            pass
        b, x = bufs[r["id"]]
        info = ctx.solve(b, x, rtol=rtol, restart=restart, maxit=maxit)
        out[r["id"]] = (time.perf_counter() - t0 - r["t"] * time_scale, 0 if info["converged"] else 1, info)
    return out, time.perf_counter() - t0


def summarize(results, makespan):
    lat = np.array([v[0] for v in results.values()]) * 1e3
    conv = sum(1 for v in results.values() if v[2]["converged"])
    return {
        "requests": len(results),
        "converged": conv,
        "solves_per_s": len(results) / makespan,
        "makespan_s": makespan,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(lat.mean()),
    }
