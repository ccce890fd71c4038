"""Continuous-batching server for scattering requests.

Requests (a scatterer, a wavenumber, incident directions, a boundary condition)
arrive over time.  Each request is admitted when a slot is free and its device
memory -- from the operator's size model, computed by a host-only plan before
anything is allocated -- fits the remaining HBM budget.  Admitted requests run
concurrently, one HIP stream per slot: geometry, operator assembly, the
lockstep multi-direction CFIE solve (mixed precision with fp64 refinement) and
the far field.  Waiting requests for the same scattering problem (star, level,
wavenumber, boundary condition) join the admitted one as further columns of
its lockstep block: one operator, one block matvec per Arnoldi step.  A
request's result depends only on the request: every reduction in the library
has a fixed order, slots share no state and each column of a block keeps its
own Krylov basis, so a request gives the same far field alone and in the mix
(bitwise when it runs alone in its slot; within the solver's tolerance when
its block shares columns with another request).

All numerical work runs in the HIP library; this module schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time

import numpy as np

from . import binding as B
from . import inputs as I


@dataclasses.dataclass
class ServeConfig:
    slots: int = 4
    hbm_budget: int = 200 * 10 ** 9
    precision: int = B.MIX_BF16          # sound-soft requests
    precision_hard: int = B.MIX_BF16     # sound-hard requests
    p: int = 2
    q: int = 8
    eta_adm: float = 1.6
    # cap on kappa * diameter of interpolated clusters (0: the paper's rule alone).
    # Without it a block at high kappa may span several wavelengths and its
    # interpolation error, not the solver tolerance, bounds the result's accuracy
    kcap: float = 0.0
    leaf_depth: int = 2
    # one Gauss point per direction fewer than the library default in the near
    # field: entries ~1e-9 relative (hard ~1e-8), far below the H2 compression
    # error at q = 8, for ~30% less assembly time
    quad_extra: int = -1
    tol: float = 1e-8
    nobs: int = 64
    device: int = 0
    # GMRES restart (the paper's 30 for both systems)
    restart_soft: int = 30
    restart_hard: int = 30
    maxit: int = 1500        # Arnoldi steps per direction; a request that reaches it is reported unconverged
    # requests for the same scattering problem (star, level, wavenumber, boundary
    # condition) that wait together are solved as one lockstep block of up to
    # merge_max_dirs directions on one operator (0: every request alone)
    merge_max_dirs: int = 64
    # autotuned operator shapes (leaf depth, stored / on-the-fly couplings) per request class;
    # classes without an entry use leaf_depth and stored couplings
    tune_cache: object = None


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    done: float
    n: int
    est_bytes: int
    iters: int
    matvecs: int
    relres_true: float
    converged: int
    escalated: int        # directions finished on the fp64 operator
    uinf: np.ndarray      # (ndir, nobs)
    stages: dict = dataclasses.field(default_factory=dict)   # seconds per stage
    batch: tuple = ()     # ids of the requests solved in the same block (this one first)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def problem_key(req: I.Request):
    """Requests with equal keys have the same operator."""
    return (req.seed, req.m, req.kappa, req.bc)


def percentile(values, pct):
    """Nearest-rank percentile."""
    v = np.sort(np.asarray(values, dtype=float))
    if len(v) == 0:
        return float("nan")
    k = max(1, int(np.ceil(pct / 100.0 * len(v))))
    return float(v[k - 1])


class Server:
    """`solve_fn(req, slot)` and `estimate_fn(req)` replace the device work and
    the size model (used to test the scheduler without a GPU)."""

    def __init__(self, cfg: ServeConfig | None = None, solve_fn=None, estimate_fn=None):
        self.cfg = cfg or ServeConfig()
        self.obs = I.fibonacci_directions(self.cfg.nobs)
        self.solve_fn = solve_fn
        self.estimate_fn = estimate_fn
        self.plan_ctx = B.Context(B.IGB_HOST_ONLY) if estimate_fn is None else None
        self.ctxs = None
        if solve_fn is None:
            import torch
            torch.cuda.init()      # initialise the runtime once, before worker threads use it
            self.ctxs = [B.Context(self.cfg.device) for _ in range(self.cfg.slots)]
        self.peak_reserved = 0

    # -------------------------------------------------------------- pieces
    def _patches(self, req: I.Request):
        return I.star_patches(req.seed, I.star_geometry_level(req.m))

    def _op_args(self, req: I.Request):
        c = self.cfg
        bc = B.SOFT if req.bc == "soft" else B.HARD
        prec = c.precision if req.bc == "soft" else c.precision_hard
        args = dict(kappa=req.kappa, bc=bc, q=c.q, eta_adm=c.eta_adm, kcap=c.kcap, leaf_depth=c.leaf_depth,
                    precision=prec, quad_extra=c.quad_extra)
        if c.tune_cache is not None:
            from . import autotune as T
            ch = c.tune_cache.get(T.TuneKey(T.device_arch(), req.m, c.p, c.q, bc, prec,
                                            round(math.log2(req.kappa)), T.nrhs_bucket(len(req.dirs))))
            if ch is not None:
                args.update(leaf_depth=ch.leaf_depth, far_on_the_fly=ch.far_on_the_fly,
                            recompress_tol=ch.recompress_tol)
        return args

    def estimate(self, req: I.Request) -> int:
        """Device bytes of the request (host-only plan: nothing is allocated)."""
        geo = B.Geometry(self.plan_ctx, self._patches(req), req.m, self.cfg.p)
        op = B.Operator(self.plan_ctx, geo, **self._op_args(req))
        nd = len(req.dirs)
        geom_bytes = geo.nelem * (16 * 4 * 8 + 8) + 4096
        restart = self.cfg.restart_soft if req.bc == "soft" else self.cfg.restart_hard
        # the library's size model of the operator after an nd-direction solve and
        # its far field (data, matvec work vectors, Krylov bases, refinement and
        # quadrature buffers), plus the caller's coefficient and far-field arrays
        return int(op.solve_bytes(nd, restart) + geom_bytes + nd * (op.n + self.cfg.nobs) * 16 + (1 << 20))

    def solve(self, req: I.Request, ctx: B.Context):
        """Returns (n, solve info, far field [ndir][nobs], stage seconds)."""
        import torch
        t0 = time.perf_counter()
        geo = B.Geometry(ctx, self._patches(req), req.m, self.cfg.p)
        t1 = time.perf_counter()
        op = B.Operator(ctx, geo, **self._op_args(req))
        t2 = time.perf_counter()
        nd = len(req.dirs)
        dev = torch.device("cuda", self.cfg.device)
        coeff = torch.empty((nd, op.n), dtype=torch.complex128, device=dev)
        uinf = torch.empty((nd, self.cfg.nobs), dtype=torch.complex128, device=dev)
        restart = self.cfg.restart_soft if req.bc == "soft" else self.cfg.restart_hard
        info, st = op.cfie_solve(req.dirs, coeff, tol=self.cfg.tol, restart=restart, maxit=self.cfg.maxit)
        t3 = time.perf_counter()
        op.farfield(coeff, self.obs, uinf, ndir=nd, stream=B.CONTEXT_STREAM)
        u = uinf.cpu().numpy()
        t4 = time.perf_counter()
        oi = op.info
        stages = {"geometry": t1 - t0, "assembly": t2 - t1, "assembly_near_gpu": oi.assembly_near_ms * 1e-3,
                  "assembly_far_gpu": oi.assembly_far_ms * 1e-3, "solve": t3 - t2, "farfield": t4 - t3}
        n = op.n
        del op, geo, coeff, uinf
        return n, info, u, stages

    # -------------------------------------------------------------- serving
    def run(self, requests, realtime: bool = True, log=None):
        """Serve `requests` (sorted by arrival).  With realtime, a request
        becomes visible at its arrival time; otherwise all are visible at once.
        `log(result)` is called as each request completes.  Returns the
        results in request order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        estimate = self.estimate_fn or self.estimate
        est = {r.rid: estimate(r) for r in reqs}
        for r in reqs:
            if est[r.rid] > self.cfg.hbm_budget:
                raise ValueError(f"request {r.rid} needs {est[r.rid]} bytes, more than the whole budget")
        lock = threading.Condition()
        pending = collections.deque()
        results = {}
        state = {"free": self.cfg.hbm_budget, "arrived": 0, "errors": []}
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        def feeder():
            for r in reqs:
                if realtime:
                    dt = r.arrival - now()
                    if dt > 0:
                        time.sleep(dt)
                with lock:
                    pending.append(r)
                    state["arrived"] += 1
                    lock.notify_all()

        def worker(slot):
            while True:
                with lock:
                    while True:
                        pick = None
                        for r in pending:                      # oldest request that fits
                            if est[r.rid] <= state["free"]:
                                pick = r
                                break
                        if pick is not None:
                            pending.remove(pick)
                            state["free"] -= est[pick.rid]
                            # waiting requests for the same problem join the block
                            # (each reserves its own estimate: an upper bound)
                            batch, ndir = [pick], len(pick.dirs)
                            for r in list(pending):
                                if (problem_key(r) == problem_key(pick)
                                        and ndir + len(r.dirs) <= self.cfg.merge_max_dirs
                                        and est[r.rid] <= state["free"]):
                                    pending.remove(r)
                                    state["free"] -= est[r.rid]
                                    batch.append(r)
                                    ndir += len(r.dirs)
                            self.peak_reserved = max(self.peak_reserved, self.cfg.hbm_budget - state["free"])
                            break
                        if state["arrived"] == len(reqs) and not pending:
                            return
                        lock.wait(0.05)
                admitted = now()
                job = pick if len(batch) == 1 else dataclasses.replace(
                    pick, dirs=np.concatenate([r.dirs for r in batch]))
                reserved = sum(est[r.rid] for r in batch)
                try:
                    if self.solve_fn is not None:
                        n, info, u, *rest = self.solve_fn(job, slot)
                    else:
                        n, info, u, *rest = self.solve(job, self.ctxs[slot])
                except Exception as exc:  # recorded, the stream continues
                    with lock:
                        state["errors"].extend((r.rid, repr(exc)) for r in batch)
                        state["free"] += reserved
                        lock.notify_all()
                    continue
                done = now()
                # the block's far field split back by request; the solve's counts
                # are the block's (unconverged columns are not attributed, so a
                # request counts as converged only when the whole block is)
                ids, off, out = tuple(r.rid for r in batch), 0, []
                total = len(job.dirs)
                for r in batch:
                    nd = len(r.dirs)
                    conv = nd if info.converged == total else max(0, info.converged - (total - nd))
                    out.append(Result(r.rid, r.arrival, admitted, done, n, est[r.rid], info.iters,
                                      info.matvecs * nd // total,
                                      info.relres_true, conv, getattr(info, "escalated", 0), u[off:off + nd],
                                      rest[0] if rest else {}, (r.rid,) + tuple(i for i in ids if i != r.rid)))
                    off += nd
                with lock:
                    for res in out:
                        results[res.rid] = res
                    state["free"] += reserved
                    lock.notify_all()
                if log is not None:
                    for res in out:
                        log(res)

        threads = [threading.Thread(target=feeder, daemon=True)]
        threads += [threading.Thread(target=worker, args=(i,), daemon=True) for i in range(self.cfg.slots)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        if state["errors"]:
            raise RuntimeError(f"requests failed: {state['errors']}")
        self.wall = now()
        return [results[r.rid] for r in sorted(reqs, key=lambda r: r.rid)]

    @staticmethod
    def summary(results, wall):
        lat = [r.latency for r in results]
        cols = sum(r.uinf.shape[0] for r in results)
        return {"requests": len(results), "wall_s": wall, "requests_per_s": len(results) / wall,
                "direction_solves_per_s": cols / wall, "column_matvecs_per_s": sum(r.matvecs for r in results) / wall,
                "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
                "max_relres_true": max(r.relres_true for r in results),
                "escalated_directions": sum(r.escalated for r in results),
                "merged_requests": sum(1 for r in results if len(r.batch) > 1),
                "all_converged": all(r.converged == r.uinf.shape[0] for r in results)}
