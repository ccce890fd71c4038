"""Autotuner over the operator's shape: the leaf depth d (cluster size, hence
how the work splits between the near field and the coupling tiles, and how
many tiles there are), stored versus on-the-fly fp64 couplings, and stored
tiles versus tiles recompressed to low-rank factors at a given tolerance,
measured on the device for a workload class and cached per class.

Every candidate keeps the admissibility rule and the interpolation degree, so
the interpolation error bound is the same (a recompression tolerance adds its
own relative error per tile, far below it at 1e-8); only time and memory are
traded.  The cost of a candidate is its assembly time plus an expected number
of block matvecs at the class's column count (a served request assembles once
and applies the operator a few hundred times).  Timing is wall time around
synchronised launches; nothing here computes any part of the method.
"""
from __future__ import annotations

import dataclasses
import json
import math
import os
import time

from . import binding as B


def nrhs_bucket(ncol: int) -> int:
    """Column counts tuned together: 1, 2-4, 5-8, 9-16, 17-32, ..."""
    return 1 if ncol <= 1 else 1 << max(2, math.ceil(math.log2(ncol)))


@dataclasses.dataclass(frozen=True)
class TuneKey:
    arch: str
    m: int
    p: int
    q: int
    bc: int
    precision: int
    kappa_band: int     # round(log2 kappa)
    nrhs: int           # nrhs_bucket(column count)

    def as_str(self) -> str:
        return "/".join(str(v) for v in dataclasses.astuple(self))


@dataclasses.dataclass
class Choice:
    leaf_depth: int
    far_on_the_fly: bool
    matvec_ms: float
    assembly_ms: float
    device_bytes: int
    recompress_tol: float = 0.0
    far_pairs: int = -1


class TuneCache:
    """Choices per TuneKey, optionally persisted as JSON."""

    def __init__(self, path: str | None = None):
        self.path = path
        self.table: dict[str, Choice] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                for k, v in json.load(f).items():
                    self.table[k] = Choice(**v)

    def get(self, key: TuneKey) -> Choice | None:
        return self.table.get(key.as_str())

    def put(self, key: TuneKey, choice: Choice) -> None:
        self.table[key.as_str()] = choice
        if self.path:
            with open(self.path, "w") as f:
                json.dump({k: dataclasses.asdict(v) for k, v in self.table.items()}, f, indent=1)


def device_arch() -> str:
    import torch
    return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gfx").split(":")[0]


def measure(ctx, geo, ncol: int, reps: int = 5, **op_args) -> Choice | None:
    """Assembles one candidate and times its block matvec of ncol columns
    (reduced-precision operators: the inner matvec of the refinement).  None if
    the candidate does not fit the context's budget or is not supported."""
    import torch
    from . import inputs as I
    t0 = time.perf_counter()
    try:
        op = B.Operator(ctx, geo, **op_args)
    except B.IgbError:
        return None
    torch.cuda.synchronize()
    t_asm = (time.perf_counter() - t0) * 1e3
    x = torch.from_numpy(I.random_complex(4321, (ncol, op.n))).cuda()
    y = torch.zeros_like(x)
    parts = B.PART_ALL | (0 if op_args.get("precision", B.FP64) == B.FP64 else B.MV_LOWPREC)
    op.h2_matvec(x, y, nrhs=ncol, parts=parts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        op.h2_matvec(x, y, nrhs=ncol, parts=parts)
    torch.cuda.synchronize()
    t_mv = (time.perf_counter() - t0) / reps * 1e3
    ch = Choice(op_args.get("leaf_depth", 2), bool(op_args.get("far_on_the_fly", False)), t_mv, t_asm,
                op.info.device_bytes, float(op_args.get("recompress_tol", 0.0)), int(op.info.far_pairs))
    del op
    torch.cuda.empty_cache()
    return ch


def tune(ctx, geo, m: int, p: int, ncol: int, kappa: float, bc: int = B.SOFT, q: int = 8,
         precision: int = B.FP64, eta_adm: float = 1.6, quad_extra: int = 0, matvecs: int = 200,
         leaf_depths=(1, 2, 3, 4), on_the_fly=(False, True), recompress_tols=(0.0,),
         cache: TuneCache | None = None, reps: int = 5, require_far: bool = False):
    """Best (leaf depth, stored / on-the-fly, recompression tolerance) for the
    class of this operator; returns (choice, [every measured candidate]).  A
    cached choice is returned without measuring.  Recompression applies to
    stored fp64 tiles only (on-the-fly and reduced-precision candidates take
    tolerance 0).  With require_far, candidates without admissible blocks (a
    leaf depth so coarse that the whole operator is near field, i.e. dense)
    are measured and listed but not chosen."""
    key = TuneKey(device_arch(), m, p, q, bc, precision, round(math.log2(kappa)), nrhs_bucket(ncol))
    if cache is not None and cache.get(key) is not None:
        return cache.get(key), []
    measured = []
    for d in leaf_depths:
        if d > m:
            continue
        for otf in on_the_fly:
            tols = (0.0,) if otf or precision != B.FP64 else recompress_tols
            for rt in tols:
                ch = measure(ctx, geo, ncol, reps, kappa=kappa, bc=bc, q=q, eta_adm=eta_adm, leaf_depth=d,
                             precision=precision, far_on_the_fly=otf, quad_extra=quad_extra, recompress_tol=rt)
                if ch is not None:
                    measured.append(ch)
    eligible = [c for c in measured if c.far_pairs != 0] if require_far else measured
    if not eligible:
        raise RuntimeError("autotune: no candidate could be assembled")
    best = min(eligible, key=lambda c: (c.assembly_ms + matvecs * c.matvec_ms, c.device_bytes))
    if cache is not None:
        cache.put(key, best)
    return best, measured


def tune_tile_shape(op, ncol: int, reps: int = 10, parts: int | None = None):
    """Kernel tile shapes of an fp64 operator's block product of ncol columns:
    each (coupling, near) pair of column tiles per workgroup in {1, 2, 4}
    that divides the block's 16-column tile count is set on the operator
    (igb_op_set_tile_shape) and its block matvec timed; the fastest is left
    set.  The shapes do not change any result.  Returns (choice, [(coupling,
    near, ms)])."""
    import torch
    from . import inputs as I
    ntile = (ncol + 15) // 16
    shapes = [c for c in (1, 2, 4) if ntile % c == 0]
    x = torch.from_numpy(I.random_complex(4322, (ncol, op.n))).cuda()
    y = torch.zeros_like(x)
    parts = B.PART_ALL if parts is None else parts
    measured = []
    for cc in shapes:
        for nc in shapes:
            op.set_tile_shape(cc, nc)
            op.h2_matvec(x, y, nrhs=ncol, parts=parts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                op.h2_matvec(x, y, nrhs=ncol, parts=parts)
            torch.cuda.synchronize()
            measured.append((cc, nc, (time.perf_counter() - t0) / reps * 1e3))
    best = min(measured, key=lambda t: t[2])
    op.set_tile_shape(best[0], best[1])
    return best, measured
