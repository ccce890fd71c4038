"""Benchmark: H^2 CFIE matvecs/s on one MI355X.

Workload (default): the unit sphere as six rational-quadratic patches, level
m = 5 (6144 elements), degree-2 B-splines (N = 6936), kappa = 8, sound-soft
CFIE, interpolation degree q = 6, admissibility eta = 1.6, leaf depth 2, fp64,
one incident plane wave d = (0,0,1), GMRES(30) to 1e-8.  The fp64 coupling
tiles are recompressed (pivoted QR, each tile to 1e-8 relative in Frobenius
norm) and the one-column products stream the factors; the error against the
oracle rows is that of the tiles, and the tiles themselves are timed beside it.

One timed step = one CFIE solve on the assembled operator (right-hand side,
restarted GMRES with one H^2 matvec plus CGS2 Arnoldi per iteration, final
residual check) followed by the far field at 64 directions.  `value` counts
every operator application inside the timed steps.  Operator assembly (near
field quadrature + coupling matrices) is timed separately and reported.

Beside the headline line's value: the served forms (16 directions in lockstep
with fp64, fp32 or bf16 couplings; the reduced precisions run on the matrix
cores inside fp64 iterative refinement), each block matvec's kernel times and
roofline, a continuous-batching request stream with p50/p99 latency, the same
solves with one H^2 matrix per operator (`paper_mode`) and streaming the
uncompressed tiles or factors truncated at 1e-7 (`recompressed`), and the
scattered field at points off the
boundary by direct summation and by the H^2 evaluation (`potential`).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
                    [--block 16] [--serve 32] [--serve-rate 1.0]

`--convergence` instead runs the convergence benchmark of Sec. 5.2 (torus,
kappa = 2.5, incidence along x, scattered field at 100 points on the radius-5
sphere; soft p = 0..3, hard p = 1..3, m = 0..--conv-mmax) and prints one JSON
line per solve and a final one with the l-infinity errors against the finest,
highest-degree solution of each boundary condition (or, with
`--conv-reference single_layer`, the single-layer solution) and the observed
orders.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H2 matvecs/s and CFIE solves/s vs plain FP64 at 1e-6 rel err; p50/p99 latency"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the matvec kernels on the sphere_m5_p2_k8 workload,
# keyed by (kernel or block form, leaf depth), from two rocprofv3 passes over
# `bench.py --kernels-only` (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0; the factors
# make a plain 1 GiB device copy read and write 1 GiB), taken for the kernels
# as they stand: profiles/matvec_kernels_sphere_m5_p2_k8_counters.md.  An
# entry is removed whenever its kernel changes.
MEASURED_TRAFFIC = {("spmv_groups<16>", 3): 398.1e6, ("m2l_chunks_lowrank", 3): 148.1e6,
                    ("fp64 16col", 3): 226.0e6, ("fp64 64col", 3): 554.4e6, ("bf16 16col", 3): 60.7e6,
                    ("fp64 16col", 2): 2743.0e6, ("fp64 64col", 2): 5054.1e6, ("bf16 16col", 2): 644.8e6,
                    ("fp32 16col", 2): 1281.7e6}

WORKLOADS = {
    # leaf depth and recompression are tuned per run (tune_leaf_depths x {tiles,
    # recompress_tol}); leaf_depth is the choice measured on MI355X and
    # served_leaf_depth the one for served 16-column bf16 blocks, which the
    # kernel-only counter runs use
    "sphere_m5_p2_k8": dict(geometry="sphere", m=5, p=2, kappa=8.0, q=6, eta_adm=1.6, leaf_depth=3,
                            served_leaf_depth=2,
                            tune_leaf_depths=(2, 3, 4), kcap=0.0, tol=1e-8, golden="sphere_m5_p2_k8_rows",
                            recompress_tol=1e-8),
    # the star configurations: one operator solving a block of directions
    "star_m6_p2_k16": dict(geometry="star", m=6, p=2, kappa=16.0, q=8, eta_adm=1.6, leaf_depth=3, kcap=5.0,
                           tol=1e-8, bc="soft", ndir=64, precision="fp64", on_the_fly=False, dir_seed=1,
                           golden="star_m6_p2_k16_rows"),
    "star_m7_p2_k32_hard": dict(geometry="star", m=7, p=2, kappa=32.0, q=8, eta_adm=1.6, leaf_depth=3, kcap=8.0,
                                tol=1e-8, bc="hard", ndir=16, precision="bf16", on_the_fly=True, dir_seed=2,
                                golden="star_m7_p2_k32_hard_rows"),
}
PEAKS = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15}


def mie_soft_farfield(ka, ct):
    """Far-field pattern of the sound-soft unit sphere (Mie series) at the
    cosines ct of the angles between observation and incidence directions."""
    from scipy.special import eval_legendre, spherical_jn, spherical_yn
    ref = np.zeros(len(ct), dtype=np.complex128)
    for nn in range(int(ka) + 30):
        h = spherical_jn(nn, ka) + 1j * spherical_yn(nn, ka)
        ref += (2 * nn + 1) * spherical_jn(nn, ka) / h * eval_legendre(nn, ct)
    return ref * (1j / ka)


def cpu_baseline(w, reps=5):
    """The oracle O1 (plain dense fp64 Galerkin BEM, NumPy) timed on the host's
    cores (all of them, or the OMP_NUM_THREADS share), each stage separately:

    * matvec (the reported value): y = A x with the dense N x N complex128
      matrix (zgemv), median of `reps` after one warm-up;
    * solve: LU (zgesv) of the dense matrix for one right-hand side, once;
    * assembly: the oracle's element row blocks (every source element against
      one target element, singular rules on touching pairs) for one target per
      core over its worker pool, extrapolated x E / cores to the whole matrix.

    The dense matrix holds seeded complex normal values plus N on the diagonal
    (so that LU meets no singular pivot): neither zgemv's nor zgesv's cost
    depends on the values, and the assembled entries are timed separately."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import galerkin as G  # test infrastructure: baseline leg only
    from paper_2306_11324_amd import inputs as I
    pts = I.sphere_patches() if w["geometry"] == "sphere" else I.star_patches(0, I.star_geometry_level(w["m"]))
    cores = G.host_cores()
    bem = G.DenseBEM(pts, p=w["p"], m=w["m"], kappa=w["kappa"], bc="soft", workers=cores)
    n, E = bem.n, bem.disc.nelem
    targets = np.sort(np.random.default_rng(4321).choice(E, cores, replace=False))
    t0 = time.perf_counter()
    for _ in bem._map_targets(targets, bem.ops):
        pass
    t_asm = time.perf_counter() - t0
    with threadpool_limits(cores):
        A = I.random_complex(99, (n, n))
        A[np.diag_indices(n)] += n
        x = I.random_complex(12345, n)
        t_mv = []
        for _ in range(reps + 1):
            t0 = time.perf_counter()
            A @ x
            t_mv.append(time.perf_counter() - t0)
        t_mv = float(np.median(t_mv[1:]))
        t0 = time.perf_counter()
        np.linalg.solve(A, x)
        t_lu = time.perf_counter() - t0
        blas = sorted({f"{d.get('internal_api')} {d.get('num_threads')} threads" for d in threadpool_info()
                       if d.get("user_api") == "blas"})
    del A
    return {"value": 1.0 / t_mv, "unit": "matvecs/s", "cores": cores, "kind": "oracle",
            "sample": f"dense N={n} complex128 matvec (zgemv, median of {reps}); LU solve of the dense matrix "
                      f"(once); the oracle's element row blocks for {cores} of the {E} target elements "
                      f"({t_asm:.1f} s), extrapolated to the whole matrix",
            "matvec_s": t_mv, "solve_lu_s": t_lu, "solves_per_s": 1.0 / t_lu,
            "assembly_s_extrapolated": t_asm * E / cores, "blas": blas}


def large_workload(name, steps, warmup, overrides=None):
    """A star configuration: one operator, a block of incident directions solved
    in lockstep (fp64, or bf16 couplings inside fp64 refinement), far fields at
    64 directions.  One step = one block solve + its far fields; `value` counts
    the column matvecs inside the timed steps.  Beside it: the single-column fp64
    matvec, the block matvec alone with per-kernel HIP-event times and the
    coupling kernel's roofline, the error against the stored oracle rows (relative
    to the operator and to this product), and the far-field invariants of the
    solved block (optical theorem per direction, reciprocity)."""
    import torch

    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    w = dict(WORKLOADS[name], **(overrides or {}))
    dev = torch.device("cuda:0")
    torch.cuda.init()
    ctx = B.Context(0)
    prec = {"fp64": B.FP64, "fp32": B.MIX_FP32, "bf16": B.MIX_BF16}[w["precision"]]
    t0 = time.perf_counter()
    geo = B.Geometry(ctx, I.star_patches(0, I.star_geometry_level(w["m"])), w["m"], w["p"])
    op = B.Operator(ctx, geo, kappa=w["kappa"], bc=B.SOFT if w["bc"] == "soft" else B.HARD, q=w["q"],
                    eta_adm=w["eta_adm"], kcap=w["kcap"], leaf_depth=w["leaf_depth"], precision=prec,
                    far_on_the_fly=w["on_the_fly"])
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = op.info
    n, nd = op.n, w["ndir"]
    print(f"# {name}: N={n} far_pairs={info.far_pairs} nnz={info.nnz} device={info.device_bytes / 1e9:.1f} GB "
          f"setup={t_setup:.1f}s", file=sys.stderr, flush=True)
    lowp = B.MV_LOWPREC if prec != B.FP64 else 0

    def timed(ncol, parts, reps):
        X = torch.from_numpy(I.random_complex(7 + ncol, (ncol, n))).to(dev)
        Y = torch.zeros_like(X)
        op.h2_matvec(X, Y, nrhs=ncol, parts=parts)
        torch.cuda.synchronize()
        op.profile(True)
        t1 = time.perf_counter()
        for _ in range(reps):
            op.h2_matvec(X, Y, nrhs=ncol, parts=parts)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        km = {}
        for k in ("m2l", "spmv", "upward", "downward"):
            cnt, ms = op.kernel_time(k)
            km[k] = ms / max(cnt, 1)
        op.profile(False)
        del X, Y
        return dt, km

    # the block kernels' tile shapes, tuned on this operator for the block width
    tile_shape = None
    if prec == B.FP64 and nd >= 32:
        from paper_2306_11324_amd import autotune as AT
        best_t, cand_t = AT.tune_tile_shape(op, nd, reps=3)
        tile_shape = {"choice": {"coupling_col_tiles": best_t[0], "near_col_tiles": best_t[1]},
                      "candidates": [{"coupling_col_tiles": a, "near_col_tiles": b, "matvec_ms": t}
                                     for a, b, t in cand_t]}
    dt1, km1 = timed(1, B.PART_ALL, 5)
    dtb, kmb = timed(nd, B.PART_ALL | lowp, 5)
    nq2 = info.nq * info.nq
    ntile = 2 if w["bc"] == "hard" else 1
    nvec = 10 if w["bc"] == "hard" else 1      # hard: G on 6 vectors, H on 4
    flops = 8.0 * info.far_pairs * nq2 * nd * (nvec if w["bc"] == "hard" else 1)
    esz = {"fp64": 16, "fp32": 8, "bf16": 4}[w["precision"]]
    tile_bytes = float(info.far_pairs * ntile * nq2 * esz)
    m2l_s = kmb["m2l"] * 1e-3
    if w["precision"] == "fp64":
        roof = {"bound": "mfma", "achieved": flops / m2l_s / 1e12, "peak": PEAKS["fp64"] / 1e12, "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": tile_bytes / m2l_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof.update({"frac": roof["achieved"] / roof["peak"], "traffic": None,
                 "kernel": "m2l_mfma64_soft (fp64 matrix cores)" if w["precision"] == "fp64" else
                           "m2l_mfma<bf16, hard> (bf16 matrix cores)",
                 "avg_launch_ms": kmb["m2l"], "algorithmic_bytes": tile_bytes, "algorithmic_flops": flops})
    # error against the stored oracle rows (fp64 product; also the reduced-precision one)
    g = np.load(os.path.join(ROOT, "tests", "golden", w["golden"] + ".npz"))
    errs = {}
    for label, parts in (("fp64", B.PART_ALL), (w["precision"], B.PART_ALL | lowp)):
        if label in errs:
            continue
        xg = torch.from_numpy(g["x"]).to(dev)
        yg = torch.zeros_like(xg)
        op.h2_matvec(xg, yg, parts=parts)
        torch.cuda.synchronize()
        yr = yg.cpu().numpy()[g["rows"]]
        errs[label] = {"operator_relative": float(np.max(np.abs(yr - g["y"]) / (g["rownorm1"] * np.abs(g["x"]).max()))),
                       "vector_relative": float(np.max(np.abs(yr - g["y"])) / np.max(np.abs(g["y"])))}
    # block solves
    dirs = I.random_directions(w["dir_seed"], nd)
    obs = I.fibonacci_directions(64)
    coeff = torch.zeros((nd, n), dtype=torch.complex128, device=dev)
    uinf = torch.zeros((nd, 64), dtype=torch.complex128, device=dev)
    for _ in range(warmup):
        op.cfie_solve(dirs, coeff, tol=w["tol"], restart=30, maxit=3000)
        op.farfield(coeff, obs, uinf, ndir=nd)
    torch.cuda.synchronize()
    mv, t_solve = 0, 0.0
    t1 = time.perf_counter()
    for _ in range(steps):
        si, st = op.cfie_solve(dirs, coeff, tol=w["tol"], restart=30, maxit=3000)
        op.farfield(coeff, obs, uinf, ndir=nd)
        mv += si.matvecs
    torch.cuda.synchronize()
    T = time.perf_counter() - t1
    # far-field invariants of the solved block (16,384-point Fibonacci lattice)
    fobs = I.fibonacci_directions(16384)
    u = torch.zeros((nd, len(fobs)), dtype=torch.complex128, device=dev)
    op.farfield(coeff, fobs, u, ndir=nd)
    fwd = torch.zeros((nd, nd), dtype=torch.complex128, device=dev)
    op.farfield(coeff, dirs, fwd, ndir=nd)
    back = torch.zeros((nd, nd), dtype=torch.complex128, device=dev)
    op.farfield(coeff, -dirs, back, ndir=nd)
    torch.cuda.synchronize()
    u, fwd, back = u.cpu().numpy(), np.diag(fwd.cpu().numpy()), back.cpu().numpy()
    lhs = 4 * np.pi * np.mean(np.abs(u) ** 2, axis=1)
    rhs = 4 * np.pi / w["kappa"] * fwd.imag
    out = {
        "metric": METRIC, "value": mv / T, "unit": "matvecs/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": T / steps * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if w["precision"] == "fp64" else "bf16 far field, f64 near field and refinement",
        "data": "synthetic",
        "config": {"workload": name, "geometry": "star r = 1 + 0.1 sum c_lm Y_lm (l <= 4), seed 0, 6 patches",
                   "level_m": w["m"], "degree_p": w["p"], "N": n, "kappa": w["kappa"], "bc": w["bc"],
                   "q": w["q"], "eta_adm": w["eta_adm"], "kcap": w["kcap"], "leaf_depth": w["leaf_depth"],
                   "rhs": nd, "precision": w["precision"], "fp64_far_on_the_fly": w["on_the_fly"],
                   "gmres": f"restart 30, tol {w['tol']}", "far_pairs": info.far_pairs, "nnz_near": info.nnz,
                   "device_GB": info.device_bytes / 1e9},
        "solves_per_s": steps * nd / T, "gmres_iters": si.iters, "relres_true": si.relres_true,
        "refinements": si.refinements, "escalated": si.escalated, "setup_s": t_setup,
        "assembly_near_ms": info.assembly_near_ms, "assembly_far_ms": info.assembly_far_ms,
        "single_column_fp64": {"matvecs_per_s": 1.0 / dt1, "kernel_ms": km1},
        "block_matvec": {"ncol": nd, "column_matvecs_per_s": nd / dtb, "ms": dtb * 1e3, "kernel_ms": kmb},
        "err_vs_oracle_rows": errs,
        "farfield_invariants": {"optical_theorem_max_rel": float(np.max(np.abs(lhs - rhs) / np.abs(rhs))),
                                "reciprocity_max_rel": float(np.max(np.abs(back - back.T)) / np.max(np.abs(back)))},
        "roofline": roof,
        "tile_shape": tile_shape,
    }
    print(json.dumps(out), flush=True)


def potential_sweep(counts, m=3, p=3, kappa=2.5, q=8, leaf_depth=2):
    """Scattered-field evaluation time against the number of points, direct
    summation vs the H^2 evaluation (the paper's potential-scaling figure of
    Sec. 5, there on the turbine, whose CAD is not available): the degree-3
    torus at level 3 (R = 2, r = 0.5), kappa = 2.5, q = 8, one incident
    direction along x; seeded points filling the cylinder r <= 4, |z| <= 2
    outside the tube of radius 0.75 around the torus' core circle.  One JSON
    line per point count, then the log-log slopes over the counts from 10^4 on."""
    import torch

    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    dev = torch.device("cuda:0")
    torch.cuda.init()
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.torus_patches(), m, p)
    op = B.Operator(ctx, geo, kappa=kappa, q=q, eta_adm=1.6, leaf_depth=leaf_depth)
    coeff = torch.zeros((1, op.n), dtype=torch.complex128, device=dev)
    info, st = op.cfie_solve(np.array([[1.0, 0.0, 0.0]]), coeff, tol=1e-8, restart=30, maxit=3000)
    rng = np.random.default_rng(5)
    nmax = max(counts)
    pts = np.zeros((0, 3))
    while len(pts) < nmax:
        cand = np.column_stack([rng.uniform(-4, 4, 2 * nmax), rng.uniform(-4, 4, 2 * nmax),
                                rng.uniform(-2, 2, 2 * nmax)])
        rho = np.hypot(cand[:, 0], cand[:, 1])
        keep = (rho <= 4.0) & (np.hypot(rho - 2.0, cand[:, 2]) > 0.75)
        pts = np.concatenate([pts, cand[keep]])
    pts = pts[:nmax]
    rows = []
    for npt in counts:
        P = np.ascontiguousarray(pts[:npt])
        out = {}
        for name, f in (("direct", op.potential), ("h2", op.potential_h2)):
            u = torch.zeros((1, npt), dtype=torch.complex128, device=dev)
            f(coeff, P[:min(npt, 1000)], u[:, :min(npt, 1000)])   # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            f(coeff, P, u)
            torch.cuda.synchronize()
            out[name] = (time.perf_counter() - t0, u.cpu().numpy())
        e = float(np.abs(out["h2"][1] - out["direct"][1]).max() / np.abs(out["direct"][1]).max())
        rec = {"sweep": "potential points", "geometry": "torus R=2 r=0.5", "m": m, "p": p, "kappa": kappa, "q": q,
               "points": npt, "direct_s": out["direct"][0], "h2_s": out["h2"][0],
               "speedup": out["direct"][0] / out["h2"][0], "h2_rel_diff_vs_direct": e}
        rows.append(rec)
        print(json.dumps(rec), flush=True)
    big = [r for r in rows if r["points"] >= 10000]
    if len(big) >= 2:
        lx = np.log([r["points"] for r in big])
        print(json.dumps({"sweep": "potential points", "loglog_slope_vs_points": {
            k: float(np.polyfit(lx, np.log([r[k] for r in big]), 1)[0]) for k in ("direct_s", "h2_s")}}), flush=True)


def scaling_sweep(levels, kappa=2.0, q=6, leaf_depth=2):
    """Matvec time, operator bytes and solve against the level m on the sphere
    at fixed kappa and q (the paper's log-linear time-to-solution claim of Sec.
    5.2): one JSON line per level."""
    import torch

    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    dev = torch.device("cuda:0")
    torch.cuda.init()
    ctx = B.Context(0)
    d = np.array([[0.0, 0.0, 1.0]])
    rows = []
    for m in levels:
        t0 = time.perf_counter()
        geo = B.Geometry(ctx, I.sphere_patches(), m, 2)
        op = B.Operator(ctx, geo, kappa=kappa, q=q, eta_adm=1.6, leaf_depth=leaf_depth)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        x = torch.from_numpy(I.random_complex(12345, op.n)).to(dev)
        y = torch.zeros_like(x)
        op.h2_matvec(x, y)
        torch.cuda.synchronize()
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            op.h2_matvec(x, y)
        torch.cuda.synchronize()
        t_mv = (time.perf_counter() - t0) / reps
        coeff = torch.zeros((1, op.n), dtype=torch.complex128, device=dev)
        info, st = op.cfie_solve(d, coeff, tol=1e-8, restart=30, maxit=3000)
        oi = op.info
        nq2 = oi.nq * oi.nq
        rec = {"sweep": "sphere level", "m": m, "N": op.n, "kappa": kappa, "q": q, "leaf_depth": leaf_depth,
               "far_pairs": oi.far_pairs, "nnz_near": oi.nnz,
               "stream_bytes": oi.far_pairs * nq2 * 16 + oi.nnz * 16, "device_bytes": oi.device_bytes,
               "matvec_ms": t_mv * 1e3, "setup_s": t_setup, "gmres_iters": info.iters,
               "solve_s": info.seconds, "relres_true": info.relres_true}
        rows.append(rec)
        print(json.dumps(rec), flush=True)
        del op, geo, x, y, coeff
        torch.cuda.empty_cache()
    # slopes of log(quantity) against log(N) over the levels whose matrix has a
    # far field from the previous level on (below that the operator is the dense
    # near field), and the paper's guide line m 4^m: time / (m 4^m) per level
    far = [r for r in rows if r["far_pairs"] > 0][1:]
    if len(far) > 1:
        lN = np.log([r["N"] for r in far])
        fit = {k: float(np.polyfit(lN, np.log([r[k] for r in far]), 1)[0])
               for k in ("matvec_ms", "stream_bytes", "setup_s", "solve_s")}
        guide = {r["m"]: r["matvec_ms"] / (r["m"] * 4.0 ** r["m"]) for r in rows}
        print(json.dumps({"sweep": "sphere level", "levels_fitted": [r["m"] for r in far],
                          "loglog_slope_vs_N": fit, "matvec_ms_over_m4m": guide}), flush=True)


def serve_stream(nreq, rate, catalog=0):
    """Continuous batching of a Poisson request stream: each request a seeded
    star-shaped scatterer at level 3..6, kappa in [1, 32], 1..16 directions,
    sound-soft or sound-hard, bf16 couplings with fp64 refinement, admitted by
    HBM budget into 4 concurrent slots.  Latency = completion - arrival.  With
    catalog > 0 the scattering problems come from a catalog of that many, and
    waiting requests for one problem share a block."""
    from paper_2306_11324_amd import inputs as I
    from paper_2306_11324_amd.serving import ServeConfig, Server
    cfg = ServeConfig(slots=4)
    reqs = I.request_stream(nreq, rate=rate, seed=3, catalog=catalog)
    srv = Server(cfg)

    def log(r):
        print(f"# served request {r.rid}: N={r.n} directions={r.uinf.shape[0]} converged={r.converged} "
              f"escalated={r.escalated} latency={r.latency:.2f}s", file=sys.stderr, flush=True)

    res = srv.run(reqs, realtime=True, log=log)
    out = Server.summary(res, srv.wall)
    stages = {}
    for r in res:
        for k, v in r.stages.items():
            stages[k] = stages.get(k, 0.0) + v
    out.update({"arrival_rate_per_s": rate, "slots": cfg.slots, "hbm_budget_GB": cfg.hbm_budget / 1e9,
                "precision": "bf16 couplings, fp64 near field and refinement", "q": cfg.q,
                "leaf_depth": cfg.leaf_depth, "tol": cfg.tol, "peak_reserved_GB": srv.peak_reserved / 1e9,
                "stage_seconds_total": stages,
                "stream": "request_stream(seed=3): level 3..6, kappa U[1,32], 1..16 directions, soft/hard"
                          + (f", problems from a catalog of {catalog}" if catalog else "")})
    return out


def trace_overlap(path):
    """Device overlap of a rocprofv3 kernel trace (its kernel_trace.csv): the
    time at least one kernel runs (busy), the summed kernel durations, and the
    share of busy time during which two or more kernels run, overall and for
    the kernels of different queues (HIP streams map to hardware queues), so
    that work of concurrent requests on their own streams shows as overlap."""
    import csv
    ev = []
    for r in csv.DictReader(open(path)):
        ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r.get("Queue_Id", "0")))
    if not ev:
        print(json.dumps({"error": "no kernels in the trace"}))
        return
    pts = sorted([(s0, 1, q) for s0, e0, q in ev] + [(e0, -1, q) for s0, e0, q in ev], key=lambda t: (t[0], t[1]))
    busy = multi = cross = 0
    running, per_q = 0, {}
    last = pts[0][0]
    for t, d, q in pts:
        dt = t - last
        if running >= 1:
            busy += dt
        if running >= 2:
            multi += dt
        if sum(1 for v in per_q.values() if v > 0) >= 2:
            cross += dt
        running += d
        per_q[q] = per_q.get(q, 0) + d
        last = t
    summed = sum(e0 - s0 for s0, e0, q in ev)
    span = max(e0 for s0, e0, q in ev) - min(s0 for s0, e0, q in ev)
    print(json.dumps({"kernels": len(ev), "queues": len({q for _, _, q in ev}), "span_s": span / 1e9,
                      "busy_s": busy / 1e9, "summed_kernel_s": summed / 1e9,
                      "overlap_factor": summed / max(busy, 1), "busy_share_two_or_more": multi / max(busy, 1),
                      "busy_share_two_or_more_queues": cross / max(busy, 1)}), flush=True)


def kernels_only(reps=20):
    """The matvecs of the default workload alone, for counter runs (rocprofv3
    --pmc) and kernel traces: at the headline's leaf depth the one-column
    product (tile factors), the fp64 blocks of 16 and 64 columns (matrix-core
    coupling and near tiles) and the bf16 block of 16 columns; at the served
    blocks' leaf depth the fp64 blocks of 16 and 64 columns and the bf16 and
    fp32 blocks of 16 columns; then a plain 1 GiB device copy (the counters'
    calibration)."""
    import torch

    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    w = WORKLOADS["sphere_m5_p2_k8"]
    dev = torch.device("cuda:0")
    torch.cuda.init()
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), w["m"], w["p"])
    kw = dict(kappa=w["kappa"], q=w["q"], eta_adm=w["eta_adm"], kcap=w["kcap"])
    d1, d2 = w["leaf_depth"], w["served_leaf_depth"]
    op = B.Operator(ctx, geo, recompress_tol=w["recompress_tol"], leaf_depth=d1, **kw)
    lo = B.Operator(ctx, geo, precision=B.MIX_BF16, leaf_depth=d1, **kw)
    runs = [(op, 1, B.PART_ALL, f"depth {d1}: fp64 1 column"), (op, 16, B.PART_ALL, f"depth {d1}: fp64 16 columns"),
            (op, 64, B.PART_ALL, f"depth {d1}: fp64 64 columns"),
            (lo, 16, B.PART_ALL | B.MV_LOWPREC, f"depth {d1}: bf16 16 columns")]
    if d2 != d1:
        op2 = B.Operator(ctx, geo, leaf_depth=d2, **kw)
        lo2 = B.Operator(ctx, geo, precision=B.MIX_BF16, leaf_depth=d2, **kw)
        f32 = B.Operator(ctx, geo, precision=B.MIX_FP32, leaf_depth=d2, **kw)
        runs += [(op2, 16, B.PART_ALL, f"depth {d2}: fp64 16 columns"),
                 (op2, 64, B.PART_ALL, f"depth {d2}: fp64 64 columns"),
                 (lo2, 16, B.PART_ALL | B.MV_LOWPREC, f"depth {d2}: bf16 16 columns"),
                 (f32, 16, B.PART_ALL | B.MV_LOWPREC, f"depth {d2}: fp32 16 columns")]
    for o, nc, parts, label in runs:
        X = torch.from_numpy(I.random_complex(5, (nc, o.n))).to(dev)
        Y = torch.zeros_like(X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            o.h2_matvec(X, Y, nrhs=nc, parts=parts)
        torch.cuda.synchronize()
        print(f"# {label}: {(time.perf_counter() - t0) / reps * 1e3:.3f} ms per matvec", flush=True)
        del X, Y
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("# copy calibration: 3 x 1 GiB device copies", flush=True)


def counter_summary(dirs, simds=1024):
    """Markdown table of rocprofv3 --pmc runs of `--kernels-only` (their
    run_counter_collection.csv files): per kernel and grid, the mean per
    dispatch of FETCH_SIZE and WRITE_SIZE (bytes, from KiB) and, where
    collected, the MFMA busy fraction SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE
    x SIMDs) and the fp64 / bf16 matrix flops (MOPS x 512) per dispatch, with the
    plain 1 GiB device copy's FETCH_SIZE and WRITE_SIZE as the calibration."""
    import collections
    import csv
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for d in dirs:
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            key = (r["Kernel_Name"].split("(")[0], int(r["Grid_Size"]))
            acc[key][r["Counter_Name"]].append(float(r["Counter_Value"]))
    print("| kernel | grid | dispatches | FETCH_SIZE (MB) | WRITE_SIZE (MB) | MFMA busy | fp64 MFMA GFLOP | bf16 MFMA GFLOP |")
    print("|---|---|---|---|---|---|---|---|")
    for (name, grid), c in sorted(acc.items(), key=lambda kv: -np.mean(kv[1].get("FETCH_SIZE", [0]))):
        def mean(k):
            return float(np.mean(c[k])) if k in c else None
        fetch, write = mean("FETCH_SIZE"), mean("WRITE_SIZE")
        busy, act = mean("SQ_VALU_MFMA_BUSY_CYCLES"), mean("GRBM_GUI_ACTIVE")
        f64, b16 = mean("SQ_INSTS_VALU_MFMA_MOPS_F64"), mean("SQ_INSTS_VALU_MFMA_MOPS_BF16")
        n = max(len(v) for v in c.values())
        if (fetch or 0) < 1024 and not f64 and not b16:   # skip kernels below 1 MB of traffic
            continue
        cell = lambda v, f: "" if v is None else f.format(v)
        print(f"| `{name}` | {grid} | {n} | {cell(fetch and fetch * 1024 / 1e6, '{:.1f}')} | "
              f"{cell(write and write * 1024 / 1e6, '{:.1f}')} | "
              f"{cell(busy / (act * simds) if busy and act else None, '{:.1%}')} | "
              f"{cell(f64 and f64 * 512 / 1e9, '{:.2f}')} | {cell(b16 and b16 * 512 / 1e9, '{:.2f}')} |")


def serve_study(capacity=None, n_capacity=48, n_sweep=48, fractions=(0.4, 0.6, 0.8, 1.0), n_main=200,
                main_fraction=0.8):
    """The serving protocol: capacity (every request visible at once: requests
    served per second), then Poisson streams at fractions of that capacity
    (p50 / p99 latency per rate), then `n_main` requests at `main_fraction` of
    capacity.  Each stream is the seeded request_stream (levels 3..6, kappa in
    [1, 32], 1..16 directions, soft / hard), one JSON line per stream;
    `mean_in_service` = summed admitted-to-done time / wall time (requests
    being served at once)."""
    from paper_2306_11324_amd import inputs as I
    from paper_2306_11324_amd.serving import ServeConfig, Server, percentile
    cfg = ServeConfig(slots=4)
    srv = Server(cfg)

    def log(r):
        print(f"# served request {r.rid}: N={r.n} directions={r.uinf.shape[0]} latency={r.latency:.2f}s",
              file=sys.stderr, flush=True)

    def run(n, rate, realtime, label):
        reqs = I.request_stream(n, rate=rate, seed=3)
        res = srv.run(reqs, realtime=realtime, log=log)
        out = Server.summary(res, srv.wall)
        out["mean_in_service"] = sum(r.done - r.admitted for r in res) / srv.wall
        if not realtime:   # every request visible at time 0: latency = completion time
            lat = [r.done for r in res]
            out["p50_latency_s"], out["p99_latency_s"] = percentile(lat, 50), percentile(lat, 99)
        out.update({"stream": label, "arrival_rate_per_s": rate if realtime else None, "slots": cfg.slots})
        print(json.dumps(out), flush=True)
        return out

    if capacity is None:
        capacity = run(n_capacity, 1.0, False, "capacity: all requests visible at once")["requests_per_s"]
    for f in fractions:
        run(n_sweep, f * capacity, True, f"rate sweep: {f:.1f} x capacity {capacity:.3f}/s")
    if n_main:
        run(n_main, main_fraction * capacity, True, f"{n_main} requests at {main_fraction:.1f} x capacity")


def convergence_study(mmax, q, quad_extra, bcs=("soft", "hard"), out_path=None, reference="cfie"):
    import torch

    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    ctx = B.Context(0)
    dev = torch.device("cuda:0")
    d = np.array([[1.0, 0.0, 0.0]])
    pts = 5.0 * I.fibonacci_directions(100)
    patches = I.torus_patches(2.0, 0.5)
    series = [(bc, p) for bc in bcs for p in range(0 if bc == "soft" else 1, 4)]
    vals, lines = {}, []
    sink = open(out_path, "w") if out_path else None
    runs = [(bc, p, m, "cfie") for bc, p in series for m in range(mmax + 1)]
    if reference == "single_layer":
        runs += [(bc, 3, mmax, "single_layer") for bc in bcs]
    for bc, p, m, form in runs:
        t0 = time.perf_counter()
        geo = B.Geometry(ctx, patches, m, p)
        op = B.Operator(ctx, geo, kappa=2.5, bc=B.SOFT if bc == "soft" else B.HARD, q=q, eta_adm=1.6,
                        leaf_depth=3, quad_extra=quad_extra,
                        formulation=B.SINGLE_LAYER if form == "single_layer" else B.CFIE)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        coeff = torch.zeros((1, op.n), dtype=torch.complex128, device=dev)
        info, st = op.cfie_solve(d, coeff, tol=1e-12, restart=50, maxit=3000)
        u = torch.zeros((1, len(pts)), dtype=torch.complex128, device=dev)
        op.potential(coeff, pts, u)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        key = (bc, p, m) if form == "cfie" else (bc, "single_layer")
        vals[key] = u.cpu().numpy()[0]
        rec = dict(bc=bc, p=p, m=m, formulation=form, n=op.n, status=st, iters=info.iters, converged=info.converged,
                   relres_true=info.relres_true, assembly_s=t1 - t0, solve_s=t2 - t1)
        lines.append(rec)
        print(json.dumps(rec), flush=True)
        if sink:
            sink.write(json.dumps(dict(rec, u_re=vals[key].real.tolist(), u_im=vals[key].imag.tolist())) + "\n")
            sink.flush()
        del op, geo
    summary = {}
    for bc in bcs:
        pmax = 3
        ref = vals[(bc, pmax, mmax)] if reference == "cfie" else vals[(bc, "single_layer")]
        for p in range(0 if bc == "soft" else 1, 4):
            errs = [float(np.abs(vals[(bc, p, m)] - ref).max()) for m in range(mmax + 1)]
            if p == pmax and reference == "cfie":
                errs[-1] = None
            eoc = [None if (a is None or b is None or b == 0) else float(np.log2(a / b))
                   for a, b in zip(errs[:-1], errs[1:])]
            summary[f"{bc}_p{p}"] = dict(err=errs, eoc=eoc, expected=2 * p + 2 if bc == "soft" else 2 * p + 1)
    out = {"study": "torus convergence", "kappa": 2.5, "q": q, "quad_extra": quad_extra, "mmax": mmax,
           "points": "100 on |x| = 5",
           "reference": ("finest level, p = 3, same boundary condition" if reference == "cfie" else
                         "single-layer formulation, finest level, p = 3, same boundary condition"),
           "series": summary}
    print(json.dumps(out), flush=True)
    if sink:
        sink.write(json.dumps(out) + "\n")
        sink.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sphere_m5_p2_k8", choices=sorted(WORKLOADS))
    ap.add_argument("--matvecs", type=int, default=50, help="matvec-only timing loop length")
    ap.add_argument("--kcap", type=float, default=None, help="star workloads: kappa*diam cap override")
    ap.add_argument("--q", type=int, default=None, help="star workloads: interpolation degree override")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--block", type=int, default=16, help="directions per served block (0: skip)")
    ap.add_argument("--serve", type=int, default=32, help="requests in the served stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=1.0, help="Poisson arrival rate of the stream (1/s)")
    ap.add_argument("--convergence", action="store_true", help="run the torus convergence benchmark instead")
    ap.add_argument("--conv-mmax", type=int, default=6)
    ap.add_argument("--conv-q", type=int, default=8)
    ap.add_argument("--conv-quad-extra", type=int, default=2,
                    help="raise every near-field quadrature order (the default orders leave a floor near 2e-7)")
    ap.add_argument("--conv-bc", default="soft,hard")
    ap.add_argument("--conv-reference", default="cfie", choices=["cfie", "single_layer"],
                    help="reference solution: the finest CFIE solution or the single-layer one (as the paper)")
    ap.add_argument("--conv-out", default=None, help="also write the study's JSON lines to this file")
    ap.add_argument("--sweep", default=None, help="levels m for the scaling sweep, e.g. 3,4,5,6,7")
    ap.add_argument("--potential-sweep", default=None,
                    help="point counts for the scattered-field sweep (direct vs H^2), e.g. 1000,10000,100000")
    ap.add_argument("--counter-summary", nargs="+", default=None,
                    help="summarise rocprofv3 --pmc output directories of --kernels-only (no GPU)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the default workload's matvecs (and a 1 GiB copy), for counter runs")
    ap.add_argument("--serve-study", action="store_true",
                    help="serving protocol: capacity, rate sweep, --serve-main requests at 0.8 x capacity")
    ap.add_argument("--serve-capacity", type=float, default=None, help="skip the capacity run (requests/s)")
    ap.add_argument("--serve-fractions", default="0.4,0.6,0.8,1.0")
    ap.add_argument("--serve-main", type=int, default=200)
    ap.add_argument("--serve-catalog", type=int, default=0,
                    help="draw the stream's scattering problems from a catalog of this many (0: all distinct)")
    ap.add_argument("--serve-only", action="store_true",
                    help="only the request stream (--serve requests at --serve-rate), e.g. under a kernel trace")
    ap.add_argument("--trace-overlap", default=None,
                    help="device overlap of a rocprofv3 kernel_trace.csv (no GPU)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration for profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (sharding an operator or "
                                   "a request stream across GPUs is not built)"}))
        sys.exit(2)

    if args.convergence:
        convergence_study(args.conv_mmax, args.conv_q, args.conv_quad_extra, tuple(args.conv_bc.split(",")),
                          args.conv_out, args.conv_reference)
        return
    if args.sweep:
        scaling_sweep([int(v) for v in args.sweep.split(",")])
        return
    if args.potential_sweep:
        potential_sweep([int(v) for v in args.potential_sweep.split(",")])
        return
    if args.counter_summary:
        counter_summary(args.counter_summary)
        return
    if args.kernels_only:
        kernels_only()
        return
    if args.trace_overlap:
        trace_overlap(args.trace_overlap)
        return
    if args.serve_only:
        print(json.dumps(serve_stream(args.serve, args.serve_rate, args.serve_catalog)), flush=True)
        return
    if args.serve_study:
        fr = tuple(float(v) for v in args.serve_fractions.split(",")) if args.serve_fractions else ()
        serve_study(args.serve_capacity, fractions=fr, n_main=args.serve_main)
        return
    if args.workload != "sphere_m5_p2_k8":
        large_workload(args.workload, args.steps, args.warmup,
                       {k: v for k, v in (("kcap", args.kcap), ("q", args.q)) if v is not None})
        return

    import torch

    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I

    w = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.init()
    ctx = B.Context(0)
    pts = I.sphere_patches() if w["geometry"] == "sphere" else I.star_patches(0, I.star_geometry_level(w["m"]))
    geo = B.Geometry(ctx, pts, w["m"], w["p"])
    # the operator's shape for this workload: the autotuner over leaf depth and
    # tiles / recompressed factors, costed by matvec time (the operator serves
    # every timed solve), among shapes with admissible blocks; a leaf depth
    # without any (the dense matrix) is measured and listed beside them
    from paper_2306_11324_amd import autotune as AT
    best, cand = AT.tune(ctx, geo, w["m"], w["p"], 1, w["kappa"], q=w["q"], precision=B.FP64, eta_adm=w["eta_adm"],
                        leaf_depths=w["tune_leaf_depths"], on_the_fly=(False,),
                        recompress_tols=(0.0, w["recompress_tol"]), matvecs=10 ** 6, reps=20, require_far=True)
    LD, RT = best.leaf_depth, best.recompress_tol
    headline_tuning = {"choice": {"leaf_depth": LD, "far_recompress_tol": RT},
                       "candidates": [{"leaf_depth": c.leaf_depth, "far_recompress_tol": c.recompress_tol,
                                       "far_pairs": c.far_pairs, "matvec_ms": c.matvec_ms,
                                       "assembly_ms": c.assembly_ms, "device_bytes": c.device_bytes}
                                      for c in cand],
                       "note": "one fp64 column, 20 timed matvecs per candidate; far_pairs = 0 is the dense "
                               "matrix (no admissible blocks), listed and not chosen"}
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    op = B.Operator(ctx, geo, kappa=w["kappa"], q=w["q"], eta_adm=w["eta_adm"], kcap=w["kcap"],
                    leaf_depth=LD, recompress_tol=RT)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = op.info
    n = op.n
    print(f"# workload {args.workload}: N={n} far_pairs={info.far_pairs} near_pairs={info.near_elem_pairs} "
          f"nnz={info.nnz} device={info.device_bytes / 1e9:.2f} GB setup={t_setup:.2f}s "
          f"(near {info.assembly_near_ms:.0f} ms, far {info.assembly_far_ms:.0f} ms)", file=sys.stderr, flush=True)

    d = np.array([[0.0, 0.0, 1.0]])
    obs = I.fibonacci_directions(64)

    def run_solves(o, dirs, steps, warmup):
        """Timed lockstep solves of all `dirs` + far fields; returns rates."""
        nd = len(dirs)
        coeff = torch.zeros((nd, o.n), dtype=torch.complex128, device=dev)
        uinf = torch.zeros((nd, 64), dtype=torch.complex128, device=dev)
        for _ in range(warmup):
            o.cfie_solve(dirs, coeff, tol=w["tol"], restart=30, maxit=2000)
            o.farfield(coeff, obs, uinf, ndir=nd)
        torch.cuda.synchronize()
        mv, its, relt, refs = 0, 0, 0.0, 0
        t0 = time.perf_counter()
        for _ in range(steps):
            si, st = o.cfie_solve(dirs, coeff, tol=w["tol"], restart=30, maxit=2000)
            o.farfield(coeff, obs, uinf, ndir=nd)
            mv += si.matvecs
            its = si.iters
            relt = max(relt, si.relres_true)
            refs = si.refinements
        torch.cuda.synchronize()
        T = time.perf_counter() - t0
        return dict(T=T, matvecs_per_s=mv / T, solves_per_s=steps * nd / T, ms_per_step=T / steps * 1e3,
                    gmres_iters=its, relres_true=relt, refinements=refs, coeff=coeff, uinf=uinf)

    elem_bytes = {"fp64": 16, "fp32": 8, "bf16": 4}
    mfma_peak = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15}

    def block_matvec(o, prec_name, xb, yb, reps):
        """Block matvec (args.block columns) timed alone; the coupling kernel's
        algorithmic bytes are the stored tiles (q+1)^4 per far pair."""
        parts = B.PART_ALL | (0 if prec_name == "fp64" else B.MV_LOWPREC)
        nc = xb.shape[0]
        o.h2_matvec(xb, yb, nrhs=nc, parts=parts)
        torch.cuda.synchronize()
        o.profile(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            o.h2_matvec(xb, yb, nrhs=nc, parts=parts)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / reps
        km = {}
        for k in ("m2l", "spmv", "upward", "downward"):
            cnt, ms = o.kernel_time(k)
            km[k] = ms / max(cnt, 1)
        o.profile(False)
        avg = km["m2l"] / 1e3
        oi = o.info
        nq2 = oi.nq * oi.nq
        flops = 8.0 * oi.far_pairs * nq2 * nc
        byts = float(oi.far_pairs * nq2 * elem_bytes[prec_name])
        return {"ncol": nc, "column_matvecs_per_s": nc / tb, "ms_per_block_matvec": tb * 1e3, "kernel_ms": km,
                "m2l_algorithmic_bytes": byts,
                "m2l_traffic_bytes": MEASURED_TRAFFIC.get((f"{prec_name} {nc}col", w["m"] - o.info.leaf_level)),
                "leaf_depth": w["m"] - o.info.leaf_level,
                "m2l_kernel": "m2l_mfma64_soft (fp64 matrix cores)" if prec_name == "fp64" else
                              f"m2l_mfma_soft ({prec_name} matrix cores)",
                "m2l_GBps": byts / avg / 1e9, "m2l_TFLOPs": flops / avg / 1e12,
                "m2l_frac_hbm_peak": byts / avg / (HBM_PEAK_GBS * 1e9),
                "m2l_frac_matrix_peak": flops / avg / mfma_peak[prec_name]}

    g_rows = np.load(os.path.join(ROOT, "tests", "golden", w["golden"] + ".npz"))

    def oracle_row_error(y):
        yr = y[g_rows["rows"]]
        return {"operator_relative": float(np.max(np.abs(yr - g_rows["y"]) /
                                                  (g_rows["rownorm1"] * np.abs(g_rows["x"]).max()))),
                "vector_relative": float(np.max(np.abs(yr - g_rows["y"])) / np.max(np.abs(g_rows["y"])))}

    plain = run_solves(op, d, args.steps, args.warmup)
    value = plain["matvecs_per_s"]
    # scattered field of the plain solution at points on the radius-2 sphere
    pot_pts = 2.0 * I.fibonacci_directions(4096)
    pot_u = torch.zeros(len(pot_pts), dtype=torch.complex128, device=dev)
    op.potential(plain["coeff"], pot_pts, pot_u)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op.potential(plain["coeff"], pot_pts, pot_u)
    torch.cuda.synchronize()
    t_pot = time.perf_counter() - t0
    pot_evals = len(pot_pts) * info.nelem * 64
    potential = {"points": len(pot_pts), "seconds": t_pot, "points_per_s": len(pot_pts) / t_pot,
                 "kernel_evaluations_per_s": pot_evals / t_pot,
                 "note": "u_s at 4096 points on |x| = 2, 8 x 8 Gauss points on each of the elements"}
    # direct summation against the H^2 evaluation on a seeded shell of 200,000 points
    rng = np.random.default_rng(2024)
    sh = rng.normal(size=(200000, 3))
    sh = sh / np.linalg.norm(sh, axis=1, keepdims=True) * rng.uniform(1.2, 4.0, size=(200000, 1))
    shell = {}
    ush = {}
    for name, f in (("direct", op.potential), ("h2", op.potential_h2)):
        uu = torch.zeros(len(sh), dtype=torch.complex128, device=dev)
        f(plain["coeff"], sh[:4096], uu[:4096])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f(plain["coeff"], sh, uu)
        torch.cuda.synchronize()
        shell[f"{name}_seconds"] = time.perf_counter() - t0
        ush[name] = uu.cpu().numpy()
    shell["h2_rel_diff_vs_direct"] = float(np.abs(ush["h2"] - ush["direct"]).max() / np.abs(ush["direct"]).max())
    shell["h2_speedup"] = shell["direct_seconds"] / shell["h2_seconds"]
    shell["note"] = "200,000 seeded points in 1.2 <= |x| <= 4 (potential vs potential_h2, host plan included)"
    potential["shell_200k"] = shell
    op.use_graphs(True)
    plain_graphs = run_solves(op, d, args.steps, args.warmup)
    op.use_graphs(False)
    # the same solves with one H^2 matrix per operator summed lazily (Sec. 5.1's set-up)
    op_sep = B.Operator(ctx, geo, kappa=w["kappa"], q=w["q"], eta_adm=w["eta_adm"], kcap=w["kcap"],
                        leaf_depth=LD, separate=True)
    sep = run_solves(op_sep, d, args.steps, args.warmup)
    paper_mode = {
        "matvecs_per_s": sep["matvecs_per_s"], "solves_per_s": sep["solves_per_s"],
        "device_bytes": op_sep.info.device_bytes, "fused_device_bytes": info.device_bytes,
        "fused_speedup": value / sep["matvecs_per_s"],
        "far_field_rel_diff_vs_fused": float((sep["uinf"] - plain["uinf"]).abs().max() / plain["uinf"].abs().max()),
        "note": "separate H^2 matrices of 1/2 M + K* and V, applied as a lazy sum, against the fused kernel"}
    del op_sep, sep
    torch.cuda.empty_cache()
    # the autotuner's view of the served block form: leaf depth for 16 bf16 columns
    # (costed as a served request: assembly plus 200 block matvecs)
    tuned = {"fp64_1col": headline_tuning}
    for label, prec, nc in (("bf16_16col", B.MIX_BF16, 16),):
        bb, cc = AT.tune(ctx, geo, w["m"], w["p"], nc, w["kappa"], q=w["q"], precision=prec,
                         eta_adm=w["eta_adm"], leaf_depths=(2, 3, 4), on_the_fly=(False,), reps=5,
                         require_far=True)
        tuned[label] = {"choice_leaf_depth": bb.leaf_depth,
                        "candidates": [{"leaf_depth": c.leaf_depth, "far_pairs": c.far_pairs, "matvec_ms": c.matvec_ms,
                                        "assembly_ms": c.assembly_ms, "device_bytes": c.device_bytes}
                                       for c in cc]}
    torch.cuda.empty_cache()
    # the same solves streaming the coupling tiles themselves (no recompression),
    # with the factors truncated at 1e-7, and at leaf depth 2 (smaller leaves:
    # a sparser near field, four times the coupling tiles)
    recompressed = {}
    for label, ld, rt in (("tiles", LD, 0.0), ("tol_1e-7", LD, 1e-7), ("leaf_depth_2", 2, RT)):
        if label == "leaf_depth_2" and LD == 2:
            continue
        op_t = B.Operator(ctx, geo, kappa=w["kappa"], q=w["q"], eta_adm=w["eta_adm"], kcap=w["kcap"],
                          leaf_depth=ld, recompress_tol=rt)
        rs = run_solves(op_t, d, args.steps, args.warmup)
        xt = torch.from_numpy(g_rows["x"]).to(dev)
        yt = torch.zeros_like(xt)
        op_t.h2_matvec(xt, yt)
        torch.cuda.synchronize()
        recompressed[label] = {
            "leaf_depth": ld, "far_recompress_tol": rt, "matvecs_per_s": rs["matvecs_per_s"],
            "solves_per_s": rs["solves_per_s"], "gmres_iters": rs["gmres_iters"],
            "headline_speedup": value / rs["matvecs_per_s"], "device_bytes": op_t.info.device_bytes,
            "err_matvec_vs_oracle_rows": oracle_row_error(yt.cpu().numpy()),
            "far_field_rel_diff_vs_headline": float((rs["uinf"] - plain["uinf"]).abs().max()
                                                    / plain["uinf"].abs().max())}
        del op_t, rs, xt, yt
    torch.cuda.empty_cache()
    T = plain["T"]
    iters = [plain["gmres_iters"]]
    relres_true = plain["relres_true"]
    uinf = plain["uinf"][0]

    # served forms: a block of incident directions in lockstep, fp64 and mixed
    # precision, and the block matvec alone with per-kernel HIP-event times
    served, block_mv = {}, {}
    if args.block > 0:
        dirs_b = I.random_directions(1, args.block)
        ref_coeff = None
        xb = torch.from_numpy(I.random_complex(777, (args.block, n))).to(dev)
        yb = torch.zeros_like(xb)
        # the served blocks at the leaf depth the autotuner chose for served requests
        # of 16 bf16 columns (assembly + 200 block matvecs), every precision alike;
        # the fp64 block on the headline operator when the depths agree
        ld_lo = tuned["bf16_16col"]["choice_leaf_depth"]
        served["leaf_depth"] = ld_lo
        op64 = op if ld_lo == LD else None
        for prec_name, prec in (("fp64", B.FP64), ("fp32", B.MIX_FP32), ("bf16", B.MIX_BF16)):
            if prec == B.FP64 and op64 is not None:
                o = op64
            else:
                o = B.Operator(ctx, geo, kappa=w["kappa"], q=w["q"], eta_adm=w["eta_adm"], kcap=w["kcap"],
                               leaf_depth=ld_lo, precision=prec)
                if prec == B.FP64:
                    op64 = o
            r = run_solves(o, dirs_b, max(1, args.steps // 2), 1)
            c = r.pop("coeff").cpu().numpy()
            u = r.pop("uinf").cpu().numpy()
            if ref_coeff is None:
                ref_coeff, ref_uinf = c, u
            r["solution_rel_diff_vs_fp64_block"] = float(np.abs(c - ref_coeff).max() / np.abs(ref_coeff).max())
            # the result's own error: far field per direction against the fp64
            # block's and against the Mie series of the sphere
            r["farfield_rel_diff_vs_fp64_block"] = float(np.abs(u - ref_uinf).max() / np.abs(ref_uinf).max())
            if w["geometry"] == "sphere" and w.get("bc", "soft") == "soft":
                r["farfield_max_rel_err_vs_mie"] = max(
                    float(np.abs(u[i] - mref).max() / np.abs(mref).max())
                    for i, mref in enumerate(mie_soft_farfield(w["kappa"], obs @ dv) for dv in dirs_b))
            r["speedup_matvecs_vs_plain_fp64"] = r["matvecs_per_s"] / value
            r["speedup_solves_vs_plain_fp64"] = r["solves_per_s"] / plain["solves_per_s"]
            r.pop("T")
            served[f"{prec_name}_block{args.block}"] = r
            block_mv[prec_name] = block_matvec(o, prec_name, xb, yb, max(5, args.matvecs // 5))
            # the same solves with the matvec captured into HIP graphs
            o.use_graphs(True)
            rg = run_solves(o, dirs_b, max(1, args.steps // 2), 1)
            o.use_graphs(False)
            served[f"{prec_name}_block{args.block}_graphs"] = {
                "matvecs_per_s": rg["matvecs_per_s"], "solves_per_s": rg["solves_per_s"],
                "ms_per_step": rg["ms_per_step"], "relres_true": rg["relres_true"]}
            if prec != B.FP64:
                del o
            torch.cuda.empty_cache()
        # fp64 at 64 columns (the width of a 64-direction block): the coupling's
        # arithmetic intensity passes the fp64 ridge, the matrix-core roofline applies
        x64 = torch.from_numpy(I.random_complex(778, (64, n))).to(dev)
        y64 = torch.zeros_like(x64)
        best_t, cand_t = AT.tune_tile_shape(op64, 64, reps=5)
        block_mv["fp64_64col"] = block_matvec(op64, "fp64", x64, y64, max(5, args.matvecs // 5))
        block_mv["fp64_64col"]["tile_shape"] = {
            "choice": {"coupling_col_tiles": best_t[0], "near_col_tiles": best_t[1]},
            "candidates": [{"coupling_col_tiles": a, "near_col_tiles": b, "matvec_ms": t} for a, b, t in cand_t]}
        op64.set_tile_shape(0, 0)
        if op64 is not op:
            del op64
        # the fp64 and bf16 blocks at the headline's own shape (assembly not counted)
        if ld_lo != LD:
            for prec_name, prec in (("fp64", B.FP64), ("bf16", B.MIX_BF16)):
                ob = op if prec == B.FP64 else B.Operator(ctx, geo, kappa=w["kappa"], q=w["q"],
                                                          eta_adm=w["eta_adm"], kcap=w["kcap"], leaf_depth=LD,
                                                          precision=prec)
                r = run_solves(ob, dirs_b, max(1, args.steps // 2), 1)
                r.pop("coeff"), r.pop("uinf"), r.pop("T")
                r["speedup_matvecs_vs_plain_fp64"] = r["matvecs_per_s"] / value
                r["leaf_depth"] = LD
                served[f"{prec_name}_block{args.block}_headline_shape"] = r
                if ob is not op:
                    del ob
        del xb, yb, x64, y64
        torch.cuda.empty_cache()

    # matvec-only loop with HIP-event kernel timing on the launch stream
    x = torch.from_numpy(I.random_complex(12345, n)).to(dev)
    y = torch.zeros_like(x)
    op.h2_matvec(x, y)
    torch.cuda.synchronize()
    op.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.matvecs):
        op.h2_matvec(x, y)
    torch.cuda.synchronize()
    t_mv = (time.perf_counter() - t0) / args.matvecs
    m2l_n, m2l_ms = op.kernel_time("m2l")
    spmv_n, spmv_ms = op.kernel_time("spmv")
    up_n, up_ms = op.kernel_time("upward")
    dn_n, dn_ms = op.kernel_time("downward")
    op.profile(False)
    op.h2_matvec(x, y)
    torch.cuda.synchronize()
    yv = y.cpu().numpy()

    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    nq = info.nq
    # algorithmic bytes of the single-column coupling: the tile factors (or the
    # tiles), the source moments of every pair and the chunk partials
    nchunk_est = info.far_pairs / 8.0
    tile_or_factor = info.far_factor_entries * 16 if info.far_factor_entries else info.far_pairs * nq * nq * 16
    m2l_bytes = tile_or_factor + info.far_pairs * nq * 16 + nchunk_est * nq * 16
    m2l_avg = m2l_ms / max(m2l_n, 1) / 1e3
    # ... and of the one-column near product: the values, the groups' column
    # lists, row pointers and list offsets, x, the far part and y
    spmv_bytes = info.nnz * 16 + info.near_col_entries * 4 + n * 16 + 3 * n * 16
    spmv_avg = spmv_ms / max(spmv_n, 1) / 1e3
    # the roofline of the kernel that takes the most time per matvec
    near_kernel = "spmv_groups<16>" if info.near_group_staged else "spmv_combine<1>"
    if spmv_n and spmv_avg > m2l_avg:
        roof_kernel, roof_bytes, roof_avg = near_kernel, spmv_bytes, spmv_avg
    else:
        roof_kernel = "m2l_chunks_lowrank" if info.far_factor_entries else "m2l_chunks_wave"
        roof_bytes, roof_avg = m2l_bytes, m2l_avg
    achieved = roof_bytes / roof_avg / 1e9 if roof_avg > 0 else None

    # error against the stored fp64 oracle rows / Mie
    xg = torch.from_numpy(g_rows["x"]).to(dev)
    yg = torch.zeros_like(xg)
    op.h2_matvec(xg, yg)
    torch.cuda.synchronize()
    err_rows = oracle_row_error(yg.cpu().numpy())
    err_oracle = err_rows["operator_relative"]
    err_mie = None
    if w["geometry"] == "sphere":
        ref = mie_soft_farfield(w["kappa"], obs @ d[0])
        u = uinf.cpu().numpy()
        err_mie = float(np.abs(u - ref).max() / np.abs(ref).max())

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "geometry": "unit sphere, 6 rational-quadratic patches",
                   "level_m": w["m"], "degree_p": w["p"], "N": n, "kappa": w["kappa"], "bc": "soft",
                   "q": w["q"], "eta_adm": w["eta_adm"], "kcap": w["kcap"], "leaf_depth": LD,
                   "far_recompress_tol": RT, "shape": "autotuned (leaf depth, tiles / factors)",
                   "rhs": 1, "gmres": f"restart 30, tol {w['tol']}", "far_pairs": info.far_pairs,
                   "nnz_near": info.nnz},
        "solves_per_s": plain["solves_per_s"],
        "graphs": {"matvecs_per_s": plain_graphs["matvecs_per_s"], "solves_per_s": plain_graphs["solves_per_s"],
                   "note": "same solves with the matvec captured into HIP graphs (igb_op_use_graphs)"},
        "paper_mode": paper_mode,
        "recompressed": recompressed,
        "autotune": tuned,
        "gmres_iters": iters[-1],
        "relres_true": relres_true,
        "matvec_only_per_s": 1.0 / t_mv,
        "assembly_ms": info.assembly_near_ms + info.assembly_far_ms,
        "assembly_near_ms": info.assembly_near_ms,
        "assembly_far_ms": info.assembly_far_ms,
        "kernel_ms": {"m2l": m2l_ms / max(m2l_n, 1), "spmv": spmv_ms / max(spmv_n, 1),
                      "upward": up_ms / max(up_n, 1), "downward": dn_ms / max(dn_n, 1)},
        "potential": potential,
        "served": served,
        "block_matvec": block_mv,
        "err_matvec_vs_oracle_rows": err_oracle,
        "err_matvec_vs_oracle_rows_measures": err_rows,
        "far_factor_avg_rank": info.far_factor_entries / (2.0 * nq * info.far_pairs) if info.far_factor_entries
                               else None,
        "err_farfield_vs_mie": err_mie,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": MEASURED_TRAFFIC.get((roof_kernel, LD)),
                     "kernel": roof_kernel, "bytes_per_launch": roof_bytes, "avg_launch_ms": roof_avg * 1e3,
                     "coupling": {"kernel": "m2l_chunks_lowrank" if info.far_factor_entries else "m2l_chunks_wave",
                                  "bytes_per_launch": m2l_bytes, "avg_launch_ms": m2l_avg * 1e3,
                                  "achieved_GBps": m2l_bytes / m2l_avg / 1e9 if m2l_n else None,
                                  "traffic": MEASURED_TRAFFIC.get(
                                      ("m2l_chunks_lowrank" if info.far_factor_entries else "m2l_chunks_wave", LD))},
                     "near": {"kernel": near_kernel, "bytes_per_launch": spmv_bytes,
                              "avg_launch_ms": spmv_avg * 1e3,
                              "achieved_GBps": spmv_bytes / spmv_avg / 1e9 if spmv_n else None,
                              "traffic": MEASURED_TRAFFIC.get((near_kernel, LD))}},
    }
    if args.serve > 0:
        out["serving"] = serve_stream(args.serve, args.serve_rate)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
