"""Scheduler of the serving loop without a GPU: a stub executor models only
durations and bytes.  Checks admission by HBM budget, slot reuse, completion of
every request, FIFO order among requests that fit, and the latency statistics."""
import threading
import time
import types

import numpy as np

from paper_2306_11324_amd import inputs as I
from paper_2306_11324_amd.serving import ServeConfig, Server, percentile


def test_request_stream_is_seeded_and_in_range():
    a = I.request_stream(20, rate=5.0, seed=3)
    b = I.request_stream(20, rate=5.0, seed=3)
    assert [(r.seed, r.m, r.kappa, r.bc, r.dirs.shape) for r in a] == \
           [(r.seed, r.m, r.kappa, r.bc, r.dirs.shape) for r in b]
    assert all(3 <= r.m <= 6 and 1 <= r.kappa <= 32 and 1 <= len(r.dirs) <= 16 for r in a)
    assert all(np.allclose(np.linalg.norm(r.dirs, axis=1), 1) for r in a)
    assert np.all(np.diff([r.arrival for r in a]) > 0)


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50 and percentile(v, 99) == 99 and percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0


def _stub(budget, slots, sizes, durations):
    active = {"n": 0, "bytes": 0, "max_n": 0, "max_bytes": 0}
    lock = threading.Lock()

    def est(req):
        return sizes[req.rid]

    def solve(req, slot):
        with lock:
            active["n"] += 1
            active["bytes"] += sizes[req.rid]
            active["max_n"] = max(active["max_n"], active["n"])
            active["max_bytes"] = max(active["max_bytes"], active["bytes"])
        time.sleep(durations[req.rid])
        with lock:
            active["n"] -= 1
            active["bytes"] -= sizes[req.rid]
        info = types.SimpleNamespace(iters=1, matvecs=2, relres_true=0.0, converged=len(req.dirs))
        return 10, info, np.zeros((len(req.dirs), 4), complex)

    srv = Server(ServeConfig(slots=slots, hbm_budget=budget, nobs=4), solve_fn=solve, estimate_fn=est)
    return srv, active


def test_admission_respects_budget_and_slots():
    reqs = I.request_stream(24, rate=200.0, seed=11)
    rng = np.random.default_rng(0)
    sizes = {r.rid: int(rng.integers(10, 60)) for r in reqs}
    durations = {r.rid: float(rng.uniform(0.005, 0.02)) for r in reqs}
    srv, active = _stub(100, 4, sizes, durations)
    res = srv.run(reqs)
    assert [r.rid for r in res] == [r.rid for r in reqs]
    assert active["max_bytes"] <= 100 and active["max_n"] <= 4
    assert srv.peak_reserved <= 100
    assert active["max_n"] >= 2              # requests did overlap
    assert all(r.done >= r.admitted >= r.arrival - 1e-3 for r in res)
    s = Server.summary(res, srv.wall)
    assert s["requests"] == 24 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_tiny_budget_serialises():
    reqs = I.request_stream(6, rate=1000.0, seed=5)
    sizes = {r.rid: 50 for r in reqs}
    durations = {r.rid: 0.01 for r in reqs}
    srv, active = _stub(60, 4, sizes, durations)
    res = srv.run(reqs)
    assert len(res) == 6 and active["max_n"] == 1


def test_request_larger_than_budget_is_rejected():
    reqs = I.request_stream(2, rate=10.0, seed=5)
    srv, _ = _stub(10, 2, {r.rid: 50 for r in reqs}, {r.rid: 0.0 for r in reqs})
    try:
        srv.run(reqs)
    except ValueError:
        return
    raise AssertionError("expected a ValueError")


def test_kappa_cap_reaches_the_size_model():
    """ServeConfig.kcap is passed to the operator: on a level-4 request at
    kappa = 32 a cap of 4 keeps coarse blocks out of the far field, so the
    host plan's size estimate changes (no device memory is touched)."""
    req = I.Request(rid=0, arrival=0.0, seed=5, m=4, kappa=32.0, dirs=I.random_directions(0, 2), bc="soft")
    sizes = {}
    for kcap in (0.0, 4.0):
        srv = Server(ServeConfig(kcap=kcap, nobs=4), solve_fn=lambda r, s: None)
        assert srv._op_args(req)["kcap"] == kcap
        sizes[kcap] = srv.estimate(req)
    assert sizes[0.0] > 0 and sizes[4.0] > 0 and sizes[0.0] != sizes[4.0]


def test_requests_for_one_problem_share_a_block():
    """Requests of a catalog stream that wait together for the same problem are
    solved as one block: the executor sees their directions concatenated, and
    each result holds exactly its own directions' far field."""
    reqs = I.request_stream(30, rate=1000.0, seed=5, catalog=3, max_dirs=6)
    keys = {(r.seed, r.m, r.kappa, r.bc) for r in reqs}
    assert len(keys) == 3
    jobs = []

    def solve(job, slot):
        jobs.append(len(job.dirs))
        time.sleep(0.002)
        info = types.SimpleNamespace(iters=1, matvecs=2 * len(job.dirs), relres_true=0.0,
                                     converged=len(job.dirs))
        return 10, info, job.dirs[:, :2].astype(complex)   # a far field that names its direction

    srv = Server(ServeConfig(slots=1, hbm_budget=10 ** 6, nobs=2, merge_max_dirs=40),
                 solve_fn=solve, estimate_fn=lambda r: 10)
    res = srv.run(reqs, realtime=False)
    assert max(jobs) > 6 and sum(jobs) == sum(len(r.dirs) for r in reqs)
    for r, out in zip(sorted(reqs, key=lambda r: r.rid), res):
        assert np.array_equal(out.uinf, r.dirs[:, :2].astype(complex)) and out.converged == len(r.dirs)
        assert out.batch[0] == r.rid
        assert all((reqs[i].seed, reqs[i].m, reqs[i].kappa, reqs[i].bc) == (r.seed, r.m, r.kappa, r.bc)
                   for i in out.batch)
    assert Server.summary(res, srv.wall)["merged_requests"] > 0
    # merging off: one job per request
    jobs.clear()
    srv = Server(ServeConfig(slots=1, hbm_budget=10 ** 6, nobs=2, merge_max_dirs=0),
                 solve_fn=solve, estimate_fn=lambda r: 10)
    srv.run(reqs, realtime=False)
    assert len(jobs) == len(reqs)
