"""Serving loop on the GPU: requests solved concurrently in the mix give
bitwise the same far fields as each request solved alone."""
import numpy as np
import pytest

pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_each_result_same_alone_and_in_mix():
    from paper_2306_11324_amd import inputs as I
    from paper_2306_11324_amd.serving import ServeConfig, Server
    reqs = I.request_stream(5, rate=50.0, seed=21, m_values=(2, 3), kappa_range=(1.0, 6.0), max_dirs=3)
    print("case: 5 requests m in {2,3}, kappa in [1,6], <= 3 directions, soft/hard, bf16 far field", flush=True)
    cfg = ServeConfig(slots=3, q=6, leaf_depth=1, nobs=16)
    mix = Server(cfg).run(reqs, realtime=False)
    assert all(r.converged == r.uinf.shape[0] and r.relres_true <= 1e-8 for r in mix)
    alone = Server(ServeConfig(slots=1, q=6, leaf_depth=1, nobs=16))
    for r in reqs:
        a = alone.run([r], realtime=False)[0]
        m = mix[r.rid]
        assert np.array_equal(a.uinf, m.uinf), r.rid
    assert {r.bc for r in reqs} == {"soft", "hard"}


def test_larger_requests_same_alone_and_in_mix():
    """Levels 4 and 5 (up to N = 6,936), kappa in [4, 16], up to 13 directions,
    bf16 couplings for soft and hard requests with fp64 refinement, 4 requests
    in 3 slots: each far field bitwise the same alone and in the mix."""
    from paper_2306_11324_amd import inputs as I
    from paper_2306_11324_amd.serving import ServeConfig, Server
    reqs = I.request_stream(4, rate=50.0, seed=30, m_values=(4, 5), kappa_range=(4.0, 16.0), max_dirs=16)
    print("case: 4 requests m in {4,5}, kappa in [4,16], <= 13 directions, soft/hard bf16", flush=True)
    assert {r.bc for r in reqs} == {"soft", "hard"} and any(r.m == 5 and r.bc == "hard" for r in reqs)
    cfg = dict(q=6, leaf_depth=2, nobs=16)
    mix = Server(ServeConfig(slots=3, **cfg)).run(reqs, realtime=False)
    assert all(r.converged == r.uinf.shape[0] and r.relres_true <= 1e-8 for r in mix)
    alone = Server(ServeConfig(slots=1, **cfg))
    for r in reqs:
        a = alone.run([r], realtime=False)[0]
        assert np.array_equal(a.uinf, mix[r.rid].uinf), r.rid


def test_requests_sharing_a_block_match_their_solves_alone():
    """Requests for the same problem (a catalog of 2 problems, levels 3 and 4,
    soft and hard, bf16 couplings with fp64 refinement) that wait together are
    solved as one lockstep block; each far field equals the request's own
    solve within 1e-6 relative (the columns keep their own Krylov bases; the
    block's refinement may take a column one step further than its own solve)."""
    from paper_2306_11324_amd import inputs as I
    from paper_2306_11324_amd.serving import ServeConfig, Server
    reqs = I.request_stream(6, rate=50.0, seed=8, catalog=2, m_values=(3, 4), kappa_range=(2.0, 8.0), max_dirs=4)
    print("case: 6 requests, catalog of 2 problems, m in {3,4}, kappa in [2,8], <= 4 directions, bf16", flush=True)
    cfg = dict(q=6, leaf_depth=1, nobs=16)
    mix = Server(ServeConfig(slots=2, **cfg)).run(reqs, realtime=False)
    assert any(len(r.batch) > 1 for r in mix)
    assert all(r.converged == r.uinf.shape[0] and r.relres_true <= 1e-8 for r in mix)
    alone = Server(ServeConfig(slots=1, merge_max_dirs=0, **cfg))
    worst = 0.0
    for r in reqs:
        a = alone.run([r], realtime=False)[0]
        m = mix[r.rid]
        worst = max(worst, float(np.abs(a.uinf - m.uinf).max() / np.abs(a.uinf).max()))
    print(f"largest far-field difference, in a block vs alone: {worst:.2e}", flush=True)
    assert worst <= 1e-6
