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
