"""Continuous-batching server: each result equals the same solve run alone
(bit for bit), requests overlap on several streams, and a request larger
than the HBM budget is refused."""
import numpy as np
import pytest

from paper_2508_02626_amd import inputs
from gpu_util import say

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    from paper_2508_02626_amd import serve
    reqs = []
    for i in range(14):
        rng = np.random.default_rng(500 + i)
        n = int(rng.integers(800, 30_000))
        x, q = (inputs.uniform if i % 2 else inputs.plummer)(n, 600 + i)
        reqs.append((x, q, [1e-4, 1e-7, 1e-9][i % 3]))
    srv = serve.Server(hbm_budget_bytes=8 << 30, slots=3, pack_threshold=20_000, max_pack=8)
    futs = [srv.submit(x, q, e) for x, q, e in reqs]
    outs = [f.result(timeout=120) for f in futs]
    srv.close()
    for (x, q, e), (phi, fld, lat) in zip(reqs, outs):
        a_phi, a_fld = serve.solve_alone(x, q, e)
        assert np.array_equal(phi, a_phi) and np.array_equal(fld, a_fld)
        assert lat > 0
    say("  served %d requests, latencies ms:" % len(outs), [round(1e3 * o[2], 1) for o in outs])


def test_request_over_budget_is_refused():
    from paper_2508_02626_amd import serve
    srv = serve.Server(hbm_budget_bytes=1 << 20, slots=1)
    x, q = inputs.uniform(50_000, 1)
    f = srv.submit(x, q, 1e-7)
    with pytest.raises(MemoryError):
        f.result(timeout=10)
    srv.close()
