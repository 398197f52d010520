"""GPU: the continuous-batching loop over the real engine.  Requests of
different domains, grids, k, M and seeds arrive over time; each completed
result is bit-identical to the same request solved alone for the same number
of iterations (the mix does not change any instance's arithmetic)."""
import math

import numpy as np
import pytest

from paper_2308_11469_amd import fkh, serving
from paper_2308_11469_amd import workloads as W

from gpu_util import require_lib, say

pytestmark = pytest.mark.gpu


def stream():
    rng = np.random.default_rng(17)
    reqs = []
    t = 0.0
    for r in range(10):
        t += float(rng.exponential(0.01))
        if r % 3 == 2:
            p = W.scatter_problem(k=float(rng.uniform(1.0, 3.0)), theta=float(rng.uniform(0, 6.28)),
                                  N=int(rng.integers(17, 34)), M=int(64 * rng.integers(2, 6)), seed=5000 + r,
                                  precision=32, h=2e-3, table_len=2048)
        else:
            a, b = float(rng.uniform(0.5, 1.5)), float(rng.uniform(0.5, 1.5))
            c = float(rng.uniform(0.2, 0.8))
            p = W.Problem(name="rect%d" % r, x1=a, y1=b, nx=int(rng.integers(9, 30)), ny=int(rng.integers(9, 30)),
                          k=c * math.pi * math.sqrt(1 / a ** 2 + 1 / b ** 2), h=2e-3, M=int(64 * rng.integers(2, 6)),
                          seed=1000 + r, outer=W.BC("plane_wave", 1.0, float(rng.uniform(0, 6.28))), precision=32)
        p = p.replace(max_iters=12, tol=0.0)
        reqs.append(serving.Request(r, t, p))
    # one request far above k_max: rejected at admission
    bad = W.cavity_small().replace(k=6.0, precision=32, name="divergent")
    reqs.append(serving.Request(99, 0.0, bad))
    return reqs


def test_stream_results_equal_alone_and_batching_happened():
    require_lib()
    eng = fkh.Engine(4, precision=32, max_grid_nodes=1 << 15, max_items=1 << 15, max_table=1 << 13,
                     max_instance_nodes=2048)
    srv = serving.Server(eng)
    reqs = stream()
    res = srv.run(reqs)
    eng.close()
    assert res[99].outcome == "rejected"
    done = [r for r in res.values() if r.rid != 99]
    assert all(r.outcome in ("converged", "max_iters") for r in done), [(r.rid, r.outcome) for r in done]
    # continuous batching: some request joined while others were resident
    assert any(r.admitted_tick > 0 for r in done)
    assert max(t["resident"] for t in srv.tick_log) >= 2
    s = serving.latency_summary(res, wall=max(r.completed for r in done))
    say("serving", s)
    # every result equals the same request alone, iterated the same number of times
    for r in done:
        p = reqs[r.rid].problem
        e1 = fkh.Engine(1, precision=32, max_grid_nodes=1 << 12, max_items=1 << 12, max_table=1 << 12,
                        max_instance_nodes=2048)
        sl = e1.add(p)
        for _ in range(r.iterations):
            e1.tick()
        u, _ = e1.get(sl)
        e1.close()
        assert np.array_equal(u, r.u), r.rid
