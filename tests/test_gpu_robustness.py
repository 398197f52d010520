"""GPU: checkpoint / resume, cancellation and fault isolation.

- Checkpoint / resume: an iterate read with ``get`` and loaded into a new
  solver (``set_iterate``) continues bit for bit as the uninterrupted run
  (the random numbers depend only on (seed, n, node, m, t), the iterate is
  the whole state).
- Cancellation: ``fk_helmholtz_cancel`` from another thread stops a running
  solve before its next iteration with FK_ECANCELLED; the iterate is the last
  completed one and the run continues bit for bit.
- Fault isolation in the batched engine: a diverging instance (k above
  k_max, common random numbers) and an instance whose iterate is overwritten
  with NaN run in one launch with converging instances; the latter stay
  bit-identical to their runs alone, the former are reported (non-finite /
  diverging).
- The engine's per-node exit-step sums are bit-exact against the oracle.
"""
import threading
import time

import numpy as np
import pytest

from oracle import fkmc
from paper_2308_11469_amd import fkh
from paper_2308_11469_amd import workloads as W

from gpu_util import require_lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    require_lib()


@pytest.mark.parametrize("precision", [64, 32])
def test_checkpoint_resume_bit_identical(precision):
    p = W.cavity_source(precision=precision).replace(nx=33, ny=29, x1=1.2, M=384, h=1e-3)
    s = fkh.Solver(p)
    s.iterate(5)
    ref, ref_se = s.get()
    s.close()
    a = fkh.Solver(p)
    a.iterate(3)
    ckpt, _ = a.get()
    a.close()
    b = fkh.Solver(p)
    b.set_iterate(ckpt, 3)
    rep = b.iterate(2)
    got, got_se = b.get()
    b.close()
    say("checkpoint/resume", precision, rep["n"])
    assert rep["n"] == 5
    assert np.array_equal(got, ref) and np.array_equal(got_se, ref_se)


def test_cancel_stops_a_running_solve_and_resumes():
    p = W.cavity_small().replace(M=128, max_iters=100000, tol=0.0)
    s = fkh.Solver(p)
    out = {}

    def run():
        out["rep"] = s.solve()

    th = threading.Thread(target=run)
    th.start()
    time.sleep(0.5)
    s.cancel()
    th.join(timeout=120)
    assert not th.is_alive()
    rep = out["rep"]
    n = rep["n"]
    say("cancelled after", n, "iterations:", rep["status"])
    assert rep["status"] == "FK_ECANCELLED" and 0 < n < 100000
    # the request is consumed: the run continues, bit for bit as without it
    s.iterate(2)
    got, _ = s.get()
    s.close()
    r = fkh.Solver(p)
    r.iterate(n + 2)
    ref, _ = r.get()
    r.close()
    assert np.array_equal(got, ref)


def test_cancel_before_a_call_is_consumed_by_it():
    p = W.cavity_small().replace(M=64, max_iters=3)
    s = fkh.Solver(p)
    s.cancel()
    rep = s.solve()
    assert rep["status"] == "FK_ECANCELLED" and rep["n"] == 0
    rep = s.solve()
    assert rep["status"] == "FK_OK" and rep["n"] == 3
    s.close()


def _mates(precision):
    a = W.cavity_small().replace(precision=precision, M=320)
    b = W.scatter_problem(k=2.0, theta=1.0, N=25, M=192, seed=5007, precision=precision, h=2e-3, table_len=2048)
    c = W.cavity_source(precision=precision).replace(nx=17, ny=13, M=128, h=2e-3)
    return [a, b, c]


def _engine(precision, n=8):
    return fkh.Engine(n, precision=precision, max_grid_nodes=1 << 16, max_items=1 << 16, max_table=1 << 14,
                      max_instance_nodes=4096)


def _alone(p, ticks, precision):
    e = _engine(precision)
    sl = e.add(p)
    for _ in range(ticks):
        e.tick()
    u = e.get(sl)[0]
    e.close()
    return u


@pytest.mark.parametrize("precision", [64, 32])
def test_diverging_and_nan_instances_do_not_touch_batch_mates(precision):
    ticks = 10
    mates = _mates(precision)
    # k = 4.6 > pi sqrt(2) with common random numbers: the change grows by
    # about 1.1 per iteration on the 9 x 9 cavity
    div = W.cavity_small().replace(precision=precision, k=4.6, crn=True, M=256, seed=77, name="diverging")
    nan = W.cavity_small().replace(precision=precision, M=192, seed=78, name="nan")
    e = _engine(precision)
    slots = [e.add(p) for p in mates]
    sd = e.add(div)
    sn = e.add(nan)
    reps = {}
    for t in range(ticks):
        if t == 2:
            u, _ = e.get(sn)
            u[4, 4] = complex(float("nan"), 0.0)
            e.set_iterate(sn, u, 2)
        reps[t] = e.tick()
    got = [e.get(s)[0] for s in slots]
    e.close()
    say("engine faults", precision, "diverging:", [reps[t][sd]["diverging"] for t in range(ticks)],
        "nan nonfinite:", [reps[t][sn]["nonfinite"] for t in range(ticks)])
    assert reps[2][sn]["nonfinite"] > 0 and reps[2][sn]["diverging"] == 1
    # the diverging instance's change grows tick over tick once the
    # transient of the first iterations is gone
    assert reps[ticks - 1][sd]["max_du"] > 1.15 * reps[ticks - 3][sd]["max_du"]
    for p, g in zip(mates, got):
        assert np.array_equal(g, _alone(p, ticks, precision)), p.name or p.nx


def test_engine_exit_step_sums_bit_exact_against_oracle():
    p = W.scatter_problem(k=2.0, theta=0.5, N=21, M=160, seed=5011, precision=64, h=2e-3, table_len=2048)
    e = _engine(64)
    sl = e.add(p)
    ids = fkmc.interior_ids(p)
    u_prev = None
    for it in range(2):
        e.tick()
        u, _ = e.get(sl)
        sj, cp = e.node_stats(sl)
        orc = fkmc.fk_nodes(p, u_prev, it, ids)
        assert np.array_equal(sj[ids], orc["sumJ"]) and np.array_equal(cp[ids], orc["capped"])
        assert np.max(np.abs(u.ravel()[ids] - orc["mean"])) < 1e-11
        u_prev = u
    e.close()
