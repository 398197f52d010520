"""Serving loop logic on the CPU with a scripted stand-in engine (a test
fixture, not a product path): admission by slots and by device-pool
footprint, FIFO order, rejection by predicted contraction ratio, requests
admitted while others are resident (continuous batching), retirement rules
and latency accounting on a virtual clock."""
import math

import numpy as np
import pytest

from paper_2308_11469_amd import serving
from paper_2308_11469_amd import workloads as W


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class ScriptedEngine:
    """Slots and a byte pool like the real engine; each instance reports
    max_du = 0.5^n and a noise ratio of 0.9 + 20 * 0.5^n, which settles
    (below 9/8) after 7 ticks unless max_iters stops it first.  A tick costs `dt` virtual seconds."""

    def __init__(self, clock, slots=3, pool=10_000, dt=0.05):
        self.clock, self.slots, self.pool, self.dt = clock, slots, pool, dt
        self.res = {}
        self.log = []

    def footprint(self, p):
        return p.nx * p.ny

    def add(self, p):
        used = sum(self.footprint(q) for q, _ in self.res.values())
        if len(self.res) >= self.slots or used + self.footprint(p) > self.pool:
            return None
        slot = min(set(range(self.slots)) - set(self.res))
        self.res[slot] = (p, 0)
        self.log.append(("add", slot, p.name))
        return slot

    def tick(self):
        self.clock.t += self.dt
        out = {}
        for s, (p, n) in list(self.res.items()):
            n += 1
            self.res[s] = (p, n)
            out[s] = dict(n=n, max_du=0.5 ** n, noise_floor=0.01, noise_ratio=0.9 + 20 * 0.5 ** n,
                          diverging=int(p.k > 100), path_steps=1000)
        return out

    def get(self, slot):
        p, n = self.res[slot]
        return np.full((p.ny, p.nx), n + 0j), np.zeros((p.ny, p.nx), complex)

    def remove(self, slot):
        del self.res[slot]
        self.log.append(("remove", slot))

    def set_pdd(self, slot, cx, cy):
        # block data of a decomposition: fits while the pool has room for it
        p, n = self.res[slot]
        used = sum(self.footprint(q) for q, _ in self.res.values())
        ok = used + len(cx) + len(cy) <= self.pool
        self.log.append(("set_pdd", slot, tuple(cx), tuple(cy), ok))
        return ok


def req(rid, t, N=40, k=1.0, max_iters=40):
    p = W.Problem(name="r%d" % rid, nx=N, ny=N, k=k, h=1e-4, M=64, max_iters=max_iters, tol=0.0)
    return serving.Request(rid, t, p)


def run(reqs, **kw):
    clk = VirtualClock()
    eng = ScriptedEngine(clk, **kw)
    srv = serving.Server(eng, clock=clk, sleep=clk.sleep)
    return srv, eng, srv.run(reqs)


def test_all_complete_with_latency_accounting():
    reqs = [req(i, 0.01 * i) for i in range(8)]
    srv, eng, res = run(reqs)
    for r in res.values():
        assert r.outcome == "converged" and r.iterations == 7
        assert r.completed >= r.admitted >= r.arrival
        assert math.isclose(r.latency, r.completed - r.arrival)
    s = serving.latency_summary(res, wall=max(r.completed for r in res.values()))
    assert s["completed"] == 8 and s["p99_s"] >= s["p50_s"] > 0


def test_slot_limit_and_continuous_batching():
    reqs = [req(i, 0.0) for i in range(3)] + [req(3, 0.12), req(4, 0.13)]
    srv, eng, res = run(reqs, slots=3)
    # requests 3 and 4 arrive while 0..2 are resident: they wait for slots and
    # are admitted between ticks as soon as retirements free them
    assert res[3].admitted_tick == 7 and res[4].admitted_tick == 7
    assert all(res[i].admitted_tick == 0 for i in range(3))
    # a request arriving mid-flight joins while others are still resident
    reqs = [req(0, 0.0), req(1, 0.12)]
    srv, eng, res = run(reqs, slots=3)
    assert res[1].admitted_tick in (2, 3) and res[0].completed > res[1].admitted


def test_admission_by_pool_footprint_fifo():
    # two 60x60 instances do not fit a 5000-byte pool together; the small one
    # behind them in the queue is admitted first (does not block on the head)
    reqs = [req(0, 0.0, N=60), req(1, 0.0, N=60), req(2, 0.0, N=20)]
    srv, eng, res = run(reqs, pool=5000)
    assert res[0].admitted_tick == 0 and res[2].admitted_tick == 0
    assert res[1].admitted_tick == 7


def test_too_large_and_rejected_by_rho():
    too_big = req(0, 0.0, N=200)
    divergent = req(1, 0.0, k=4.6)          # unit square: k^2 > lambda_1
    ok = req(2, 0.0, k=2.0)
    srv, eng, res = run([too_big, divergent, ok], pool=5000)
    assert res[0].outcome == "too_large"
    assert res[1].outcome == "rejected" and res[1].rho > 1
    assert res[2].outcome == "converged"


def test_bounded_queue_turns_away_and_reports_growth():
    # 3 slots, queue of 2: of 10 simultaneous arrivals 3 are admitted, 2 wait,
    # 5 are turned away at arrival; the waiting ones are served later
    reqs = [req(i, 0.0) for i in range(10)]
    clk = VirtualClock()
    eng = ScriptedEngine(clk, slots=3)
    ticks = []
    srv = serving.Server(eng, clock=clk, sleep=clk.sleep, max_queue=2, on_tick=ticks.append)
    res = srv.run(reqs)
    out = [res[i].outcome for i in range(10)]
    assert out.count("queue_full") == 5 and out.count("converged") == 5
    assert all(res[i].outcome == "queue_full" for i in range(5, 10))
    assert ticks == srv.tick_log and ticks[0]["arrived"] == 10
    s = serving.latency_summary(res, wall=clk.t, tick_log=srv.tick_log)
    assert s["queue_full"] == 5 and s["completed"] == 5
    # a stream arriving faster than it is served: the queue grows
    reqs = [req(i, 0.02 * i) for i in range(30)]
    clk = VirtualClock()
    srv = serving.Server(ScriptedEngine(clk, slots=1), clock=clk, sleep=clk.sleep)
    res = srv.run(reqs)
    s = serving.latency_summary(res, wall=clk.t, tick_log=srv.tick_log)
    assert s["queue_growth_per_s"] > 10


def test_max_iters_and_divergence_retire():
    reqs = [req(0, 0.0, max_iters=3)]
    srv, eng, res = run(reqs)
    assert res[0].outcome == "max_iters" and res[0].iterations == 3
    srv = serving.Server(ScriptedEngine(VirtualClock()), rho_max=1e9)
    eng = srv.engine
    srv.clock = eng.clock
    srv.sleep = eng.clock.sleep
    out = srv.run([req(0, 0.0, k=200.0)])
    assert out[0].outcome == "diverged"


def test_settled_rule():
    assert not serving.settled(dict(n=1, noise_ratio=0.0))      # first change is the iterate itself
    assert serving.settled(dict(n=2, noise_ratio=1.1))
    assert not serving.settled(dict(n=5, noise_ratio=1.2))


def test_predicted_rho_rectangle_and_disc():
    p = W.cavity_65(k=4.0)
    rho = serving.predicted_rho(p)
    assert 0.8 < rho < 0.84                   # k^2 / lambda_1 of the BGK-enlarged square
    assert serving.predicted_rho(p.replace(k=4.6)) > 1
    # with a shift and damping: |alpha + i p| / (lambda_1 + alpha - k^2)
    lam_sq = serving.predicted_rho(p.replace(k=1.0)) ** -1
    g = p.replace(k=1.0, alpha=4.0, damping=3.0)
    assert serving.predicted_rho(g) == pytest.approx(5.0 / (lam_sq + 3.0))
    q = W.scatter_problem(k=3.0, theta=0.0, N=65, M=64, seed=1, h=1e-4, table_len=64)
    lam = serving.lambda1(q)
    assert 12.5 < lam < 13.5                  # [-1,1]^2 minus the r = 0.25 disc
    assert serving.predicted_rho(q.replace(k=3.7)) > 0.98


def test_pdd_requests_get_their_cuts_and_wait_when_they_do_not_fit():
    a = req(0, 0.0)
    a.pdd = ([10, 20], [15])
    b = req(1, 0.0)
    srv, eng, res = run([a, b])
    assert ("set_pdd", 0, (10, 20), (15,), True) in eng.log
    assert all(e[0] != "set_pdd" or e[1] == 0 for e in eng.log)
    assert res[0].outcome == res[1].outcome == "converged"
    # a decomposition that does not fit: the instance is taken out again and
    # the request keeps waiting (here until nothing else is resident)
    c = req(2, 0.0, N=70)
    c.pdd = (list(range(1, 3000)), [])
    d = req(3, 0.0, N=40)
    srv, eng, res = run([d, c], pool=8000)
    assert ("set_pdd", 1, tuple(range(1, 3000)), (), False) in eng.log and ("remove", 1) in eng.log
    assert res[2].admitted_tick == 7 and res[2].outcome == "converged"


def test_grid_cuts():
    assert serving.grid_cuts(129, 32) == [32, 64, 96]
    assert serving.grid_cuts(33, 32) == []
    assert serving.grid_cuts(34, 32) == [32]
    with pytest.raises(ValueError):
        serving.grid_cuts(129, 80)


def test_jsonl_log_of_ticks_and_requests(tmp_path):
    import json
    path = tmp_path / "serve.jsonl"
    clk = VirtualClock()
    eng = ScriptedEngine(clk, slots=2)
    srv = serving.Server(eng, clock=clk, sleep=clk.sleep, log_path=str(path))
    res = srv.run([req(i, 0.0) for i in range(3)] + [req(9, 0.0, k=4.6)])
    recs = [json.loads(ln) for ln in path.read_text().splitlines()]
    ticks = [r for r in recs if r["event"] == "tick"]
    done = [r for r in recs if r["event"] == "done"]
    away = [r for r in recs if r["event"] == "turned_away"]
    assert len(ticks) == srv.ticks and ticks[0]["resident"] == 2 and ticks[0]["path_steps"] == 2000
    assert sorted(r["rid"] for r in done) == [0, 1, 2] and all(r["iterations"] == 7 for r in done)
    assert [r["rid"] for r in away] == [9] and away[0]["outcome"] == "rejected"
    assert all(math.isclose(r["latency"], res[r["rid"]].latency) for r in done)


def test_tuner_sets_the_launch_parameters_of_admitted_instances():
    class Tuner:
        def instance_config(self, p):
            return {"paths_per_item": 128, "gather_layout": "cells"}

    class Eng(ScriptedEngine):
        def add(self, p, **cfg):
            self.log.append(("cfg", cfg))
            return super().add(p)

    clk = VirtualClock()
    eng = Eng(clk)
    srv = serving.Server(eng, clock=clk, sleep=clk.sleep, tuner=Tuner())
    res = srv.run([req(0, 0.0), req(1, 0.0)])
    assert [e for e in eng.log if e[0] == "cfg"] == [("cfg", {"paths_per_item": 128, "gather_layout": "cells"})] * 2
    assert all(r.outcome == "converged" for r in res.values())
