"""Continuous-batching request loop over the batched engine.

Requests (Helmholtz instances) arrive over time.  Between engine ticks the
loop admits waiting requests into free engine slots while the engine's device
pool can hold their footprint (the engine answers FK_ENOMEM / FK_EBUSY
otherwise and the request keeps waiting), so requests that arrive while
others are on the GPU join the next tick and share its persistent launch.
Each tick advances every resident instance by one fixed-point iteration
(Sec. 1 eq. (1.4) with alpha = k^2); an instance retires when its sup-norm
change falls below tol (the control of Sec. 3), when the change is down to
Monte Carlo noise (``settled``), when it diverges, or at max_iters.

With fresh paths every iteration (Remark 2.1) the change never reaches a
small tol: once the deterministic contraction has died out it is the noise
of two independent estimates.  The engine reports R = mean over nodes of
|du|^2 / (2 |SE|^2).  Noise alone (e_{n+1} = K e_n + xi, xi fresh each
iteration) gives R between 1/(1 + rho) and 1 -- near 1 in practice, since
independent per-node noise lies mostly in modes that K barely propagates --
and a deterministic change d adds |d|^2 / (2 SE^2).  An instance settles
when R < 9/8: the remaining deterministic change is below about half a
standard error (root mean square over the nodes).  Requests whose
predicted contraction ratio k^2 / lambda_1 is too close to one are rejected
at admission: the iteration cannot converge there (Sec. 2.4).

Latency = completion time - arrival time.  The engine is deterministic per
instance, so each result is bit-identical to the same request solved alone.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional

import numpy as np

BGK_BETA = 0.5825971579390106   # -zeta(1/2) / sqrt(2 pi)


# ------------------------------------------------------------- predictors

_lambda_cache: Dict[tuple, float] = {}


def lambda1(p) -> float:
    """First Dirichlet eigenvalue of -Delta on the problem's domain.
    Rectangle: pi^2 (1/a^2 + 1/b^2).  Rectangle minus a disc: smallest
    eigenvalue of the 5-point Laplacian on a 97 x 97 grid of the domain
    (sparse shift-invert), cached per geometry."""
    a, b = p.x1 - p.x0, p.y1 - p.y0
    if p.domain_kind == "rect":
        return math.pi ** 2 * (1 / a ** 2 + 1 / b ** 2)
    key = (round(p.x0, 12), round(p.x1, 12), round(p.y0, 12), round(p.y1, 12),
           round(p.cx, 12), round(p.cy, 12), round(p.r, 12))
    if key not in _lambda_cache:
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        n = 97
        xs = np.linspace(p.x0, p.x1, n)
        ys = np.linspace(p.y0, p.y1, n)
        X, Y = np.meshgrid(xs, ys)
        inside = np.ones((n, n), bool)
        inside[0, :] = inside[-1, :] = inside[:, 0] = inside[:, -1] = False
        inside &= (X - p.cx) ** 2 + (Y - p.cy) ** 2 > p.r ** 2
        idx = -np.ones((n, n), int)
        idx[inside] = np.arange(inside.sum())
        dx, dy = xs[1] - xs[0], ys[1] - ys[0]
        rows, cols, vals = [], [], []
        for j, i in zip(*np.nonzero(inside)):
            r = idx[j, i]
            rows.append(r); cols.append(r); vals.append(2 / dx ** 2 + 2 / dy ** 2)
            for jj, ii, w in ((j, i - 1, dx), (j, i + 1, dx), (j - 1, i, dy), (j + 1, i, dy)):
                if inside[jj, ii]:
                    rows.append(r); cols.append(idx[jj, ii]); vals.append(-1 / w ** 2)
        A = sp.csc_matrix((vals, (rows, cols)))
        _lambda_cache[key] = float(spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0])
    return _lambda_cache[key]


def predicted_rho(p) -> float:
    """Contraction ratio of the iteration as the estimator sees it:
    |alpha + i p| / (lambda_1 + alpha - k^2) (k^2 / lambda_1 without shift or
    damping; the iteration of Sec. 2.2 multiplies the first mode by this), with
    lambda_1 of the domain enlarged by the discrete-monitoring shift
    delta = beta sqrt(2h) (outer boundary out by delta, hole in by delta).
    Absorbing edge only: with a reflecting edge there is no such closed form
    (NaN; the sufficient bound of Theorem 2.3 comes from the estimators
    ``exit_time_problem`` and ``local_time_problem``)."""
    if getattr(p, "reflect", False):
        return math.nan
    d = BGK_BETA * math.sqrt(2 * p.h)
    a, b = p.x1 - p.x0, p.y1 - p.y0
    if p.domain_kind == "rect":
        lam = math.pi ** 2 * (1 / (a + 2 * d) ** 2 + 1 / (b + 2 * d) ** 2)
    else:
        grown = p.replace(x0=p.x0 - d, x1=p.x1 + d, y0=p.y0 - d, y1=p.y1 + d, r=max(p.r - d, 1e-9))
        lam = lambda1(grown)
    alpha = p.k ** 2 if getattr(p, "alpha", None) is None else p.alpha
    return abs(complex(alpha, getattr(p, "damping", 0.0))) / (lam + alpha - p.k ** 2)


SETTLE_RATIO = 1.125


def settled(rep: dict) -> bool:
    """The change of this iteration is down to Monte Carlo noise (see the
    module docstring); never at the first iteration."""
    return rep["n"] >= 2 and rep["noise_ratio"] < SETTLE_RATIO


def exit_time_problem(p, M=1024):
    """The same domain and grid with k = 0, f = -1, g = 0: one Feynman-Kac
    step of it estimates E[tau] at every node (Remark 2.5), whose maximum gives
    the sufficient bound k_*^C = (max E[tau])^(-1/2) (Remark 2.4).  With a
    reflecting edge (g2 = 0 there) it is the mean exit time of the reflected
    diffusion, which Theorem 2.3 uses."""
    from .workloads import BC
    return p.replace(k=0.0, alpha=None, damping=0.0, src_kind="const", src_amp=-1.0 + 0j, outer=BC("zero"),
                     inner=BC("zero"), M=M, crn=False, max_iters=1, tol=0.0)


def kstar_cavity(exit_times: np.ndarray, damping: float = 0.0) -> float:
    """k_*^C = sqrt(1 / max E[tau] - p) from an exit-time map (eq. (2.9)): the
    largest k for which the sufficient condition (alpha + p) E[tau] < 1 of
    Theorem 2.2 can hold with alpha >= k^2; 0 when even k = 0 fails it."""
    v = 1.0 / float(np.max(exit_times)) - damping
    return math.sqrt(v) if v > 0 else 0.0


def local_time_problem(p, M=1024):
    """For a reflecting edge: the same domain and grid with k = 0, f = 0,
    u = 0 on the hole and Robin datum g2 = 1 (d_n L = 1 on the edge): one
    Feynman-Kac step of it estimates the mean local time E[xi] on the edge at
    every node (the remark after Theorem 2.3)."""
    from .workloads import BC
    return p.replace(k=0.0, alpha=None, damping=0.0, src_kind="zero", outer=BC("bilinear", coeffs=(1.0 + 0j, 0j, 0j, 0j)),
                     inner=BC("zero"), M=M, crn=False, max_iters=1, tol=0.0)


def khat_annulus(exit_time, local_time):
    """Largest k with alpha = k^2 meeting alpha E[tau] + k E[xi] < 1 at a
    point: (-E[xi] + sqrt(E[xi]^2 + 4 E[tau])) / (2 E[tau]) (the remark after
    Theorem 2.3); k_*^A is its minimum over the domain."""
    E = np.asarray(exit_time, dtype=float)
    L = np.asarray(local_time, dtype=float)
    return (-L + np.sqrt(L * L + 4.0 * E)) / (2.0 * E)


def theorem23_bound(p, sup_exit_time, sup_local_time) -> float:
    """alpha sup E[tau] + k sup E[xi]: below one, the annular iteration
    converges (Theorem 2.3, a sufficient condition)."""
    alpha = p.k ** 2 if getattr(p, "alpha", None) is None else p.alpha
    return alpha * sup_exit_time + p.k * sup_local_time


# ----------------------------------------------------------------- server

def grid_cuts(n: int, spacing: int = 32) -> list:
    """Interface lines every ``spacing`` nodes of an n-node grid side for the
    probabilistic domain decomposition (blocks of spacing - 1 nodes, at most
    64: the device block solver's limit)."""
    if not 2 <= spacing <= 65:
        raise ValueError("spacing must be in [2, 65]")
    return list(range(spacing, n - 1, spacing))


@dataclass
class Request:
    rid: int
    arrival: float              # seconds after the start of the run
    problem: object             # or None with ``make`` given
    seed_note: str = ""
    make: Optional[Callable[[], object]] = None   # builds the problem when first needed
    # probabilistic domain decomposition (cuts_x, cuts_y), or None: paths
    # from every unknown node
    pdd: Optional[tuple] = None

    def get_problem(self):
        if self.problem is None and self.make is not None:
            self.problem = self.make()
        return self.problem


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = math.nan
    completed: float = math.nan
    iterations: int = 0
    outcome: str = ""           # converged | max_iters | diverged | rejected
    rho: float = math.nan
    u: Optional[np.ndarray] = None
    se: Optional[np.ndarray] = None
    admitted_tick: int = -1
    path_steps: int = 0

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class Server:
    """Drives an engine (``fkh.Engine`` or any object with add / tick / get /
    remove) with a stream of requests in wall-clock time."""

    def __init__(self, engine, rho_max: float = 0.98, keep_results: bool = True,
                 clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep,
                 max_queue: Optional[int] = None, on_tick: Optional[Callable[[dict], None]] = None,
                 log_path: Optional[str] = None, tuner=None):
        self.engine = engine
        # launch parameters per request shape (item size, gather layout) from
        # the autotuner, or the library's own choice; results never depend on them
        self.tuner = tuner
        self.rho_max = rho_max
        self.keep = keep_results
        self.clock = clock
        self.sleep = sleep
        self.max_queue = max_queue      # waiting requests beyond this are turned away (queue_full)
        self.on_tick = on_tick
        self.ticks = 0
        self.tick_log: List[dict] = []
        # JSON lines of ticks and finished requests (FKH_LOG names the file)
        self.log_path = log_path if log_path is not None else os.environ.get("FKH_LOG")
        self._log = None

    def _emit(self, rec: dict):
        if self.log_path:
            if self._log is None:
                self._log = open(self.log_path, "a")
            self._log.write(json.dumps(rec) + "\n")
            self._log.flush()

    def run(self, requests: List[Request], horizon: Optional[float] = None) -> Dict[int, Result]:
        pending = sorted(requests, key=lambda r: r.arrival)
        results = {r.rid: Result(r.rid, r.arrival) for r in pending}
        queue: List[Request] = []          # arrived, waiting for a slot / memory
        resident: Dict[int, Request] = {}  # slot -> request
        t0 = self.clock()
        i = 0
        while i < len(pending) or queue or resident:
            now = self.clock() - t0
            while i < len(pending) and pending[i].arrival <= now:
                queue.append(pending[i])
                i += 1
            if horizon is not None and now > horizon and not resident:
                break
            # admission between ticks: FIFO, skipping requests that do not fit
            # yet (no scan while every engine slot is taken)
            still = []
            cap = getattr(self.engine, "max_instances", None)
            for qi, req in enumerate(queue):
                if cap is not None and len(resident) >= cap:
                    still.extend(queue[qi:])
                    break
                res = results[req.rid]
                if math.isnan(res.rho):
                    res.rho = predicted_rho(req.get_problem())
                if res.rho >= self.rho_max:
                    res.outcome = "rejected"
                    res.completed = self.clock() - t0
                    continue
                try:
                    cfg = self.tuner.instance_config(req.get_problem()) if self.tuner is not None else {}
                    slot = self.engine.add(req.get_problem(), **cfg)
                    if slot is not None and req.pdd is not None and not self.engine.set_pdd(slot, *req.pdd):
                        self.engine.remove(slot)      # its block data do not fit now
                        slot = None
                except ValueError as ex:       # invalid problem description
                    res.outcome = "invalid: %s" % ex
                    res.completed = self.clock() - t0
                    continue
                if slot is None:
                    if not resident:        # does not fit even into an empty engine
                        res.outcome = "too_large"
                        res.completed = self.clock() - t0
                        continue
                    still.append(req)
                    continue
                resident[slot] = req
                res.admitted = self.clock() - t0
                res.admitted_tick = self.ticks
            queue = still
            if self.max_queue is not None and len(queue) > self.max_queue:
                # the waiting room is full: the latest arrivals are turned away
                for req in queue[self.max_queue:]:
                    res = results[req.rid]
                    res.outcome = "queue_full"
                    res.completed = self.clock() - t0
                queue = queue[:self.max_queue]
            if not resident:
                if i < len(pending):
                    wait = pending[i].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(wait)
                continue
            reps = self.engine.tick()
            self.ticks += 1
            now = self.clock() - t0
            self.tick_log.append(dict(tick=self.ticks, t=now, resident=len(resident), queued=len(queue),
                                      arrived=i))
            if self.log_path:
                self._emit(dict(event="tick", **self.tick_log[-1],
                                path_steps=int(sum(r.get("path_steps", 0) for r in reps.values())),
                                step_ms=max((r.get("step_ms", 0.0) for r in reps.values()), default=0.0)))
            if self.on_tick is not None:
                self.on_tick(self.tick_log[-1])
            for slot, rep in reps.items():
                req = resident.get(slot)
                if req is None:
                    continue
                res = results[req.rid]
                res.iterations = rep["n"]
                res.path_steps += rep["path_steps"]
                p = req.get_problem()
                done = None
                if rep["diverging"]:
                    done = "diverged"
                elif rep["max_du"] < p.tol or settled(rep):
                    done = "converged"
                elif rep["n"] >= p.max_iters:
                    done = "max_iters"
                if done:
                    if self.keep:
                        res.u, res.se = self.engine.get(slot)
                    self.engine.remove(slot)
                    del resident[slot]
                    res.outcome = done
                    res.completed = now
                    self._emit(dict(event="done", rid=res.rid, outcome=done, iterations=res.iterations,
                                    arrival=res.arrival, admitted=res.admitted, completed=res.completed,
                                    latency=res.latency, path_steps=res.path_steps))
        for r in results.values():
            if r.outcome in ("rejected", "queue_full", "too_large") or r.outcome.startswith("invalid"):
                self._emit(dict(event="turned_away", rid=r.rid, outcome=r.outcome, arrival=r.arrival))
        if self._log is not None:
            self._log.close()
            self._log = None
        return results


def latency_summary(results: Dict[int, Result], wall: float, tick_log: Optional[List[dict]] = None) -> dict:
    """Completed solves (converged, max_iters or diverged), their p50 / p99
    latency, solves/s over the wall time, turned-away requests by reason and,
    given the tick log, the growth of the waiting queue (requests per second,
    least-squares slope while requests were still arriving)."""
    vals = list(results.values())
    done = [r for r in vals if r.outcome in ("converged", "max_iters", "diverged")]
    lat = np.array([r.latency for r in done]) if done else np.array([math.nan])
    out = dict(completed=len(done), rejected=sum(r.outcome == "rejected" for r in vals),
               queue_full=sum(r.outcome == "queue_full" for r in vals),
               too_large=sum(r.outcome == "too_large" for r in vals),
               diverged=sum(r.outcome == "diverged" for r in vals),
               max_iters=sum(r.outcome == "max_iters" for r in vals),
               p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
               solves_per_s=len(done) / wall if wall > 0 else math.nan,
               path_steps=int(sum(r.path_steps for r in done)))
    if tick_log:
        last_arrival = max(r.arrival for r in vals)
        pts = [(t["t"], t["queued"]) for t in tick_log if t["t"] <= last_arrival]
        out["queue_growth_per_s"] = (float(np.polyfit([a for a, _ in pts], [b for _, b in pts], 1)[0])
                                     if len(pts) >= 2 else None)
    return out
