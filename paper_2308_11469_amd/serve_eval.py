"""Serving evaluation on the scattering request stream.

The stream: plane waves with k ~ U[1, 4] and theta ~ U[0, 2 pi) scattered by
the sound-soft disc r = 0.25 at the origin inside [-1, 1]^2 (outer data from
the exact disc series), grids N x N with N ~ U{33..257}, M log-uniform on
[1024, 8192], h = 1e-4, FP32 stepping, Poisson arrivals.  Requests go through
the continuous-batching server over the batched engine with a bounded
waiting queue; a request is turned away at admission when its predicted
contraction ratio is too close to one, or when the waiting queue is full.

    python -m paper_2308_11469_amd.serve_eval [--requests 400] [--rate 200]
        [--max-queue 32] [--slots 8] [--sweep 0.25,0.5,0.8] [--sweep-requests 24]

Prints one JSON line per run: completed solves/s, p50 / p99 latency of the
completed requests, turned-away counts by reason and the queue growth rate.
With --sweep, further runs offer the stream at the given fractions of the
capacity measured by the first run (its completed solves/s).
"""
import argparse
import json
import sys
import time

from . import fkh, serving
from . import workloads as W


def build_requests(n, rate, seed=5):
    """The stream's requests; each problem (with its boundary table from the
    disc series) is built when the server first looks at the request, so
    requests turned away at a full queue cost nothing."""
    arrivals, params = W.scatter_stream(n, rate, seed)
    reqs = []
    for r, (t, q) in enumerate(zip(arrivals, params)):
        make = (lambda q=q: W.scatter_problem(q["k"], q["theta"], q["N"], q["M"], q["seed"], precision=32))
        reqs.append(serving.Request(r, float(t), None, make=make))
    return reqs


def run_window(n, rate, max_queue, slots, seed=5, log=None):
    reqs = build_requests(n, rate, seed)
    eng = fkh.Engine(slots, precision=32, max_grid_nodes=slots * 257 * 257, max_items=1 << 26,
                     max_table=slots * 4 * 8192, max_instance_nodes=257 * 257)
    last = [time.perf_counter()]

    def progress(entry):
        now = time.perf_counter()
        if log is not None and now - last[0] > 10.0:
            last[0] = now
            print("  tick %d t=%.1fs resident=%d queued=%d arrived=%d" % (
                entry["tick"], entry["t"], entry["resident"], entry["queued"], entry["arrived"]),
                file=log, flush=True)

    srv = serving.Server(eng, keep_results=False, max_queue=max_queue, on_tick=progress)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    eng.close()
    out = serving.latency_summary(res, wall, srv.tick_log)
    out.update(requests=n, offered_rate_per_s=rate, max_queue=max_queue, slots=slots, wall_s=wall,
               ticks=srv.ticks, max_resident=max((t["resident"] for t in srv.tick_log), default=0),
               iterations_per_solve_median=float(_median([r.iterations for r in res.values()
                                                          if r.outcome in ("converged", "max_iters")])))
    return out


def _median(v):
    v = sorted(v)
    if not v:
        return float("nan")
    m = len(v) // 2
    return v[m] if len(v) % 2 else 0.5 * (v[m - 1] + v[m])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--max-queue", type=int, default=32)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--sweep", default="", help="comma-separated fractions of the measured capacity")
    ap.add_argument("--sweep-requests", type=int, default=24)
    a = ap.parse_args(argv)
    first = run_window(a.requests, a.rate, a.max_queue, a.slots, log=sys.stderr)
    first["run"] = "offered"
    print(json.dumps(first), flush=True)
    cap = first["solves_per_s"]
    for f in [float(x) for x in a.sweep.split(",") if x.strip()]:
        out = run_window(a.sweep_requests, f * cap, a.max_queue, a.slots, log=sys.stderr)
        out.update(run="sweep", capacity_fraction=f, capacity_solves_per_s=cap)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
