"""Autotuner of the path kernel's launch parameters.

Three parameters change the speed of the stepping kernel but not its results
(node sums are exact integers, so any split of the paths gives bit-identical
iterates):

- ``paths_per_item`` (P): paths per work item.  Small items balance better,
  large ones mean fewer queue fetches and fewer node-accumulator flushes;
- ``gather_layout``: row-major or cell-major copy of u_n.  Row-major is
  cheaper while the grid stays in the vector L1 cache, cell-major needs one
  L2 request per step instead of about two once it does not;
- ``waves_per_cu``: resident waves of the persistent launch per CU.

For a problem the tuner times one fixed-point iteration per candidate on a
proxy with the same domain, grid, h, k, data and precision and the number of
paths reduced to ``proxy_paths`` (the path length distribution, which sets
the cost per path, does not depend on M), and keeps the candidate with the
most path-steps per second of device time.  Results are cached in a JSON file
keyed by the shape that matters (precision, domain kind, grid, M bucket),
so a serving loop tunes each shape once.
"""
import json
import math
import os

from . import fkh

PPI = (64, 128, 256, 512, 1024)
AUTO = dict(paths_per_item=0, gather_layout="auto", waves_per_cu=0)   # the library's own choice
WAVES = (8, 12, 16)
LAYOUTS = ("nodes", "cells")


def candidates(problem, ppi=PPI, waves=WAVES):
    """Every (paths_per_item, gather_layout, waves_per_cu) worth timing."""
    mcap = ((int(problem.M) + 63) // 64) * 64
    ps = [p for p in ppi if p <= mcap] or [64]
    return [dict(paths_per_item=p, gather_layout=l, waves_per_cu=w) for p in ps for l in LAYOUTS for w in waves]


def shape_key(problem):
    """Cache key: what changes the best launch parameters (not k, seed or data)."""
    m_bucket = int(round(math.log2(max(int(problem.M), 1))))
    return "p%d/%s/%dx%d/M2^%d/h%.3g" % (int(problem.precision), problem.domain_kind, int(problem.nx),
                                        int(problem.ny), m_bucket, float(problem.h))


def measure_device(problem, cfg, iters=2):
    """Path-steps per second of device time of the path kernel, last of
    ``iters`` iterations (the first one warms caches and the queue)."""
    s = fkh.Solver(problem, **cfg)
    try:
        rep = None
        for _ in range(iters):
            rep = s.iterate(1)
        return rep["path_steps"] / (rep["step_ms"] / 1e3)
    finally:
        s.close()


class Tuner:
    """Times candidates and caches the best per shape.

    ``measure(problem, cfg) -> path-steps/s`` is the timing function (the
    GPU one by default; tests pass their own)."""

    def __init__(self, cache_path=None, proxy_paths=2048, measure=None, ppi=PPI, waves=WAVES):
        self.cache_path = cache_path if cache_path is not None else os.environ.get("FKH_AUTOTUNE_CACHE")
        self.proxy_paths = int(proxy_paths)
        self.measure = measure or measure_device
        self.ppi = tuple(ppi)
        self.waves = tuple(waves)
        self.cache = {}
        if self.cache_path and os.path.exists(self.cache_path):
            with open(self.cache_path) as f:
                self.cache = json.load(f)
        self.timed = 0     # candidates timed by this tuner

    def _save(self):
        if not self.cache_path:
            return
        tmp = self.cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    def best(self, problem):
        """Best launch parameters for the problem's shape (cached).  When the
        proxy has fewer paths than the problem, the proxy's winner is timed
        once more at the full M against the library's own choice, and the
        faster of the two is kept (the item count, and so the balance of the
        launch, depends on M)."""
        key = shape_key(problem)
        hit = self.cache.get(key)
        if hit is not None:
            return dict(hit["config"])
        proxy = problem.replace(M=min(int(problem.M), self.proxy_paths))
        results = []
        for cfg in candidates(proxy, self.ppi, self.waves):
            rate = float(self.measure(proxy, cfg))
            self.timed += 1
            results.append((rate, cfg))
        rate, cfg = max(results, key=lambda rc: rc[0])
        # the library's own choice, for comparison
        default = float(self.measure(proxy, AUTO))
        self.timed += 1
        rec = {"config": cfg, "path_steps_per_s": rate, "auto_path_steps_per_s": default,
               "proxy_paths": int(proxy.M), "candidates": len(results)}
        if int(proxy.M) < int(problem.M):
            full_best = float(self.measure(problem, cfg))
            full_auto = float(self.measure(problem, AUTO))
            self.timed += 2
            rec.update(full_paths=int(problem.M), full_path_steps_per_s=full_best,
                       full_auto_path_steps_per_s=full_auto)
            if full_auto > full_best:
                rec["config"] = dict(AUTO)
                rec["kept"] = "auto at full M"
            cfg = rec["config"]
        self.cache[key] = rec
        self._save()
        return dict(cfg)

    def instance_config(self, problem):
        """The per-instance part of best() (item size and gather layout),
        for admission into the batched engine, whose launch width is its own."""
        cfg = self.best(problem)
        return {"paths_per_item": cfg["paths_per_item"], "gather_layout": cfg["gather_layout"]}
