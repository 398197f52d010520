"""Host logic of the autotuner: candidate sets, cache keys, the choice of the
fastest candidate and the JSON cache round trip (timing function injected,
no GPU)."""
import json

from paper_2308_11469_amd import autotune
from paper_2308_11469_amd import workloads as W


def test_candidates_cover_the_grid_and_respect_M():
    p32 = W.cavity_65(precision=32)
    c = autotune.candidates(p32)
    assert len(c) == len(autotune.PPI) * 2 * len(autotune.WAVES)
    assert {x["gather_layout"] for x in c} == {"nodes", "cells"}
    p64 = W.cavity_65(precision=64)
    assert {x["gather_layout"] for x in autotune.candidates(p64)} == {"nodes", "cells"}
    small = W.cavity_small().replace(M=100)          # items never exceed M rounded up to 64
    assert max(x["paths_per_item"] for x in autotune.candidates(small)) == 128


def test_shape_key_ignores_k_seed_and_data_but_not_grid():
    a = W.cavity_65(k=1.0)
    assert autotune.shape_key(a) == autotune.shape_key(a.replace(k=3.0, seed=9))
    assert autotune.shape_key(a) != autotune.shape_key(a.replace(nx=129, ny=129))
    assert autotune.shape_key(a) != autotune.shape_key(a.replace(precision=32))


def test_proxy_choice_checked_at_full_m(tmp_path):
    # the proxy prefers 1024-path items, the full problem does not: the
    # library's own choice is kept
    seen = []

    def fake(problem, cfg):
        seen.append((int(problem.M), cfg))
        if cfg == autotune.AUTO:
            return 10.0 if problem.M > 512 else 1.0
        return cfg["paths_per_item"] / (100.0 if problem.M > 512 else 1.0)

    t = autotune.Tuner(cache_path=str(tmp_path / "t.json"), proxy_paths=512, measure=fake)
    p = W.cavity_65(precision=32)
    assert t.best(p) == autotune.AUTO
    assert (p.M, dict(paths_per_item=512, gather_layout="nodes", waves_per_cu=8)) in seen
    assert t.cache[autotune.shape_key(p)]["kept"] == "auto at full M"
    assert t.instance_config(p) == {"paths_per_item": 0, "gather_layout": "auto"}


def test_best_picks_fastest_and_caches(tmp_path):
    calls = []

    def fake(problem, cfg):
        calls.append(cfg)
        if cfg == autotune.AUTO:
            return 1.0
        return cfg["paths_per_item"] * (2 if cfg["gather_layout"] == "cells" else 1) + cfg["waves_per_cu"]

    path = tmp_path / "tune.json"
    t = autotune.Tuner(cache_path=str(path), proxy_paths=512, measure=fake)
    p = W.cavity_65(precision=32)
    best = t.best(p)
    assert best == dict(paths_per_item=512, gather_layout="cells", waves_per_cu=16)
    n = len(calls)
    # the proxy's candidates and the library's choice, then both at full M
    assert n == len(autotune.candidates(p.replace(M=512))) + 3
    # second call: cache hit, nothing timed
    assert t.best(p.replace(k=3.5)) == best and len(calls) == n
    # a fresh tuner reads the file
    t2 = autotune.Tuner(cache_path=str(path), measure=fake)
    assert t2.best(p) == best and len(calls) == n
    rec = json.loads(path.read_text())[autotune.shape_key(p)]
    assert rec["auto_path_steps_per_s"] == 1.0 and rec["proxy_paths"] == 512
