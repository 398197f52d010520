"""The autotuner on the GPU: it times real launches, returns one of its
candidates, and the tuned launch gives the same iterates as the library's
own choice (launch parameters never change results)."""
import numpy as np
import pytest

from paper_2308_11469_amd import autotune, fkh
from paper_2308_11469_amd import workloads as W

from gpu_util import require_lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    require_lib()


@pytest.mark.parametrize("precision", [32, 64])
def test_tuned_launch_matches_default(tmp_path, precision):
    p = W.cavity_65(precision=precision).replace(nx=33, ny=33, M=384)
    t = autotune.Tuner(cache_path=str(tmp_path / "t.json"), proxy_paths=256, ppi=(64, 256), waves=(8, 16))
    best = t.best(p)
    say("tuned", precision, best, t.cache[autotune.shape_key(p)]["path_steps_per_s"])
    assert best in autotune.candidates(p.replace(M=256), (64, 256), (8, 16)) or best == autotune.AUTO
    # the proxy's candidates, the library's choice, then both at the full M
    assert t.timed == len(autotune.candidates(p.replace(M=256), (64, 256), (8, 16))) + 3
    runs = []
    for cfg in (best, autotune.AUTO):
        s = fkh.Solver(p, **cfg)
        s.iterate(2)
        runs.append(s.get())
        s.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
