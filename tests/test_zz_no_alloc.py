"""GPU: the entry point that allocates no device memory
(fk_helmholtz_step_static, its working memory in a static device array)
gives the same iterate, standard errors and report as the allocating path
(create + set_iterate + iterate + get), bit for bit, on two calls in a row,
the second with a smaller problem than the first; and it rejects a problem
whose working memory exceeds the array."""
import numpy as np
import pytest
import torch

from paper_2308_11469_amd import fkh
from paper_2308_11469_amd import workloads as W

from gpu_util import require_lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    require_lib()


def allocating(p, u_n, n):
    """u_{n+1}, SE and report by the solver (its arena allocated by the library)."""
    s = fkh.Solver(p)
    if u_n is not None:
        s.set_iterate(u_n, n)
    rep = s.iterate(1)
    u, se = s.get()
    s.close()
    return u, se, rep


def static(p, u_n, n):
    dev = torch.device("cuda")
    shape = (p.ny, p.nx)
    u_in = None if u_n is None else torch.from_numpy(np.ascontiguousarray(u_n)).to(dev)
    u_out = torch.full(shape, complex("nan"), dtype=torch.complex128, device=dev)
    se_out = torch.full(shape, complex("nan"), dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    rep = fkh.step_static(p, u_in, n, u_out, se_out)
    return u_out.cpu().numpy(), se_out.cpu().numpy(), rep


def same_report(a, b):
    for key in ("max_du", "sup", "max_se", "path_steps", "capped", "nonfinite", "noise_ratio", "diverging"):
        assert a[key] == b[key], (key, a[key], b[key])


@pytest.mark.parametrize("precision", [64, 32])
def test_static_step_matches_allocating_path_on_two_calls(precision):
    # first call: the 33 x 33 source cavity from u_0 = 0, then its second
    # iterate from u_1; then a smaller problem (the 9 x 9 cavity) from a
    # given iterate: the array keeps the previous call's contents, which
    # must not leak into the next one
    big = W.cavity_source(precision=precision).replace(nx=33, ny=33, M=512, h=1e-3)
    small = W.cavity_small().replace(precision=precision, M=256)
    u1, se1, r1 = allocating(big, None, 0)
    v1, sv1, q1 = static(big, None, 0)
    say("static step", precision, "big n=0", r1["path_steps"])
    assert np.array_equal(u1, v1) and np.array_equal(se1, sv1)
    same_report(r1, q1)
    assert q1["n"] == 1
    u2, se2, r2 = allocating(big, u1, 1)
    v2, sv2, q2 = static(big, v1, 1)
    assert np.array_equal(u2, v2) and np.array_equal(se2, sv2)
    same_report(r2, q2)
    # the smaller problem, from a non-trivial iterate at index 3
    rng = np.random.default_rng(3)
    u_in = rng.standard_normal((small.ny, small.nx)) + 1j * rng.standard_normal((small.ny, small.nx))
    u3, se3, r3 = allocating(small, u_in, 3)
    v3, sv3, q3 = static(small, u_in, 3)
    say("static step", precision, "small n=3", r3["path_steps"])
    assert np.array_equal(u3, v3) and np.array_equal(se3, sv3)
    same_report(r3, q3)
    assert q3["n"] == 4


@pytest.mark.parametrize("precision", [64, 32])
def test_static_step_on_a_disc_domain(precision):
    # a disc domain at k > 0: the exterior nodes take their nearest unknown
    # node's value after the update in both paths, so that the second call's
    # paths read the same extended iterate
    p = W.annulus_shape2(n=21, k=1.0, M=128, precision=precision).replace(
        outer=W.BC("plane_wave_robin", 1.0, 0.4), inner=W.BC("plane_wave", 1.0, 0.4))
    u1, se1, r1 = allocating(p, None, 0)
    v1, sv1, q1 = static(p, None, 0)
    say("static step disc", r1["path_steps"])
    assert np.array_equal(u1, v1) and np.array_equal(se1, sv1)
    same_report(r1, q1)
    u2, se2, r2 = allocating(p, u1, 1)
    v2, sv2, q2 = static(p, v1, 1)
    assert np.array_equal(u2, v2) and np.array_equal(se2, sv2)
    same_report(r2, q2)


def test_static_step_rejects_a_problem_beyond_the_array():
    p = W.cavity_65().replace(nx=513, ny=513, M=64)
    out = torch.zeros((p.ny, p.nx), dtype=torch.complex128, device="cuda")
    with pytest.raises(fkh.FkInvalid, match="static"):
        fkh.step_static(p, None, 0, out)
    with pytest.raises(fkh.FkInvalid):
        fkh.step_static(W.cavity_small(), None, 2, out)
