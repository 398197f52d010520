"""Helpers shared by the GPU tests (no test collection here)."""
import math

import numpy as np

from oracle import fkmc
from paper_2308_11469_amd import build, fkh


def require_lib():
    if not build.is_built():
        raise RuntimeError("libfk_helmholtz.so is not built")
    return fkh.lib()


def say(*a):
    print("[gpu-test]", *a, flush=True)


def score_scale(mean, var_re, var_im, M):
    """sqrt(mean of |s|^2) over the paths of a node: the size of one score,
    the scale at which FP64 round-off of the two implementations is judged."""
    return np.sqrt(var_re * (M - 1) / M + var_im * (M - 1) / M + np.abs(mean) ** 2)


def assert_fp64_node_parity(gpu_mean, gpu_sumJ, orc, M, rel=1e-12, label=""):
    """FP64: exit-step sums bit-exact, means within rel * score scale."""
    scale = score_scale(orc["mean"], orc["var_re"], orc["var_im"], M)
    err = np.abs(gpu_mean - orc["mean"])
    bad = err > rel * np.maximum(scale, 1e-300)
    assert not bad.any(), "%s: %d nodes off, worst %.3g (scale %.3g)" % (
        label, bad.sum(), err.max(), scale[np.argmax(err)])
    assert np.array_equal(gpu_sumJ, orc["sumJ"]), "%s: exit-step sums differ at %d nodes" % (
        label, int((gpu_sumJ != orc["sumJ"]).sum()))


def interior_values(p, grid):
    return grid.ravel()[fkmc.interior_ids(p)]


def assert_se_parity(gpu_se, orc, M, label=""):
    """Per-node standard errors against the oracle's two-pass variances.  The
    library forms var = (sum s^2 - (sum s)^2 / M) / (M - 1) from exact
    fixed-point sums whose squares keep 2^-40 per path, so its variance may
    differ by M 2^-40 / (M - 1) plus the rounding of that difference
    (a few ulp of sum s^2): for a node whose scores barely vary that bound,
    not 1e-8 relative, is the scale of agreement."""
    for comp, var_o in (("re", orc["var_re"]), ("im", orc["var_im"])):
        se_g = np.real(gpu_se) if comp == "re" else np.imag(gpu_se)
        var_g = se_g ** 2 * M
        mean = np.real(orc["mean"]) if comp == "re" else np.imag(orc["mean"])
        q = M * (var_o + mean ** 2)
        tol = 1e-8 * var_o + 2.0 * (M * 2.0 ** -40 + 8.0 * 2.0 ** -53 * q) / (M - 1)
        bad = np.abs(var_g - var_o) > tol
        assert not bad.any(), "%s: SE_%s off at %d nodes (worst %.3g vs tol %.3g)" % (
            label, comp, bad.sum(), np.abs(var_g - var_o).max(), tol[np.argmax(np.abs(var_g - var_o))])
