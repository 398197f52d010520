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
