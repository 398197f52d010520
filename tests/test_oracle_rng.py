"""Pins of the oracle's random-number pipeline (CPU only).

* Philox4x32-10 words against PyTorch's own Philox engine (ATen's header-only
  ``philox_engine``, built here from torch's include directory): an
  independent implementation of the same published generator.
* The uniform map is exact in binary32 and stays inside (0, 1).
* Box-Muller normals: moments and a Kolmogorov-Smirnov test against N(0, 1).
"""
import math
import os
import subprocess

import numpy as np
import pytest
import scipy.stats

from oracle import fkmc

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    exe = str(tmp_path_factory.mktemp("philox") / "torch_philox")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + inc,
                    os.path.join(HERE, "helpers", "torch_philox.cpp"), "-o", exe], check=True)

    def run(keys, ctrs):
        lines = "".join("%d %d %d %d %d %d\n" % (k[0], k[1], c[0], c[1], c[2], c[3])
                        for k, c in zip(keys, ctrs))
        out = subprocess.run([exe], input=lines, capture_output=True, text=True, check=True).stdout
        return np.array([[int(w) for w in ln.split()] for ln in out.strip().splitlines()], dtype=np.uint32)
    return run


def test_philox_matches_torch_engine(torch_philox):
    rng = np.random.default_rng(123)
    n = 3000
    keys = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    ctrs = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    # the estimator's own counter shapes too: small step, path, node, iteration words
    ctrs[:1000, 0] = rng.integers(0, 20000, 1000)
    ctrs[:1000, 1] = rng.integers(0, 16384, 1000)
    ctrs[:1000, 2] = rng.integers(0, 66049, 1000)
    ctrs[:1000, 3] = rng.integers(0, 40, 1000)
    keys[:500] = [1, 0]
    ref = torch_philox(keys, ctrs)
    mine = np.vstack([fkmc.philox(c[None, :], k) for k, c in zip(keys, ctrs)])
    assert np.array_equal(mine, ref)


def test_philox_batch_equals_single():
    rng = np.random.default_rng(5)
    ctrs = rng.integers(0, 2 ** 32, size=(64, 4), dtype=np.uint64).astype(np.uint32)
    key = np.array([17, 4], dtype=np.uint32)
    batch = fkmc.philox(ctrs, key)
    for i in range(64):
        assert np.array_equal(batch[i], fkmc.philox(ctrs[i:i + 1], key)[0])


def test_uniform_exact_in_binary32_and_open_interval():
    words = [0, 1, 511, 512, 2 ** 31, 2 ** 32 - 1, 0x12345678, 0xFFFFFE00]
    for w in words:
        u = fkmc.uniform(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u          # representable in binary32
    assert fkmc.uniform(0) == 2.0 ** -24
    assert fkmc.uniform(2 ** 32 - 1) == 1.0 - 2.0 ** -24
    # 2^23 equally spaced values with spacing 2^-23
    assert fkmc.uniform(1 << 9) - fkmc.uniform(0) == 2.0 ** -23


def test_box_muller_is_standard_normal():
    ctr = np.zeros((40000, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(40000)
    ctr[:, 2] = 99
    w = fkmc.philox(ctr, [1, 0])
    z = np.array([fkmc.box_muller(a, b) for a, b in w[:, :2]] +
                 [fkmc.box_muller(a, b) for a, b in w[:, 2:]]).ravel()
    n = len(z)
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(scipy.stats.kurtosis(z, fisher=False) - 3.0) < 0.1
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # the two coordinates of one pair are uncorrelated
    pairs = np.array([fkmc.box_muller(a, b) for a, b in w[:20000, :2]])
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 5 / math.sqrt(20000)


def test_box_muller_tail_bound():
    # the smallest uniform is 2^-24, so |z| <= sqrt(-2 ln 2^-24)
    zx, zy = fkmc.box_muller(0, 0)
    assert math.isclose(math.hypot(zx, zy), math.sqrt(-2 * math.log(2.0 ** -24)), rel_tol=1e-15)
