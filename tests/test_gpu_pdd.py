"""GPU parity of the probabilistic domain decomposition (Sec. 3's two-stage
procedure): Feynman-Kac at the interface nodes only, against the oracle's
estimator at those nodes; the device's fast-diagonalisation block solves,
against the oracle's sparse LU of each block from the same interface values;
both gather layouts; the PDD iteration on the cavity settling on the plane
wave; argument checks."""
import math

import numpy as np
import pytest

from oracle import closed_forms as CF
from oracle import fkmc, pdd
from paper_2308_11469_amd import fkh
from paper_2308_11469_amd import workloads as W

from gpu_util import assert_fp64_node_parity, require_lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    require_lib()


def _cases():
    plain = (W.cavity_small().replace(nx=33, ny=33, M=128, seed=5), [8, 16, 24], [11, 20])
    general = (W.cavity_source(precision=64).replace(nx=29, ny=21, x1=1.4, M=96, h=1e-3, alpha=20.0, damping=1.5),
               [5, 17], [11])
    wide = (W.cavity_65(k=3.0).replace(M=64, h=1e-3), [32], [])    # two 31 x 63 blocks, one interface line
    # degenerate cuts: at 1 and n - 2 (nothing outside them), adjacent lines
    # 7 and 8 (no block between), one-node-wide blocks (the DST of size 1)
    degenerate = (W.cavity_small().replace(nx=23, ny=17, M=96, seed=13), [1, 7, 8, 19, 21], [2, 8, 15])
    # the scattering problem's disc across the four middle blocks: their
    # nodes run paths like the interface, the other twelve blocks are solved
    disc = (W.scatter_problem(k=2.0, theta=0.7, N=41, M=96, seed=3, precision=64, h=2e-3, table_len=2048),
            [10, 20, 30], [10, 20, 30])
    return {"plain_33": plain, "source_general_aniso": general, "wide_blocks_65": wide,
            "degenerate_cuts": degenerate, "disc_hole_41": disc}


def frame_of(p, g, ids):
    f = fkmc.boundary_grid(p)
    f.ravel()[ids] = g.ravel()[ids]
    return f


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_pdd_interfaces_and_blocks_match_oracle(name):
    p, cx, cy = _cases()[name]
    say("pdd", name)
    s = fkh.Solver(p)
    s.set_pdd(cx, cy)
    ids = pdd.mc_ids(p, cx, cy)
    u = None
    for it in range(3):
        s.iterate(1)
        g, se = s.get()
        sj, _ = s.node_stats()
        orc = fkmc.fk_nodes(p, u, it, ids)
        assert_fp64_node_parity(g.ravel()[ids], sj[ids], orc, p.M, label="%s it %d" % (name, it))
        # blocks: the oracle's LU from the same interface values and u_n
        ref = pdd.fill_blocks(p, u, frame_of(p, g, ids), cx, cy)
        scale = max(1.0, np.abs(ref).max())
        assert np.max(np.abs(g - ref)) <= 1e-11 * scale, np.max(np.abs(g - ref))
        # Monte Carlo ran at the interface only
        mask = np.zeros(p.nx * p.ny, bool)
        mask[ids] = True
        assert np.all(se.ravel()[~mask] == 0) and np.all(sj[~mask] == 0)
        u = g
    s.close()


@pytest.mark.parametrize("precision", [64, 32])
def test_pdd_gather_layouts_identical(precision):
    # the block solve writes the gather copy the next iteration's paths read
    p = W.cavity_source(precision=precision).replace(M=64, h=1e-3)
    cuts = [32, 64, 96]
    out = []
    for layout in ("nodes", "cells"):
        s = fkh.Solver(p, gather_layout=layout)
        s.set_pdd(cuts, cuts)
        s.iterate(3)
        out.append(s.get()[0])
        s.close()
    assert np.array_equal(out[0], out[1])


def test_pdd_fp32_blocks_from_own_interfaces():
    p = W.cavity_source(precision=32).replace(M=256, h=1e-3)
    cuts = [32, 64, 96]
    s = fkh.Solver(p)
    s.set_pdd(cuts, cuts)
    ids = pdd.mc_ids(p, cuts, cuts)
    s.iterate(1)
    u1 = s.get()[0]
    s.iterate(1)
    g = s.get()[0]
    s.close()
    ref = pdd.fill_blocks(p, u1, frame_of(p, g, ids), cuts, cuts)
    assert np.max(np.abs(g - ref)) <= 1e-11 * max(1.0, np.abs(ref).max())


def test_pdd_iteration_settles_on_the_plane_wave():
    # the bench cavity with interfaces every 16 nodes: paths from 369 of the
    # 3969 unknown nodes; the blocks carry the interface noise inwards
    # harmonically, so the error is no larger than on the interfaces
    p = W.cavity_65(k=2.0, precision=32).replace(seed=9)
    cuts = [16, 32, 48]
    s = fkh.Solver(p)
    s.set_pdd(cuts, cuts)
    for _ in range(8):
        rep = s.iterate(1)
    g, se = s.get()
    s.close()
    ex = W.exact_solution(p)
    ids = fkmc.interior_ids(p)
    iface = pdd.mc_ids(p, cuts, cuts)
    err = np.abs(g.ravel()[ids] - ex.ravel()[ids])
    err_if = np.abs(g.ravel()[iface] - ex.ravel()[iface])
    max_se = np.abs(se.ravel()[iface]).max()
    # exit-bias scale of the once-per-step test: beta sqrt(2h) |grad u|
    bias = CF.bgk_beta() * math.sqrt(2.0 * p.h) * p.k
    say("pdd cavity65: max err %.4f (interfaces %.4f), rms %.4f, max SE %.4f, %d path-steps per iteration"
        % (err.max(), err_if.max(), np.sqrt(np.mean(err ** 2)), max_se, rep["path_steps"]))
    assert err.max() < 4.5 * max_se + bias
    assert np.sqrt(np.mean(err ** 2)) < max_se + bias
    assert err.max() <= err_if.max() + 1e-3


@pytest.mark.parametrize("bad", ["after_iterate", "twice", "twice_no_blocks", "reflecting", "too_wide", "no_cut",
                                 "unsorted"])
def test_pdd_argument_checks(bad):
    p = W.cavity_small().replace(nx=33, ny=33, M=64)
    cx, cy = [16], [16]
    if bad == "reflecting":
        p = W.annulus_shape3(k=0.5, nx=21, ny=33, M=64, h=1e-3, precision=64)
        cx, cy = [10], [16]
    if bad == "too_wide":
        p = W.cavity_65().replace(nx=129, ny=129, M=64)
        cx, cy = [100], [64]
    if bad == "no_cut":
        cx, cy = [], []
    if bad == "unsorted":
        cx = [20, 10]
    if bad == "twice_no_blocks":
        # every interior column a cut line: no block between them, and still
        # only one call
        cx, cy = list(range(1, p.nx - 1)), []
    s = fkh.Solver(p)
    if bad == "after_iterate":
        s.iterate(1)
    if bad in ("twice", "twice_no_blocks"):
        s.set_pdd(cx, cy)
    with pytest.raises(ValueError):
        s.set_pdd(cx, cy)
    s.close()


def test_pdd_item_size_with_m_not_a_power_of_two():
    # the item size re-derived for the interface list stays a multiple of 64
    # and never changes the result: automatic against a fixed 64 paths
    p = W.cavity_65(k=2.0).replace(nx=49, ny=49, M=150, h=1e-3)
    cuts = [12, 24, 36]
    out = []
    for ppi in (0, 64, 192):
        s = fkh.Solver(p, paths_per_item=ppi)
        s.set_pdd(cuts, cuts)
        s.iterate(2)
        out.append(s.get()[0])
        s.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def _pdd_engine(precision, n=8):
    return fkh.Engine(n, precision=precision, max_grid_nodes=1 << 16, max_items=1 << 18, max_table=1 << 14,
                      max_instance_nodes=1 << 14)


@pytest.mark.parametrize("precision", [64, 32])
def test_engine_pdd_alone_mix_and_solver_bit_identical(precision):
    # two decomposed instances (different grids and cuts) batched with two
    # full Monte Carlo instances: each result equals the single-instance
    # solver's, whatever shares the launch and its block-solve pass
    a = (W.cavity_small().replace(nx=33, ny=33, M=128, seed=5, precision=precision), [8, 16, 24], [11, 20])
    b = (W.cavity_source(precision=precision).replace(nx=29, ny=21, x1=1.4, M=96, h=1e-3, alpha=20.0,
                                                      damping=1.5), [5, 17], [11])
    plain = [W.cavity_small().replace(precision=precision, M=256, seed=21),
             W.scatter_problem(k=2.0, theta=1.0, N=21, M=128, seed=5007, precision=precision, h=2e-3,
                               table_len=2048)]
    ticks = 3
    ref = []
    for p, cx, cy in (a, b):
        s = fkh.Solver(p, paths_per_item=64)
        s.set_pdd(cx, cy)
        s.iterate(ticks)
        ref.append(s.get()[0])
        s.close()
        e = _pdd_engine(precision)
        sl = e.add(p, paths_per_item=64)
        assert e.set_pdd(sl, cx, cy)
        for _ in range(ticks):
            e.tick()
        alone = e.get(sl)[0]
        e.close()
        assert np.array_equal(alone, ref[-1])
    e = _pdd_engine(precision)
    slots = [e.add(p, paths_per_item=64) for p in plain]
    sa = e.add(a[0], paths_per_item=64)
    assert e.set_pdd(sa, a[1], a[2])
    sb = e.add(b[0], paths_per_item=64)
    assert e.set_pdd(sb, b[1], b[2])
    for _ in range(ticks):
        e.tick()
    say("engine pdd mix", precision)
    assert np.array_equal(e.get(sa)[0], ref[0]) and np.array_equal(e.get(sb)[0], ref[1])
    mixed_plain = [e.get(s)[0] for s in slots]
    # a decomposition may only be set before the instance's first tick
    with pytest.raises(ValueError):
        e.set_pdd(sa, a[1], a[2])
    e.close()
    for p, g in zip(plain, mixed_plain):
        s = fkh.Solver(p, paths_per_item=64)
        s.iterate(ticks)
        assert np.array_equal(s.get()[0], g)
        s.close()


def test_engine_pdd_matches_oracle():
    p, cx, cy = _cases()["plain_33"]
    e = _pdd_engine(64)
    sl = e.add(p)
    assert e.set_pdd(sl, cx, cy)
    ids = pdd.mc_ids(p, cx, cy)
    u = None
    for it in range(2):
        e.tick()
        g, _ = e.get(sl)
        sj, _ = e.node_stats(sl)
        orc = fkmc.fk_nodes(p, u, it, ids)
        assert_fp64_node_parity(g.ravel()[ids], sj[ids], orc, p.M, label="engine pdd it %d" % it)
        ref = pdd.fill_blocks(p, u, frame_of(p, g, ids), cx, cy)
        assert np.max(np.abs(g - ref)) <= 1e-11 * max(1.0, np.abs(ref).max())
        u = g
    e.close()
