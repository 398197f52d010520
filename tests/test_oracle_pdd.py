"""Pins of the oracle's probabilistic domain decomposition (Sec. 3's
two-stage procedure): the blocks, solved from exact interface values,
reproduce the global finite-difference step (the decomposition identity of
non-overlapping Dirichlet subdomains), the interfaces and blocks partition
the unknowns, and the PDD iteration with Monte Carlo interfaces settles on
the plane wave."""
import math

import numpy as np
import pytest

from oracle import closed_forms as CF
from oracle import fd, fkmc, pdd
from paper_2308_11469_amd import workloads as W


def smooth_field(p, seed=3):
    rng = np.random.default_rng(seed)
    X, Y = np.meshgrid(np.linspace(p.x0, p.x1, p.nx), np.linspace(p.y0, p.y1, p.ny))
    a = rng.normal(size=4) + 1j * rng.normal(size=4)
    return a[0] * np.sin(2 * X + Y) + a[1] * np.cos(3 * Y) * X + a[2] * X * Y + a[3]


@pytest.mark.parametrize("case", ["plain", "source_shift_damping_aniso"])
def test_blocks_from_exact_interfaces_reproduce_global_fd_step(case):
    p = W.cavity_small().replace(nx=33, ny=33)
    cuts_x, cuts_y = [8, 16, 24], [11, 20]
    if case != "plain":
        p = W.cavity_source(precision=64).replace(nx=29, ny=21, x1=1.4, alpha=20.0, damping=1.5)
        cuts_x, cuts_y = [5, 17], [11]
    u_prev = smooth_field(p)
    u_prev.ravel()[fkmc.node_classes(p).ravel() != 0] = fkmc.boundary_grid(p).ravel()[fkmc.node_classes(p).ravel() != 0]
    exact = fd.neumann(p, 1, u0=u_prev)[0]
    ids = pdd.interface_ids(p, cuts_x, cuts_y)
    frame = fkmc.boundary_grid(p)
    frame.ravel()[ids] = exact.ravel()[ids]
    got = pdd.fill_blocks(p, u_prev, frame, cuts_x, cuts_y)
    assert np.max(np.abs(got - exact)) < 1e-11 * max(1.0, np.abs(exact).max())
    # a wrong frame value moves its block
    frame.ravel()[ids[len(ids) // 2]] += 1.0
    bad = pdd.fill_blocks(p, u_prev, frame, cuts_x, cuts_y)
    assert np.max(np.abs(bad - exact)) > 1e-3


def _disc_case():
    # the scattering problem (sound-soft disc r = 0.25 in [-1, 1]^2, exact
    # series data) on 41 x 41: the cut lines 10, 20, 30 put the disc across
    # the four middle blocks
    p = W.scatter_problem(k=2.0, theta=0.7, N=41, M=64, seed=3, precision=64, h=2e-3, table_len=2048)
    return p, [10, 20, 30], [10, 20, 30]


def test_blocks_with_a_hole_reproduce_global_fd_step():
    # blocks touching the disc are not Dirichlet rectangles: their nodes take
    # exact values like the interface, the other blocks are solved and the
    # global FD step comes back
    p, cx, cy = _disc_case()
    cls = fkmc.node_classes(p)
    u_prev = smooth_field(p)
    u_prev[cls != 0] = fkmc.boundary_grid(p)[cls != 0]
    exact = fd.neumann(p, 1, u0=u_prev)[0]
    ids = pdd.mc_ids(p, cx, cy)
    assert len(pdd.blocks(p, cx, cy)) == 12 and len(pdd.all_blocks(p, cx, cy)) == 16
    frame = fkmc.boundary_grid(p)
    frame.ravel()[ids] = exact.ravel()[ids]
    got = pdd.fill_blocks(p, u_prev, frame, cx, cy)
    assert np.max(np.abs(got - exact)) < 1e-11 * max(1.0, np.abs(exact).max())
    # a wrong value at a node of a block touching the disc stays there (no
    # block is solved from it); one on an interface line moves its blocks
    frame2 = frame.copy()
    inner = [i for i in ids if 10 < i % p.nx < 20 and 10 < i // p.nx < 20]
    frame2.ravel()[inner[0]] += 1.0
    bad = pdd.fill_blocks(p, u_prev, frame2, cx, cy)
    assert np.count_nonzero(np.abs(bad - exact) > 1e-9) == 1


def test_interfaces_and_blocks_partition_the_unknowns_with_a_hole():
    p, cx, cy = _disc_case()
    seen = np.zeros(p.nx * p.ny, int)
    seen[pdd.mc_ids(p, cx, cy)] += 1
    for i0, i1, j0, j1 in pdd.blocks(p, cx, cy):
        for j in range(j0, j1):
            seen[j * p.nx + i0: j * p.nx + i1] += 1
    unknown = fkmc.node_classes(p).ravel() == 0
    assert np.all(seen[unknown] == 1) and np.all(seen[~unknown] == 0)
    # the Monte Carlo stage is the interface plus the middle blocks' nodes
    assert len(pdd.mc_ids(p, cx, cy)) > len(pdd.interface_ids(p, cx, cy))


def test_interfaces_and_blocks_partition_the_unknowns():
    p = W.cavity_small().replace(nx=23, ny=17)
    cuts_x, cuts_y = [1, 7, 20], [8]
    seen = np.zeros(p.nx * p.ny, int)
    seen[pdd.interface_ids(p, cuts_x, cuts_y)] += 1
    for i0, i1, j0, j1 in pdd.blocks(p, cuts_x, cuts_y):
        for j in range(j0, j1):
            seen[j * p.nx + i0: j * p.nx + i1] += 1
    unknown = fkmc.node_classes(p).ravel() == 0
    assert np.all(seen[unknown] == 1) and np.all(seen[~unknown] == 0)


@pytest.mark.parametrize("bad", [([0], []), ([5, 5], []), ([], [15]), ([], [])])
def test_bad_cuts_rejected(bad):
    with pytest.raises(ValueError):
        pdd.interface_ids(W.cavity_small().replace(nx=17, ny=16), *bad)


def test_pdd_iteration_settles_on_the_plane_wave():
    # 17 x 17 cavity, k = 2 (rho = 4 / lambda_1^h ~ 0.2): Feynman-Kac at the
    # 29 interface nodes only, FD blocks; after 6 iterations the iterate is
    # the plane wave up to interface noise and the O(sqrt h) exit bias, which
    # the blocks carry inwards harmonically (no larger than on the interfaces)
    p = W.cavity_small().replace(nx=17, ny=17, M=4000, h=1e-4, seed=7)
    cuts = [8]
    u = None
    for n in range(6):
        u, est = pdd.pdd_step(p, u, n, cuts, cuts)
    X, Y = np.meshgrid(np.linspace(0, 1, 17), np.linspace(0, 1, 17))
    ex = CF.plane_wave(2.0, math.pi / 6, X, Y)
    ids = fkmc.interior_ids(p)
    err = np.abs(u.ravel()[ids] - ex.ravel()[ids])
    iface = pdd.interface_ids(p, cuts, cuts)
    err_if = np.abs(u.ravel()[iface] - ex.ravel()[iface])
    assert err.max() < 0.05
    assert err.max() <= err_if.max() + 0.01
