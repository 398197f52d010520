"""Pins of the oracle's geometry pieces: node classes, exit test, nearest
boundary point, boundary data and bilinear interpolation (CPU only)."""
import math

import numpy as np
import pytest

from oracle import fkmc
from paper_2308_11469_amd import workloads as W


def disc_problem(N=33):
    return W.scatter_problem(k=2.0, theta=0.3, N=N, M=64, seed=3, table_len=4096)


def test_node_classes_rect():
    p = W.cavity_small()
    cls = fkmc.node_classes(p)
    assert cls.shape == (9, 9)
    assert (cls[1:-1, 1:-1] == 0).all()
    assert (cls[0, :] == 1).all() and (cls[-1, :] == 1).all()
    assert (cls[:, 0] == 1).all() and (cls[:, -1] == 1).all()
    assert len(fkmc.interior_ids(p)) == 49


def test_node_classes_disc_match_geometry():
    p = disc_problem(33)
    cls = fkmc.node_classes(p)
    xs = np.linspace(-1, 1, 33)
    X, Y = np.meshgrid(xs, xs)
    hole = (X ** 2 + Y ** 2 <= 0.25 ** 2)
    hole[0, :] = hole[-1, :] = hole[:, 0] = hole[:, -1] = False
    assert np.array_equal(cls == 2, hole)
    assert (cls == 2).sum() == 49  # lattice points with i^2 + j^2 <= 16 at spacing 1/16


@pytest.mark.parametrize("x,y,out", [(0.5, 0.5, 0), (0.0, 0.5, 1), (1.0, 0.3, 1), (0.2, 0.0, 1),
                                     (0.2, 1.0, 1), (-1e-300, 0.5, 1), (0.5, 1.0 - 1e-16, 0),
                                     (1.2, -0.4, 1)])
def test_outside_rect(x, y, out):
    assert fkmc.outside(W.cavity_small(), x, y) == bool(out)


def test_outside_disc_closed():
    p = disc_problem()
    assert fkmc.outside(p, 0.25, 0.0)          # on the circle counts as exited
    assert fkmc.outside(p, 0.0, 0.1)
    assert not fkmc.outside(p, 0.26, 0.0)
    assert not fkmc.outside(p, 0.5, 0.5)


def test_projection():
    p = W.cavity_small()
    assert fkmc.project(p, 1.3, 0.4) == (1, (1.0, 0.4))
    assert fkmc.project(p, -0.1, -0.2) == (1, (0.0, 0.0))
    assert fkmc.project(p, 0.3, 1.0) == (1, (0.3, 1.0))
    q = disc_problem()
    which, (px, py) = fkmc.project(q, 0.1, 0.1)
    assert which == 2
    assert math.isclose(math.hypot(px, py), 0.25, rel_tol=1e-15)
    assert math.isclose(px, py, rel_tol=1e-15)
    # inside the domain (a capped path): the nearest boundary part
    assert fkmc.project(p, 0.9, 0.5) == (1, (1.0, 0.5))
    which, (px, py) = fkmc.project(q, 0.3, 0.0)
    assert which == 2 and math.isclose(px, 0.25) and abs(py) < 1e-15
    assert fkmc.project(q, 0.95, 0.1) == (1, (1.0, 0.1))


def test_bilinear_interpolation_exact_on_bilinear_functions():
    p = W.Problem(x0=-0.3, x1=1.7, y0=0.2, y1=1.1, nx=13, ny=7)
    xs = p.x0 + np.arange(p.nx) * (p.x1 - p.x0) / (p.nx - 1)
    ys = p.y0 + np.arange(p.ny) * (p.y1 - p.y0) / (p.ny - 1)
    X, Y = np.meshgrid(xs, ys)
    c = (0.3 - 1.1j, 2.0 + 0.5j, -0.7 + 0.25j, 1.3 - 2.0j)
    f = lambda x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * y
    u = f(X, Y)
    rng = np.random.default_rng(0)
    for _ in range(300):
        x = rng.uniform(p.x0, p.x1)
        y = rng.uniform(p.y0, p.y1)
        assert abs(fkmc.interp(p, u, x, y) - f(x, y)) < 1e-13
    # at a node the interpolant returns the node value
    for (i, j) in [(0, 0), (12, 6), (5, 3), (12, 0)]:
        assert abs(fkmc.interp(p, u, xs[i], ys[j]) - u[j, i]) < 1e-14
    # but not on a function with an x^2 term: interpolation error is dx^2/8 * f''
    u2 = X ** 2
    x = xs[3] + 0.5 * (xs[4] - xs[3])
    err = fkmc.interp(p, u2 + 0j, x, ys[2]).real - x ** 2
    assert math.isclose(err, (xs[4] - xs[3]) ** 2 / 4, rel_tol=1e-9)


def test_boundary_data_plane_wave_and_bilinear():
    p = W.cavity_small()
    for (x, y) in [(0.0, 0.3), (1.0, 0.7), (0.2, 1.0)]:
        assert abs(fkmc.g_at(p, 1, x, y) - np.exp(2j * (x * math.cos(math.pi / 6) + y * math.sin(math.pi / 6)))) < 1e-15
    q = W.Problem(outer=W.BC("bilinear", coeffs=(1 + 2j, 3j, -1.0, 0.5 + 0.5j)))
    assert abs(fkmc.g_at(q, 1, 0.5, 0.25) - (1 + 2j + 1.5j - 0.25 + (0.5 + 0.5j) * 0.125)) < 1e-15


def test_table_boundary_data_interpolates_arclength():
    # a table sampled from a function linear in arclength is reproduced exactly
    L = 400
    p = W.Problem(x0=-1, x1=1, y0=-0.5, y1=1.5, outer=W.BC("table"))
    per = 2 * (2.0 + 2.0)
    s = np.arange(L) * per / L
    tab = np.sin(2 * math.pi * s / per) + 1j * np.cos(4 * math.pi * s / per)
    p.outer.table = tab
    px, py = W.perimeter_points(-1, 1, -0.5, 1.5, L)
    for i in range(0, L, 37):
        assert abs(fkmc.g_at(p, 1, px[i], py[i]) - tab[i]) < 1e-12
    # midway between samples: the average of the two neighbours
    i = 10
    mx, my = 0.5 * (px[i] + px[i + 1]), 0.5 * (py[i] + py[i + 1])
    assert abs(fkmc.g_at(p, 1, mx, my) - 0.5 * (tab[i] + tab[i + 1])) < 1e-12
    # periodic wrap at the start corner
    mx, my = px[0], py[0] + 0.5 * (py[L - 1] - py[0])
    assert abs(fkmc.g_at(p, 1, mx, my) - 0.5 * (tab[L - 1] + tab[0])) < 1e-12


def test_boundary_grid():
    p = disc_problem(17)
    g = fkmc.boundary_grid(p)
    cls = fkmc.node_classes(p)
    assert (g[cls == 0] == 0).all()
    xs = np.linspace(-1, 1, 17)
    X, Y = np.meshgrid(xs, xs)
    hole = cls == 2
    assert np.allclose(g[hole], -np.exp(2j * (X[hole] * math.cos(0.3) + Y[hole] * math.sin(0.3))), atol=1e-15)
    edge = cls == 1
    ex = W.disc_scattered(2.0, 0.25, 0.3, X[edge], Y[edge])
    assert np.max(np.abs(g[edge] - ex)) < 1e-5    # linear interpolation of a 4096-sample table


def test_step_cap_formula():
    p = W.cavity_small()
    assert fkmc.jmax_auto(p) == math.ceil(40 / (2 * math.pi ** 2 * 2e-3))
