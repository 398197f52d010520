"""Pins of the oracle's reflecting-edge path (the annular iteration of
Sec. 2.3) and of the finite differences for mixed problems.

The finite differences are pinned by exactness on polynomials and by the
values Table 1 prints; the Monte Carlo oracle is pinned against them (mean
exit time and mean local time of the reflected diffusion) and by the fixed
point of the iteration at a closed-form solution (a plane wave with its own
Robin datum on the edge).
"""
import math

import numpy as np
import pytest

from oracle import closed_forms as CF
from oracle import fd_mixed as FM
from oracle import fkmc
from paper_2308_11469_amd import workloads as W

import paper_values as PV

QUAD_LAP = 4.0


def quad(x, y):
    return x * x + y * y + 3.0 * x * y - 0.5 * x + 0.25 * y     # Laplacian 4


def quad_grad(x, y):
    return 2.0 * x + 3.0 * y - 0.5, 2.0 * y + 3.0 * x + 0.25


def solve_with_neumann(p, scheme, u, grad, lap):
    """Solves the scheme's system with Dirichlet u on the hole and the exact
    d_n u on each face."""
    A, ids, D, EF = FM.system(p, scheme, phi=lambda x, y: complex(u(x, y)))
    xs = p.x0 + (ids % p.nx) * ((p.x1 - p.x0) / (p.nx - 1))
    ys = p.y0 + (ids // p.nx) * ((p.y1 - p.y0) / (p.ny - 1))
    gx, gy = grad(xs, ys)
    gface = np.stack([-gx, gx, -gy, gy], axis=1)
    edge = EF.any(axis=1)
    rhs = np.full(len(ids), lap, dtype=complex)
    if scheme == "one_sided":
        rhs[edge] = 0.0
    rhs = rhs - D - (EF * gface).sum(axis=1)
    import scipy.sparse.linalg as spla
    sol = spla.spsolve(A.tocsc().astype(complex), rhs)
    return sol, u(xs, ys)


@pytest.mark.parametrize("geom", ["disc", "box_on_lines", "box_between_lines", "box_dx_ne_dy"])
def test_fd_ghost_scheme_exact_on_quadratics(geom):
    # 5-point Laplacian, central-difference ghost nodes and Shortley-Weller
    # arms are exact for quadratics, corners included
    p = {"disc": W.annulus_shape1(n=21),
         "box_on_lines": W.annulus_shape3(nx=41, ny=65),
         "box_between_lines": W.annulus_fig2(n=11),
         "box_dx_ne_dy": W.annulus_shape3(nx=41, ny=33)}[geom]
    sol, exact = solve_with_neumann(p, "ghost", quad, quad_grad, QUAD_LAP)
    assert np.max(np.abs(sol - exact)) < 1e-10


def test_fd_one_sided_scheme_exact_on_linear():
    lin = lambda x, y: 2.0 * x - 3.0 * y + 1.0
    grad = lambda x, y: (np.full_like(x, 2.0), np.full_like(y, -3.0))
    for p in (W.annulus_fig2(n=11), W.annulus_shape3(nx=41, ny=33)):
        sol, exact = solve_with_neumann(p, "one_sided", lin, grad, 0.0)
        assert np.max(np.abs(sol - exact)) < 1e-10


def test_node_classes_reflecting_edge_and_box_hole():
    p = W.annulus_shape3(nx=41, ny=65)
    cls = fkmc.node_classes(p)
    # every edge node is an unknown; the hole [-0.05, 0.05] x [-0.4, 0.4]
    # holds 5 x 33 nodes (its edges on grid lines despite x0 + i dx rounding)
    assert (cls[0, :] == 0).all() and (cls[-1, :] == 0).all()
    assert (cls[:, 0] == 0).all() and (cls[:, -1] == 0).all()
    assert (cls == 2).sum() == 5 * 33
    assert (cls == 1).sum() == 0
    assert (cls[16:49, 18:23] == 2).all()


def test_fd_table1_exit_and_local_time_suprema():
    # Table 1 (tests/golden/table1_annulus.txt): sup E[tau], sup E[xi] and
    # k_*^A of shapes 1 and 3, to the two printed digits
    t = PV.table1()
    for shape, p in ((1, W.annulus_shape1(n=121)), (3, W.annulus_shape3(nx=161, ny=257))):
        e, l = FM.exit_time(p).max(), FM.local_time(p).max()
        assert round(e, 2) == t[shape]["sup_tau"] and round(l, 2) == t[shape]["sup_xi"]
        assert round(FM.k_star_A(e, l), 2) == t[shape]["kstar_A"]


def plane_wave_problem(k=2.0, theta=0.4, n=31, **kw):
    p = W.annulus_shape1(k=k, n=n).replace(inner=W.BC("plane_wave", 1.0 + 0j, theta),
                                           outer=W.BC("plane_wave_robin", 1.0 + 0j, theta))
    return p.replace(**kw)


def test_fd_robin_direct_plane_wave_second_order():
    errs = []
    for n in (31, 61):
        p = plane_wave_problem(n=n)
        u = FM.direct(p)
        X, Y = np.meshgrid(np.linspace(p.x0, p.x1, p.nx), np.linspace(p.y0, p.y1, p.ny))
        errs.append(np.max(np.abs(u - CF.plane_wave(p.k, 0.4, X, Y))))
    assert errs[1] < errs[0] / 3.0 and errs[1] < 1e-3


def test_fd_iterate_converges_to_direct():
    # the paper's problem (g2 = 0) on shape 1 at k = 1.5 < k_*^A and the
    # plane wave with its Robin datum, shifted: both contract
    for p in (W.annulus_shape1(k=1.5, n=31), plane_wave_problem(k=1.0, alpha=1.5)):
        its = FM.iterate(p, 80)
        ref = FM.direct(p)
        assert np.max(np.abs(its[-1] - ref)) < 1e-9
        assert np.max(np.abs(its[1] - ref)) > 1e-3


def test_fd_spectral_radius_matches_iteration_growth():
    # the ratio of successive increments of the iteration tends to rho(G),
    # below and above one
    for k in (1.2, 1.5):
        p = W.annulus_fig2(n=11, k=k)
        rho = FM.spectral_radius_G(p, k, "one_sided")
        its = FM.iterate(p, 90, scheme="one_sided")
        d1 = np.linalg.norm((its[-1] - its[-2]).ravel())
        d0 = np.linalg.norm((its[-2] - its[-3]).ravel())
        assert abs(d1 / d0 - rho) < 1e-6 * rho


def test_fd_fig2_radius_crosses_one_above_k_star():
    # Sec. 2.4: on both grids the spectral radius of G reaches one only past
    # the k_*^A of the problem, as the crossings stated with the figure
    # (tests/golden/fig2_spectral_radius.txt) lie above its k_*^A; the
    # numbers themselves are not reproducible from the text
    assert min(PV.fig2_crossings().values()) > 0.81
    for n in (11, 21):
        p = W.annulus_fig2(n=n)
        ks = FM.k_star_A(FM.exit_time(p, "one_sided").max(), FM.local_time(p, "one_sided").max())
        assert FM.spectral_radius_G(p, ks) < 1.0
        grid = np.arange(ks, 3.0, 0.05)
        rho = [FM.spectral_radius_G(p, k) for k in grid]
        assert all(b > a for a, b in zip(rho, rho[1:]))
        assert rho[-1] > 1.0


# ---------------------------------------------------------- Monte Carlo

def sample_nodes(p):
    """Corner, edge and interior unknown nodes."""
    nx, ny = p.nx, p.ny
    pick = [(0, 0), (nx - 1, ny - 1), (0, ny // 2), (nx // 2, 0), (nx - 1, ny // 3), (1, 1),
            (nx // 4, ny // 4), (nx - 3, ny // 2), (2, ny - 4)]
    cls = fkmc.node_classes(p).ravel()
    ids = np.array([i + nx * j for i, j in pick if cls[i + nx * j] == 0], dtype=np.int32)
    assert len(ids) >= 8
    return ids


def shrunk(p, h):
    """The problem with the hole shrunk by the continuity correction
    beta sqrt(2h) of a discretely monitored absorbing boundary (the exit test
    runs once per step)."""
    d = CF.bgk_beta() * math.sqrt(2.0 * h)
    return p.replace(r=p.r - d)


@pytest.mark.parametrize("which", ["exit_time", "local_time"])
def test_mc_reflected_moments_match_fd(which):
    h = 2e-5
    base = W.annulus_shape1(n=13, h=h, M=6000, k=0.0)
    if which == "exit_time":
        p = base.replace(src_kind="const", src_amp=-1.0 + 0j, inner=W.BC("zero"), outer=W.BC("zero"))
    else:
        p = base.replace(inner=W.BC("zero"), outer=W.BC("bilinear", coeffs=(1.0 + 0j, 0j, 0j, 0j)))
    ids = sample_nodes(p)
    est = fkmc.fk_nodes(p, None, 0, ids)
    fine = shrunk(W.annulus_shape1(n=121), h)
    ref = (FM.exit_time(fine) if which == "exit_time" else FM.local_time(fine)).ravel()
    # node (i, j) of the 13-grid is node (10 i, 10 j) of the 121-grid
    fid = (ids % 13) * 10 + 121 * ((ids // 13) * 10)
    err = np.abs(est["mean"].real - ref[fid])
    assert np.all(err < 4.0 * est["se"].real + 0.01 * ref[fid]), (err, est["se"].real)
    assert np.all(np.abs(est["mean"].imag) == 0.0)
    assert est["capped"].sum() == 0


@pytest.mark.parametrize("case", ["plain", "shifted_damped"])
def test_mc_plane_wave_is_fixed_point(case):
    # one step of the iteration from the exact solution returns it: the
    # plane wave w solves Delta w + (k^2 + i p) w = 0 with w on the hole and
    # d_n w - i k w = g2 (its Robin datum) on the edge
    kw = {} if case == "plain" else dict(alpha=2.0, damping=0.5)
    p = plane_wave_problem(k=1.0, n=13, M=20000, h=5e-5, seed=21, **kw)
    X, Y = np.meshgrid(np.linspace(p.x0, p.x1, p.nx), np.linspace(p.y0, p.y1, p.ny))
    exact = CF.plane_wave(p.k, 0.4, X, Y, damping=p.damping)
    ids = sample_nodes(p)
    est = fkmc.fk_nodes(p, exact, 1, ids)
    err = np.abs(est["mean"] - exact.ravel()[ids])
    se = np.abs(est["se"])
    # continuity-correction scale of the exit bias: beta sqrt(2h) |grad w|
    bias = CF.bgk_beta() * math.sqrt(2.0 * p.h) * abs(np.sqrt(complex(p.k ** 2, p.damping)))
    assert np.all(err < 5.0 * se + 2.0 * bias), (err, se, bias)


def test_mc_fixed_point_check_rejects_a_wrong_field():
    # power of the check above: the plane wave of the opposite direction
    # solves the same equation but not the Robin condition with this g2, and
    # one step from it does not return it
    p = plane_wave_problem(k=1.0, n=13, M=4000, h=5e-5, seed=21)
    X, Y = np.meshgrid(np.linspace(p.x0, p.x1, p.nx), np.linspace(p.y0, p.y1, p.ny))
    other = CF.plane_wave(p.k, 0.4 + math.pi, X, Y)
    ids = sample_nodes(p)
    est = fkmc.fk_nodes(p, other, 1, ids)
    assert np.max(np.abs(est["mean"] - other.ravel()[ids])) > 0.1


def test_mc_reflected_paths_stay_in_rectangle_and_end_in_hole():
    p = W.annulus_shape3(nx=21, ny=33, h=1e-4, k=0.5)
    cls = fkmc.node_classes(p).ravel()
    starts = [0, p.nx - 1, p.nx * (p.ny - 1), int(np.nonzero(cls == 0)[0][100])]
    for nid in starts:
        for m in range(6):
            s, J, cap, (x, y) = fkmc.path(p, None, 0, nid, m)
            assert cap == 0
            assert p.x0 <= x <= p.x1 and p.y0 <= y <= p.y1
            assert p.cx - p.r <= x <= p.cx + p.r and p.cy - p.ry <= y <= p.cy + p.ry
            # u_0 = 0 and g2 = 0: the score is the inner datum at the exit
            which, (px, py) = fkmc.project(p, x, y)
            assert which == 2
            assert abs(s - fkmc.g_at(p, 2, px, py)) < 1e-15


def test_reflecting_problem_needs_explicit_step_cap():
    with pytest.raises(ValueError):
        fkmc.jmax_auto(W.annulus_shape1().replace(jmax=0))


# ------------------------------------------------ the disc's curved edge

def concentric(h, M, n=21, a=0.15):
    """The unit disc of radius 0.5 at (0.5, 0.5) with a reflecting edge,
    minus the closed disc of radius a at its centre."""
    return W.Problem(name="concentric", domain_kind=W.DISC_MINUS_DISC, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                     cx=0.5, cy=0.5, r=a, reflect=True, nx=n, ny=n, k=0.0, h=h, M=M, seed=31,
                     jmax=int(math.ceil(60.0 / h)), outer=W.BC("zero"), inner=W.BC("zero"))


def concentric_exact(which, rho, R=0.5, a=0.15):
    # Delta w = -1, w(a) = 0, w'(R) = 0:  w = R^2/2 ln(rho/a) - (rho^2 - a^2)/4
    # Delta L = 0,  L(a) = 0, L'(R) = 1:  L = R ln(rho/a)
    if which == "exit_time":
        return R * R / 2.0 * np.log(rho / a) - (rho ** 2 - a * a) / 4.0
    return R * np.log(rho / a)


@pytest.mark.parametrize("which", ["exit_time", "local_time"])
def test_mc_curved_edge_matches_concentric_closed_forms(which):
    # the radial mirror and its local time 2 x overshoot against the closed
    # forms of the concentric annulus; the hole's radius is shrunk by the
    # continuity correction of the once-per-step exit test (O(sqrt h) bias)
    h = 2e-5
    p = concentric(h, M=4000)
    if which == "exit_time":
        p = p.replace(src_kind="const", src_amp=-1.0 + 0j)
    else:
        p = p.replace(outer=W.BC("bilinear", coeffs=(1.0 + 0j, 0j, 0j, 0j)))
    cls = fkmc.node_classes(p).ravel()
    # nodes at several radii, the edge's own nodes (on the circle) included
    ids = np.array([10 + 21 * 10 + d for d in (4, 6, 8, 10)] + [10 + 21 * 0, 0 + 21 * 10], dtype=np.int32)
    assert np.all(cls[ids] == 0)
    xs = p.x0 + (ids % p.nx) * 0.05
    ys = p.y0 + (ids // p.nx) * 0.05
    rho = np.hypot(xs - 0.5, ys - 0.5)
    est = fkmc.fk_nodes(p, None, 0, ids)
    a_eff = 0.15 - CF.bgk_beta() * math.sqrt(2.0 * h)
    ref = concentric_exact(which, rho, a=a_eff)
    err = np.abs(est["mean"].real - ref)
    assert np.all(err < 4.0 * est["se"].real + 0.015 * ref), (err, est["se"].real, ref)
    assert est["capped"].sum() == 0


def test_mc_curved_edge_local_time_uses_twice_the_overshoot():
    # power of the pin above: half the local-time increment (a plausible slip)
    # misses the closed form by far more than its tolerance
    p = concentric(2e-5, M=2000).replace(outer=W.BC("bilinear", coeffs=(0.5 + 0j, 0j, 0j, 0j)))
    ids = np.array([10 + 21 * 10 + 8], dtype=np.int32)
    est = fkmc.fk_nodes(p, None, 0, ids)
    full = concentric_exact("local_time", np.array([0.4]), a=0.15 - CF.bgk_beta() * math.sqrt(4e-5))[0]
    assert abs(est["mean"].real[0] - full) > 0.3 * full


def test_disc_domain_node_classes_and_paths_stay_in_the_disc():
    p = W.annulus_shape2(n=41, h=1e-4, k=0.5)
    cls = fkmc.node_classes(p)
    X, Y = np.meshgrid(np.linspace(p.x0, p.x1, p.nx), np.linspace(p.y0, p.y1, p.ny))
    outside = (X - 0.8) ** 2 + (Y - 0.5) ** 2 > 0.45 ** 2 * (1 + 1e-12)
    rhombus = np.abs(X - 0.8) / 0.075 + np.abs(Y - 0.5) / 0.075 <= 1 + 1e-9
    assert np.array_equal(cls == 2, rhombus) and np.array_equal(cls == 3, outside & ~rhombus)
    assert np.array_equal(cls == 0, ~outside & ~rhombus)
    ids = np.nonzero(cls.ravel() == 0)[0]
    for nid in (int(ids[0]), int(ids[len(ids) // 2]), int(ids[-1])):
        for m in range(4):
            s, J, cap, (x, y) = fkmc.path(p, None, 0, nid, m)
            assert not cap
            # ends in the closed rhombus (the oracle's test: |x - cx| ry +
            # |y - cy| r <= r ry)
            assert abs(x - 0.8) * 0.075 + abs(y - 0.5) * 0.075 <= 0.075 * 0.075
            assert (x - 0.8) ** 2 + (y - 0.5) ** 2 <= 0.45 ** 2


def test_rhombus_projection_is_the_nearest_boundary_point():
    p = W.annulus_shape2(n=21)
    rng = np.random.default_rng(2)
    t = np.linspace(0.0, 1.0, 20001)
    vx = np.array([0.875, 0.8, 0.725, 0.8, 0.875])
    vy = np.array([0.5, 0.575, 0.5, 0.425, 0.5])
    pts = np.concatenate([np.stack([vx[e] + t * (vx[e + 1] - vx[e]), vy[e] + t * (vy[e + 1] - vy[e])], 1)
                          for e in range(4)])
    for _ in range(200):
        x, y = 0.8 + rng.uniform(-0.2, 0.2), 0.5 + rng.uniform(-0.2, 0.2)
        which, (px, py) = fkmc.project(p, x, y)
        assert which == 2
        brute = np.min(np.hypot(pts[:, 0] - x, pts[:, 1] - y))
        assert abs(math.hypot(px - x, py - y) - brute) < 1e-5
        assert abs(abs(px - 0.8) / 0.075 + abs(py - 0.5) / 0.075 - 1.0) < 1e-12


def disc_plane_wave(theta=0.4, **kw):
    """Shape 2 (reading: the centred rhombus) with the plane wave's own data:
    its Robin datum on the circle, the wave itself on the rhombus."""
    return W.annulus_shape2(n=41, k=1.0, h=5e-5, M=8000, seed=23).replace(
        outer=W.BC("plane_wave_robin", 1.0, theta), inner=W.BC("plane_wave", 1.0, theta), **kw)


def disc_sample(p):
    """The five unknown nodes nearest the circle (their paths mirror at once
    and their cells are cut by it) and three inside."""
    X, Y = np.meshgrid(np.linspace(p.x0, p.x1, p.nx), np.linspace(p.y0, p.y1, p.ny))
    ids0 = np.nonzero(fkmc.node_classes(p).ravel() == 0)[0]
    rad = np.hypot(X.ravel()[ids0] - 0.8, Y.ravel()[ids0] - 0.5)
    return X, Y, np.concatenate([ids0[np.argsort(-rad)[:5]], ids0[np.argsort(rad)[[40, 200, 600]]]]).astype(np.int32)


@pytest.mark.parametrize("case", ["plain", "shifted_damped"])
def test_mc_curved_edge_plane_wave_is_fixed_point(case):
    # one step of the annular iteration at k > 0 from the exact solution
    # returns it on the disc domain: the Robin coupling i k I_h[u_n] + g2 at
    # the foot with the outward radial normal, the rhombus datum, and the
    # iterate read in the cells the circle cuts through the exterior nodes'
    # nearest unknown nodes.  The exterior entries of u_n hold 1e3: they are
    # never read themselves.
    kw = {} if case == "plain" else dict(alpha=2.0, damping=0.5)
    p = disc_plane_wave(**kw)
    X, Y, ids = disc_sample(p)
    exact = CF.plane_wave(p.k, 0.4, X, Y, damping=p.damping)
    u = exact.copy()
    u.ravel()[fkmc.node_classes(p).ravel() == 3] = 1e3
    est = fkmc.fk_nodes(p, u, 1, ids)
    err = np.abs(est["mean"] - exact.ravel()[ids])
    se = np.abs(est["se"])
    kappa = abs(np.sqrt(complex(p.k ** 2, p.damping)))
    bias = CF.bgk_beta() * math.sqrt(2.0 * p.h) * kappa
    # reading a neighbour's value instead of the extension moves I_h[u_n] on
    # the circle by at most |grad w| sqrt(2) dx; the local time (mean < 0.95)
    # multiplies it by k
    remap = p.k * kappa * math.sqrt(2.0) * ((p.x1 - p.x0) / (p.nx - 1)) * 0.95
    assert np.all(err < 5.0 * se + 2.0 * bias + remap), (err, se, bias, remap)
    assert est["capped"].sum() == 0


def test_mc_curved_edge_fixed_point_check_rejects_a_wrong_field():
    # power of the check above: the opposite plane wave solves the equation,
    # not the Robin condition with this g2 on the circle
    p = disc_plane_wave().replace(M=2000)
    X, Y, ids = disc_sample(p)
    other = CF.plane_wave(p.k, 0.4 + math.pi, X, Y)
    est = fkmc.fk_nodes(p, other, 1, ids)
    assert np.min(np.abs(est["mean"] - other.ravel()[ids])) > 0.5


def test_mc_curved_edge_never_reads_exterior_entries():
    p = disc_plane_wave().replace(M=600)
    X, Y, ids = disc_sample(p)
    u = CF.plane_wave(p.k, 0.4, X, Y)
    ext = fkmc.node_classes(p).ravel() == 3
    a, b = u.copy(), u.copy()
    a.ravel()[ext] = 0.0
    b.ravel()[ext] = -7.0 + 3.0j
    ea = fkmc.fk_nodes(p, a, 1, ids[:5])
    eb = fkmc.fk_nodes(p, b, 1, ids[:5])
    assert np.array_equal(ea["mean"], eb["mean"])
