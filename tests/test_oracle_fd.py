"""Pins of the finite-difference and closed-form parts of the oracle (CPU).

* the 5-point direct solve converges to the plane wave at second order and
  equals a dense brute-force solve on small grids;
* the Neumann-series iterate equals the direct solve when k^2 < lambda_1^h and
  grows by the spectral radius k^2/lambda_1^h per step when above (Sec. 2.4);
  the DST and sparse-LU iterates agree;
* lambda_1^h: closed form against a sparse eigensolver;
* the exit-time (torsion) series against FD, and k_*^C of the unit square
  below k_max = pi sqrt(2) (Remark 2.4 and Sec. 3);
* the sound-soft disc series: scipy against mpmath, the boundary condition on
  the circle, the Helmholtz residual and the outgoing decay.
"""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import fd, fkmc
from paper_2308_11469_amd import workloads as W


def cavity(N, k=2.0, theta=math.pi / 6):
    return W.Problem(nx=N, ny=N, k=k, outer=W.BC("plane_wave", 1.0 + 0j, theta))


def test_direct_second_order_to_plane_wave():
    errs = []
    for N in (9, 17, 33, 65):
        p = cavity(N, k=3.0)
        u = fd.direct(p)
        errs.append(np.max(np.abs(u - W.exact_solution(p))))
    rates = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in rates), rates


@pytest.mark.parametrize("N", [5, 9, 17])
def test_direct_sparse_equals_dense(N):
    p = cavity(N, k=2.5).replace(src_kind="gaussian", src_amp=1 + 0.5j, src_cx=0.3, src_cy=0.6, src_sigma=0.1)
    a = fd.direct(p)
    b = fd.direct(p, dense=True)
    assert np.max(np.abs(a - b)) < 1e-12


def test_neumann_series_converges_to_direct_below_lambda1():
    p = cavity(17, k=3.0)
    its = fd.neumann(p, 80)
    assert np.max(np.abs(its[-1] - fd.direct(p))) < 1e-12
    rho = 9.0 / cf.lambda1h_rect(17, 17, 1, 1)
    d = [np.max(np.abs(its[i + 1] - its[i])) for i in range(len(its) - 1)]
    assert abs(d[20] / d[19] - rho) < 1e-6


def test_neumann_series_diverges_above_lambda1():
    p = cavity(17, k=4.6)
    lam = cf.lambda1h_rect(17, 17, 1, 1)
    assert 4.6 ** 2 > lam
    its = fd.neumann(p, 200)
    d = [np.max(np.abs(its[i + 1] - its[i])) for i in range(len(its) - 1)]
    assert abs(d[-1] / d[-2] - 4.6 ** 2 / lam) < 1e-6
    assert d[-1] > 1e3 * d[0]


def test_damped_direct_second_order_to_damped_plane_wave():
    # Delta u + (k^2 + i p) u = 0 with the damped plane wave as data
    errs = []
    for N in (9, 17, 33, 65):
        p = cavity(N, k=3.0).replace(damping=2.5)
        u = fd.direct(p)
        ex = cf.plane_wave(3.0, math.pi / 6, *np.meshgrid(np.linspace(0, 1, N), np.linspace(0, 1, N)),
                           damping=2.5)
        errs.append(np.max(np.abs(u - ex)))
    rates = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in rates), rates
    # the data really are damped: the wave decays along its direction
    assert abs(ex[-1, -1]) < 0.8 * abs(ex[0, 0])


def test_neumann_with_shift_and_damping_contracts_at_its_spectral_radius():
    # (Delta_h - (alpha - k^2)) u_{n+1} = f - (alpha + i p) u_n: mode m is
    # multiplied by -(alpha + i p) / (lambda_m + alpha - k^2); the smallest
    # lambda_m dominates
    k, alpha, damp = 2.0, 7.0, 3.0
    p = cavity(17, k=k).replace(alpha=alpha, damping=damp)
    its = fd.neumann(p, 80)
    assert np.max(np.abs(its[-1] - fd.direct(p))) < 1e-12
    lam = cf.lambda1h_rect(17, 17, 1, 1)
    rho = abs(complex(alpha, damp)) / (lam + alpha - k * k)
    d = [np.max(np.abs(its[i + 1] - its[i])) for i in range(len(its) - 1)]
    assert abs(d[10] / d[9] - rho) < 1e-6


def test_dst_iterate_equals_lu_iterate():
    p = cavity(33, k=2.0).replace(x1=1.5, nx=49, src_kind="gaussian", src_amp=1 + 0.5j,
                                  src_cx=0.3, src_cy=0.6, src_sigma=0.05)
    a = fd.neumann(p, 6)
    b = fd.neumann_dst(p, 6)
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) < 1e-12


@pytest.mark.parametrize("nx,ny,a,b", [(9, 9, 1, 1), (65, 65, 1, 1), (33, 17, 2.0, 0.7)])
def test_lambda1h_closed_form_vs_eigensolver(nx, ny, a, b):
    p = W.Problem(x1=a, y1=b, nx=nx, ny=ny)
    assert math.isclose(fd.lambda1h(p), cf.lambda1h_rect(nx, ny, a, b), rel_tol=1e-9)


def test_lambda1h_limits_and_domain_monotonicity():
    assert abs(cf.lambda1h_rect(513, 513, 1, 1) - 2 * math.pi ** 2) < 1e-3
    holed = W.scatter_problem(k=2.0, theta=0.0, N=65, M=64, seed=1, table_len=256)
    lam_holed = fd.lambda1h(holed)
    lam_box = cf.lambda1h_rect(65, 65, 2.0, 2.0)
    assert lam_holed > 2 * lam_box          # the hole raises lambda_1 (smaller domain)


def test_torsion_series_vs_fd_and_kstar():
    p = W.Problem(nx=65, ny=65)
    E = fd.torsion(p)
    xs = np.arange(65) / 64
    X, Y = np.meshgrid(xs, xs)
    S = cf.torsion_rect(1, 1, X, Y)
    assert np.max(np.abs(E - S)) < 5e-5
    emax = float(cf.torsion_rect(1, 1, 0.5, 0.5))
    kc = cf.kstar_cavity(emax)
    assert 3.68 < kc < 3.69
    assert kc < math.pi * math.sqrt(2)      # sufficient bound below the true k_max
    # rectangle scaling E_{L Omega}(L x) = L^2 E_Omega(x)
    assert math.isclose(float(cf.torsion_rect(2, 2, 1.0, 0.6)), 4 * float(cf.torsion_rect(1, 1, 0.5, 0.3)),
                        rel_tol=1e-12)


@pytest.mark.parametrize("damping", [0.0, 2.0, 6.0])
def test_cavity_kstar_with_damping_is_a_sufficient_bound(damping):
    # Theorem 2.2 asks (alpha + p) E[tau] < 1 with alpha >= k^2; at alpha = k^2
    # that is k < k_*^C = sqrt(1 / max E[tau] - p) (eq. (2.9)).  On the FD
    # model the increments of the iteration shrink by |k^2 + i p| / lambda_1^h
    # per step, and max E >= 1 / lambda_1^h, so at k_*^C the iteration must
    # contract, with room to spare; it diverges only past
    # k_max = (lambda_1^h^2 - p^2)^(1/4), which lies above k_*^C.  (Without
    # damping the contraction at k_*^C is exactly 1 / (max E lambda_1^h).)
    n = 33
    base = cavity(n, k=1.0).replace(damping=damping)
    emax = float(fd.torsion(base).max())
    lam = cf.lambda1h_rect(n, n, 1, 1)
    kc = cf.kstar_cavity(emax, damping)
    assert emax * lam > 1.0
    assert abs((kc * kc + damping) * emax - 1.0) < 1e-12
    kmax = (lam * lam - damping * damping) ** 0.25
    assert kc < kmax

    def growth(k):
        its = fd.neumann(base.replace(k=k), 24)   # increments still far above rounding
        d = [np.max(np.abs(its[i + 1] - its[i])) for i in range(len(its) - 1)]
        return d[-1] / d[-2]

    r = growth(kc)
    assert abs(r - abs(complex(kc * kc, damping)) / lam) < 1e-6
    assert r <= 1.0 / (emax * lam) + 1e-6 < 1.0
    assert growth(1.03 * kmax) > 1.0
    # the bound falls as the damping grows
    assert cf.kstar_cavity(emax, damping + 1.0) < kc


def test_bgk_constant():
    assert abs(cf.bgk_beta() - 0.5825971579) < 1e-9


@pytest.mark.parametrize("k,x,y", [(1.0, 0.5, 0.2), (4.0, -0.9, 0.7), (2.5, 1.0, -1.0), (3.3, 0.26, 0.0)])
def test_disc_series_scipy_vs_mpmath(k, x, y):
    a = cf.disc_scattered(k, 0.25, 0.7, x, y)
    b = cf.disc_scattered_mp(k, 0.25, 0.7, x, y)
    assert abs(a - b) < 1e-12 * max(1.0, abs(b))
    # the workload module's own evaluation agrees
    assert abs(W.disc_scattered(k, 0.25, 0.7, x, y) - b) < 1e-12 * max(1.0, abs(b))


def test_disc_series_boundary_condition_and_pde():
    k, a, th = 3.0, 0.25, 1.1
    phi = np.linspace(0, 2 * math.pi, 37)
    x, y = a * np.cos(phi), a * np.sin(phi)
    usc = cf.disc_scattered(k, a, th, x, y)
    assert np.max(np.abs(usc + cf.plane_wave(k, th, x, y))) < 1e-12
    # Helmholtz residual by centred differences (second order in the step)
    for (x0, y0) in [(0.6, 0.1), (-0.4, -0.7)]:
        res = []
        for e in (1e-2, 5e-3):
            c = cf.disc_scattered(k, a, th, x0, y0)
            lap = (cf.disc_scattered(k, a, th, x0 + e, y0) + cf.disc_scattered(k, a, th, x0 - e, y0)
                   + cf.disc_scattered(k, a, th, x0, y0 + e) + cf.disc_scattered(k, a, th, x0, y0 - e) - 4 * c) / e ** 2
            res.append(abs(lap + k ** 2 * c))
        assert res[1] < res[0] / 3 and res[1] < 1e-3
    # outgoing: sqrt(r) |u_sc| tends to a constant along a ray
    r = np.array([50.0, 100.0, 200.0])
    v = np.sqrt(r) * np.abs(cf.disc_scattered(k, a, th, r * math.cos(th), r * math.sin(th)))
    assert abs(v[2] / v[1] - 1) < 0.02 and abs(v[1] / v[0] - 1) < 0.04


def test_fd_on_disc_domain_approaches_series():
    errs = []
    for N in (33, 65, 129):
        p = W.scatter_problem(k=2.0, theta=0.4, N=N, M=64, seed=1, table_len=8192)
        u = fd.direct(p)
        cls = fkmc.node_classes(p)
        ex = W.exact_solution(p)
        errs.append(np.max(np.abs(u - ex)[cls == 0]))
    # the staircase treatment of the circle is first order
    assert errs[2] < errs[1] < errs[0]
    assert errs[0] / errs[2] > 2.5 and errs[2] < 0.06
