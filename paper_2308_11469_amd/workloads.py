"""Seeded, synthetic problem descriptions for the Feynman-Kac Helmholtz path.

This module is the one place both the HIP library's callers and the CPU oracle
take their inputs from.  It holds problem *descriptions* only (geometry, data,
sampling parameters and seeds) and the closed-form boundary data of the
workloads; it contains none of the estimator's arithmetic and imports neither
the HIP binding nor the oracle.

Workloads (the paper runs no Monte Carlo experiments of its own; these are
synthetic stand-ins shaped like its two scenarios, the cavity of Sec. 2.2 and
plane-wave scattering by a sound-soft obstacle of Sec. 1):

* ``cavity_small``   unit square, 9x9 grid, plane-wave data, k = 2, M = 500,
                     h = 2e-3, 10 fixed-point iterations, FP64, seed 1.
* ``cavity_65``      unit square, 65x65 grid, k in {1, 2, 3, 4} (4.6 diverges),
                     M = 4096, h = 1e-4, up to 40 iterations, FP64.
* ``cavity_source``  unit square, 129x129, k = 3.5, complex Gaussian source,
                     M = 16384, h = 5e-5, FP32 stepping.
* ``rect_batch``     256 rectangles with random sides, grids, k, theta, M.
* ``scatter_stream`` sound-soft disc r = 0.25 in [-1, 1]^2 with exact outer
                     Dirichlet data from the Hankel series, Poisson arrivals.
* ``annulus_shape1`` / ``annulus_shape3`` / ``annulus_fig2``  the annular
                     problems of Sec. 2.3 and Sec. 2.5: a rectangle whose edge
                     carries the Robin condition d_n u - i k u = 0 (reflected
                     paths with local time) around an absorbing hole with
                     u = -exp(-i k x); the geometries of the paper's shapes 1
                     and 3 and of its finite-difference example.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

RECT = "rect"
RECT_MINUS_DISC = "rect_minus_disc"
RECT_MINUS_BOX = "rect_minus_box"
# the disc inscribed in the square [x0, x1] x [y0, y1], with a reflecting
# edge, minus a closed rhombus |x - cx| / r + |y - cy| / ry <= 1 or a closed
# disc of radius r at (cx, cy)
DISC_MINUS_RHOMBUS = "disc_minus_rhombus"
DISC_MINUS_DISC = "disc_minus_disc"


@dataclass
class BC:
    """Datum on one boundary part: the Dirichlet value, or on a reflecting
    edge the Robin datum g2 of d_n u - i k u = g2.

    kind: ``zero``; ``plane_wave`` (``amp * exp(i k (x cos theta + y sin theta))``
    with the problem's k); ``bilinear`` (``c0 + c1 x + c2 y + c3 x y`` with complex
    ``coeffs``, harmonic); ``table`` (complex samples at equal arclength steps
    round the rectangle, counter-clockwise from ``(x0, y0)``; outer boundary only);
    ``plane_wave_robin`` (reflecting edge only: the Robin datum of the plane
    wave of ``plane_wave``, so that the plane wave solves the Robin problem).
    """
    kind: str = "zero"
    amp: complex = 1.0 + 0.0j
    theta: float = 0.0
    coeffs: Tuple[complex, complex, complex, complex] = (0j, 0j, 0j, 0j)
    table: Optional[np.ndarray] = None


@dataclass
class Problem:
    """One Helmholtz instance  Delta u + k^2 u = f in Omega, u = g on dOmega.

    Omega is the open rectangle ``(x0, x1) x (y0, y1)``, minus the closed disc
    of radius ``r`` at ``(cx, cy)`` when ``domain_kind == 'rect_minus_disc'``,
    or minus the closed box ``[cx - r, cx + r] x [cy - ry, cy + ry]`` when
    ``domain_kind == 'rect_minus_box'``.  With ``reflect`` the rectangle's
    edge belongs to the domain and carries the Robin condition
    ``d_n u - i k u = g2`` (``outer`` gives g2); the hole stays Dirichlet.
    The grid has ``nx * ny`` nodes including the edges; node ``(i, j)`` has id
    ``i + nx * j``.
    """
    domain_kind: str = RECT
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    cx: float = 0.0
    cy: float = 0.0
    r: float = 0.0
    ry: float = 0.0
    reflect: bool = False
    nx: int = 9
    ny: int = 9
    # source f: 'zero' | 'const' (src_amp) | 'gaussian' (src_amp * exp(-|x-c|^2 / (2 sigma^2)))
    src_kind: str = "zero"
    src_amp: complex = 0j
    src_cx: float = 0.0
    src_cy: float = 0.0
    src_sigma: float = 1.0
    outer: BC = field(default_factory=BC)
    inner: BC = field(default_factory=BC)
    k: float = 0.0
    # shift alpha >= k^2 of the iteration (None: k^2) and damping p of
    # Delta u + (k^2 + i p) u = f (Sec. 2.2); plane-wave data then use the
    # wavenumber sqrt(k^2 + i p)
    alpha: Optional[float] = None
    damping: float = 0.0
    h: float = 1e-3
    M: int = 64
    seed: int = 1
    jmax: int = 0            # 0: ceil(40 / (lambda_1(bounding rectangle) h))
    crn: bool = False        # common random numbers across iterations
    g_unprojected: bool = False  # verification variant: g at X_J, not at its projection
    precision: int = 64
    max_iters: int = 10
    tol: float = 0.0
    name: str = ""

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny


# ----------------------------------------------------------------- exact data

def plane_wave(k: float, theta: float, x, y, amp: complex = 1.0, damping: float = 0.0):
    """``amp * exp(i kappa (x cos theta + y sin theta))`` with kappa =
    sqrt(k^2 + i p) (principal root; kappa = k when p = 0): an entire solution
    of Delta u + (k^2 + i p) u = 0 (the incident field of Sec. 1, damped as in
    Sec. 2.2)."""
    kappa = k if damping == 0.0 else complex(np.sqrt(complex(k * k, damping)))
    return amp * np.exp(1j * kappa * (np.asarray(x) * math.cos(theta) + np.asarray(y) * math.sin(theta)))


def disc_scattered(k: float, a: float, theta: float, x, y, nterms: int = 50, amp: complex = 1.0):
    """Field scattered by the sound-soft disc |x| <= a from the plane wave of
    direction theta: ``u_sc = -sum_n eps_n i^n J_n(ka)/H1_n(ka) H1_n(kr) cos(n(phi-theta))``
    (Jacobi-Anger expansion of the incident wave; outgoing H1 for the time
    factor exp(-i omega t) of Sec. 1; u_sc = -u_inc on r = a)."""
    from scipy.special import hankel1, jv
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    rr = np.hypot(x, y)
    ph = np.arctan2(y, x)
    out = np.zeros(np.broadcast(x, y).shape, dtype=np.complex128)
    rmin = float(np.min(rr)) if rr.size else 1.0
    rmax = float(np.max(rr)) if rr.size else 1.0
    for n in range(nterms):
        eps = 1.0 if n == 0 else 2.0
        coef = eps * (1j ** n) * jv(n, k * a) / hankel1(n, k * a)
        # |H1_n| decreases in its argument, so |coef H1_n(k rmin)| bounds the
        # term on every point; past n = k rmax the terms only shrink, and a
        # bound below 1e-20 is under half an ulp of any sample of size 1e-3
        if n > k * rmax and abs(coef) * abs(hankel1(n, k * rmin)) < 1e-20:
            break
        out -= coef * hankel1(n, k * rr) * np.cos(n * (ph - theta))
    return amp * out


def perimeter_points(x0, x1, y0, y1, L):
    """L points at equal arclength steps round the rectangle, counter-clockwise
    from (x0, y0)."""
    a, b = x1 - x0, y1 - y0
    s = np.arange(L) * (2.0 * (a + b) / L)
    px = np.empty(L)
    py = np.empty(L)
    e0 = s < a
    e1 = (s >= a) & (s < a + b)
    e2 = (s >= a + b) & (s < 2 * a + b)
    e3 = s >= 2 * a + b
    px[e0], py[e0] = x0 + s[e0], y0
    px[e1], py[e1] = x1, y0 + (s[e1] - a)
    px[e2], py[e2] = x1 - (s[e2] - a - b), y1
    px[e3], py[e3] = x0, y1 - (s[e3] - 2 * a - b)
    return px, py


def exact_solution(p: Problem) -> Optional[np.ndarray]:
    """Exact u at every grid node (complex, shape (ny, nx)) when the workload
    has one: the plane wave (cavity with plane-wave data and f = 0) or the disc
    series (scattering workload).  None otherwise."""
    xs = p.x0 + np.arange(p.nx) * ((p.x1 - p.x0) / (p.nx - 1))
    ys = p.y0 + np.arange(p.ny) * ((p.y1 - p.y0) / (p.ny - 1))
    X, Y = np.meshgrid(xs, ys)
    if p.src_kind != "zero":
        return None
    if p.domain_kind == RECT and p.outer.kind == "plane_wave":
        return plane_wave(p.k, p.outer.theta, X, Y, p.outer.amp, p.damping)
    if p.damping != 0.0:
        return None
    if p.domain_kind == RECT_MINUS_DISC and p.outer.kind == "table" and p.inner.kind == "plane_wave":
        inc_amp = -p.inner.amp
        return disc_scattered(p.k, p.r, p.inner.theta, X - p.cx, Y - p.cy, amp=inc_amp)
    return None


# ------------------------------------------------------------------ workloads

def cavity_small() -> Problem:
    """Unit square, 9x9 grid (49 interior nodes), g = plane wave theta = pi/6,
    k = 2, f = 0, u_0 = 0, 10 iterations, M = 500, h = 2e-3, FP64, seed 1."""
    return Problem(name="cavity_9x9_k2_M500", nx=9, ny=9, k=2.0, h=2e-3, M=500, seed=1,
                   outer=BC("plane_wave", 1.0 + 0j, math.pi / 6), precision=64,
                   max_iters=10, tol=0.0)


def cavity_65(k: float = 2.0, precision: int = 64) -> Problem:
    """Unit square, 65x65 grid (3969 interior nodes), plane-wave data theta =
    pi/6, M = 4096, h = 1e-4, up to 40 iterations to a 1e-6 change, seed 1."""
    return Problem(name="cavity_65x65_k%g_M4096" % k, nx=65, ny=65, k=k, h=1e-4, M=4096,
                   seed=1, outer=BC("plane_wave", 1.0 + 0j, math.pi / 6),
                   precision=precision, max_iters=40, tol=1e-6)


def cavity_source(precision: int = 32) -> Problem:
    """Unit square, 129x129, k = 3.5, f = (1 + 0.5i) exp(-|x - (0.3, 0.6)|^2 /
    (2 0.05^2)) plus plane-wave data theta = pi/6, M = 16384, h = 5e-5."""
    return Problem(name="cavity_129x129_k3.5_gauss_M16384", nx=129, ny=129, k=3.5, h=5e-5,
                   M=16384, seed=1, src_kind="gaussian", src_amp=1.0 + 0.5j,
                   src_cx=0.3, src_cy=0.6, src_sigma=0.05,
                   outer=BC("plane_wave", 1.0 + 0j, math.pi / 6),
                   precision=precision, max_iters=40, tol=1e-6)


def _round64(m: float) -> int:
    return int(max(64, 64 * round(m / 64.0)))


def rect_batch(n: int = 256, precision: int = 32, seed: int = 4) -> List[Problem]:
    """Rectangles [0, a] x [0, b], a, b ~ U[0.5, 2]; nx, ny ~ U{33..257};
    k = c pi sqrt(1/a^2 + 1/b^2), c ~ U[0.2, 0.9]; theta ~ U[0, 2 pi);
    M log-uniform on [1024, 16384] rounded to 64; h = 1e-4; instance i has
    seed 1000 + i.  Parameters drawn in that order per instance from PCG64."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        a = float(rng.uniform(0.5, 2.0))
        b = float(rng.uniform(0.5, 2.0))
        nx = int(rng.integers(33, 258))
        ny = int(rng.integers(33, 258))
        c = float(rng.uniform(0.2, 0.9))
        th = float(rng.uniform(0.0, 2 * math.pi))
        M = _round64(math.exp(rng.uniform(math.log(1024), math.log(16384))))
        k = c * math.pi * math.sqrt(1 / a ** 2 + 1 / b ** 2)
        out.append(Problem(name="rect%03d" % i, x0=0.0, x1=a, y0=0.0, y1=b, nx=nx, ny=ny,
                           k=k, h=1e-4, M=M, seed=1000 + i,
                           outer=BC("plane_wave", 1.0 + 0j, th), precision=precision,
                           max_iters=40, tol=1e-3))
    return out


def scatter_problem(k: float, theta: float, N: int, M: int, seed: int, precision: int = 32,
                    h: float = 1e-4, table_len: int = 4 * 8192, name: str = "") -> Problem:
    """[-1, 1]^2 minus the sound-soft disc r = 0.25 at the origin.  Unknown:
    the scattered field; inner datum -u_inc (a plane wave of amplitude -1);
    outer datum the exact scattered field sampled from the disc series."""
    px, py = perimeter_points(-1.0, 1.0, -1.0, 1.0, table_len)
    tab = disc_scattered(k, 0.25, theta, px, py)
    return Problem(name=name or "scatter_k%.3f_N%d" % (k, N), domain_kind=RECT_MINUS_DISC,
                   x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, cx=0.0, cy=0.0, r=0.25, nx=N, ny=N,
                   k=k, h=h, M=M, seed=seed,
                   outer=BC("table", table=tab.astype(np.complex128)),
                   inner=BC("plane_wave", -1.0 + 0j, theta), precision=precision,
                   max_iters=40, tol=1e-3)


def _annulus(name, x0, x1, y0, y1, hole, nx, ny, k, h, M, jmax, precision, seed):
    """Rectangle with a reflecting (Robin) edge around an absorbing hole;
    inner datum u = -exp(-i k x) (the plane wave of amplitude -1 and
    direction theta = pi), Robin datum g2 = 0 (Sec. 2.3)."""
    kind, cx, cy, r, ry = hole
    return Problem(name=name, domain_kind=kind, x0=x0, x1=x1, y0=y0, y1=y1, cx=cx, cy=cy, r=r, ry=ry,
                   reflect=True, nx=nx, ny=ny, k=k, h=h, M=M, seed=seed, jmax=jmax,
                   outer=BC("zero"), inner=BC("plane_wave", -1.0 + 0j, math.pi),
                   precision=precision, max_iters=30, tol=0.0)


def annulus_shape1(k: float = 1.5, n: int = 61, M: int = 4096, h: float = 1e-4, precision: int = 64,
                   seed: int = 11) -> Problem:
    """The paper's shape 1: the square [-0.3, 0.3]^2 with the circular hole of
    radius 0.15 at the origin; n x n grid.  Step cap 40 x 0.25 / h: the
    mean exit time is at most about 0.03 here."""
    return _annulus("annulus_shape1_k%g_n%d" % (k, n), -0.3, 0.3, -0.3, 0.3,
                    (RECT_MINUS_DISC, 0.0, 0.0, 0.15, 0.0), n, n, k, h, M, int(math.ceil(10.0 / h)),
                    precision, seed)


def annulus_shape3(k: float = 0.5, nx: int = 41, ny: int = 65, M: int = 4096, h: float = 1e-4,
                   precision: int = 64, seed: int = 13) -> Problem:
    """The paper's shape 3: the rectangle [-0.5, 0.5] x [-0.8, 0.8] with the
    rectangular hole [-0.05, 0.05] x [-0.4, 0.4]; nx x ny grid (41 x 65
    puts the hole's edges on grid lines).  Step cap 40 x 1.6 / h: the mean
    exit time is at most about 0.2 here."""
    return _annulus("annulus_shape3_k%g_%dx%d" % (k, nx, ny), -0.5, 0.5, -0.8, 0.8,
                    (RECT_MINUS_BOX, 0.0, 0.0, 0.05, 0.4), nx, ny, k, h, M, int(math.ceil(64.0 / h)),
                    precision, seed)


def annulus_shape2(k: float = 0.0, n: int = 41, M: int = 4096, h: float = 1e-4, precision: int = 64,
                   seed: int = 12) -> Problem:
    """The paper's shape 2 as read here: the disc of radius 0.45 at
    (0.8, 0.5) with a reflecting edge, minus the rhombus of diagonals 0.15
    (half-diagonals 0.075 along x and y) at the disc's centre (the printed
    hole centre (0, 0) lies outside the disc); n x n grid on the disc's
    bounding square.  Step cap 60 / h."""
    return _annulus("annulus_shape2", 0.35, 1.25, 0.05, 0.95, (DISC_MINUS_RHOMBUS, 0.8, 0.5, 0.075, 0.075),
                    n, n, k, h, M, int(math.ceil(60.0 / h)), precision, seed)


def annulus_fig2(k: float = 0.8, n: int = 21, M: int = 4096, h: float = 1e-4, precision: int = 64,
                 seed: int = 17) -> Problem:
    """The finite-difference example of Sec. 2.4: the square [-0.5, 0.5]^2
    with the square hole [-0.15, 0.15]^2; n x n grid (21: grid step 0.05,
    the hole's edges on grid lines)."""
    return _annulus("annulus_fig2_k%g_n%d" % (k, n), -0.5, 0.5, -0.5, 0.5,
                    (RECT_MINUS_BOX, 0.0, 0.0, 0.15, 0.15), n, n, k, h, M, int(math.ceil(20.0 / h)),
                    precision, seed)


def scatter_stream(n: int = 400, rate: float = 200.0, seed: int = 5, precision: int = 32):
    """Request stream for the serving workload: k ~ U[1, 4], theta ~ U[0, 2 pi),
    N ~ U{33..257}, M log-uniform on [1024, 8192] rounded to 64, exponential
    inter-arrival gaps at ``rate`` per second; request r has seed 5000 + r.
    Returns (arrival_times, parameter dicts); tables are built on admission."""
    rng = np.random.default_rng(seed)
    t = 0.0
    arrivals, params = [], []
    for r in range(n):
        t += float(rng.exponential(1.0 / rate))
        k = float(rng.uniform(1.0, 4.0))
        th = float(rng.uniform(0.0, 2 * math.pi))
        N = int(rng.integers(33, 258))
        M = _round64(math.exp(rng.uniform(math.log(1024), math.log(8192))))
        arrivals.append(t)
        params.append(dict(k=k, theta=th, N=N, M=M, seed=5000 + r, precision=precision))
    return arrivals, params
