"""Closed-form solutions that pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import math

import numpy as np


def plane_wave(k, theta, x, y, amp=1.0, damping=0.0):
    """amp exp(i kappa (x cos theta + y sin theta)) with kappa^2 = k^2 + i p:
    solves Delta u + (k^2 + i p) u = 0 everywhere, so with its own trace as
    Dirichlet datum it is the exact solution in any cavity (Sec. 1, the
    incident field; Sec. 2.2 with damping p)."""
    kappa = k if damping == 0.0 else complex(np.sqrt(complex(k * k, damping)))
    return amp * np.exp(1j * kappa * (np.asarray(x) * math.cos(theta) + np.asarray(y) * math.sin(theta)))


def disc_scattered(k, a, theta, x, y, nterms=50):
    """Sound-soft disc of radius a at the origin hit by the plane wave of
    direction theta.  Scattered field (outgoing, time factor exp(-i omega t) as
    in Sec. 1; u_sc = -u_inc on r = a as in Sec. 1's sound-soft condition):
        u_sc = - sum_{n<nterms} eps_n i^n J_n(ka)/H1_n(ka) H1_n(kr) cos(n (phi - theta)),
    eps_0 = 1, eps_n = 2.  scipy Bessel functions."""
    from scipy.special import hankel1, jv
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    r = np.hypot(x, y)
    ph = np.arctan2(y, x)
    out = np.zeros(np.broadcast(x, y).shape, dtype=complex)
    for n in range(nterms):
        eps = 1.0 if n == 0 else 2.0
        out -= eps * (1j ** n) * jv(n, k * a) / hankel1(n, k * a) * hankel1(n, k * r) * np.cos(n * (ph - theta))
    return out


def disc_scattered_mp(k, a, theta, x, y, nterms=50, dps=30):
    """The same series evaluated with mpmath at ``dps`` digits (an independent
    library, used to pin the scipy evaluation)."""
    import mpmath as mp
    mp.mp.dps = dps
    r = mp.sqrt(mp.mpf(x) ** 2 + mp.mpf(y) ** 2)
    ph = mp.atan2(mp.mpf(y), mp.mpf(x))
    s = mp.mpc(0)
    for n in range(nterms):
        eps = 1 if n == 0 else 2
        hka = mp.besselj(n, k * a) + 1j * mp.bessely(n, k * a)
        hkr = mp.besselj(n, k * r) + 1j * mp.bessely(n, k * r)
        s -= eps * (mp.mpc(0, 1) ** n) * mp.besselj(n, k * a) / hka * hkr * mp.cos(n * (ph - theta))
    return complex(s)


def torsion_rect(a, b, x, y, nterms=201):
    """Mean exit time E[tau] of y + sqrt(2) W from the rectangle (0,a)x(0,b):
    the solution of Delta E = -1, E = 0 on the boundary (Remark 2.5, eq. (2.10)),
    by its double sine series over odd m, n:
        E = sum 16 / (pi^4 m n (m^2/a^2 + n^2/b^2)) sin(m pi x/a) sin(n pi y/b)."""
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    out = np.zeros(np.broadcast(x, y).shape)
    ms = np.arange(1, nterms + 1, 2)
    for m in ms:
        sx = np.sin(m * math.pi * x / a)
        for n in ms:
            out += 16.0 / (math.pi ** 4 * m * n * (m * m / a ** 2 + n * n / b ** 2)) * sx * np.sin(n * math.pi * y / b)
    return out


def lambda1_rect(a, b):
    """First Dirichlet eigenvalue of -Delta on an a x b rectangle."""
    return math.pi ** 2 * (1.0 / a ** 2 + 1.0 / b ** 2)


def lambda1h_rect(nx, ny, a, b):
    """First eigenvalue of the 5-point -Delta_h with Dirichlet edges on an
    nx x ny node grid of the a x b rectangle."""
    dx, dy = a / (nx - 1), b / (ny - 1)
    return 4.0 / dx ** 2 * math.sin(math.pi * dx / (2 * a)) ** 2 + 4.0 / dy ** 2 * math.sin(math.pi * dy / (2 * b)) ** 2


def kstar_cavity(max_exit_time, p=0.0):
    """k_*^C = sqrt(1 / max E[tau] - p)  (Remark 2.4, eq. (2.9))."""
    return math.sqrt(1.0 / max_exit_time - p)


def bgk_beta():
    """Broadie-Glasserman-Kou continuity correction constant
    beta = -zeta(1/2) / sqrt(2 pi) ~ 0.5826: a discretely monitored barrier with
    per-step standard deviation s behaves like a continuous barrier moved out
    by beta s."""
    import mpmath as mp
    return float(-mp.zeta(0.5) / mp.sqrt(2 * mp.pi))
