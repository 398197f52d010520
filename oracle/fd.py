"""Five-point finite differences for the Helmholtz problem and its iteration.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``direct``: the 5-point discretisation of Delta u + k^2 u = f on interior
  nodes with the Dirichlet values moved to the right-hand side, solved by
  sparse LU (complex128).
* ``neumann``: the fixed-point iterate Delta_h u_{n+1} = f - k^2 u_n with the
  same Dirichlet values, u_0 = 0.  In matrix form u_{n+1} = b + G u_n with
  G = k^2 (-Delta_h)^{-1} on interior nodes; the Neumann series converges iff
  the spectral radius of G is below one (Sec. 2.4), here iff k^2 < lambda_1^h.
* ``neumann_dst``: the same iterate on rectangles by the type-I discrete sine
  transform, which diagonalises Delta_h.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fkmc


def _grid(p):
    xs = p.x0 + np.arange(p.nx) * ((p.x1 - p.x0) / (p.nx - 1))
    ys = p.y0 + np.arange(p.ny) * ((p.y1 - p.y0) / (p.ny - 1))
    return np.meshgrid(xs, ys)


def source_grid(p) -> np.ndarray:
    X, Y = _grid(p)
    if p.src_kind == "zero":
        return np.zeros_like(X, dtype=complex)
    if p.src_kind == "const":
        return np.full(X.shape, complex(p.src_amp))
    if p.src_kind == "gaussian":
        return complex(p.src_amp) * np.exp(-((X - p.src_cx) ** 2 + (Y - p.src_cy) ** 2) / (2 * p.src_sigma ** 2))
    raise ValueError(p.src_kind)


def laplacian(p):
    """(L, ids, B): L is the 5-point Delta_h restricted to interior nodes (ids,
    grid order), B maps the full grid's Dirichlet values to the interior
    right-hand-side contribution, so Delta_h u = L u_int + B u_full."""
    cls = fkmc.node_classes(p).ravel()
    ids = np.nonzero(cls == 0)[0]
    pos = -np.ones(p.nx * p.ny, dtype=np.int64)
    pos[ids] = np.arange(len(ids))
    dx = (p.x1 - p.x0) / (p.nx - 1)
    dy = (p.y1 - p.y0) / (p.ny - 1)
    rows, cols, vals = [], [], []
    brow, bcol, bval = [], [], []
    for r, g in enumerate(ids):
        i, j = g % p.nx, g // p.nx
        rows.append(r); cols.append(r); vals.append(-2.0 / dx ** 2 - 2.0 / dy ** 2)
        for (ii, jj, w) in ((i - 1, j, 1 / dx ** 2), (i + 1, j, 1 / dx ** 2),
                            (i, j - 1, 1 / dy ** 2), (i, j + 1, 1 / dy ** 2)):
            nb = ii + p.nx * jj
            if pos[nb] >= 0:
                rows.append(r); cols.append(pos[nb]); vals.append(w)
            else:
                brow.append(r); bcol.append(nb); bval.append(w)
    n = len(ids)
    L = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    B = sp.csr_matrix((bval, (brow, bcol)), shape=(n, p.nx * p.ny))
    return L, ids, B


def direct(p, dense=False) -> np.ndarray:
    """Direct 5-point solve of (Delta_h + k^2 + i p) u = f (p the damping of
    Sec. 2.2, eq. (2.4)); returns the full complex grid (ny, nx) with
    Dirichlet values on edge and hole nodes."""
    L, ids, B = laplacian(p)
    full = fkmc.boundary_grid(p)
    f = source_grid(p).ravel()[ids]
    rhs = f - B @ full.ravel()
    A = (L.astype(complex) + complex(p.k ** 2, p.damping) * sp.identity(L.shape[0], format="csc"))
    if dense:
        sol = np.linalg.solve(A.toarray(), rhs)
    else:
        sol = spla.spsolve(A.tocsc(), rhs)
    out = full.copy()
    out.ravel()[ids] = sol
    return out


def neumann(p, n_iters, u0=None):
    """Iterates of (Delta_h - (alpha - k^2)) u_{n+1} = f - (alpha + i p) u_n
    (Dirichlet g; alpha = k^2 and p = 0 unless the problem sets them: the
    FD form of the iteration of Sec. 2.2), u_0 = 0 unless given.  Returns the
    list [u_1, ..., u_n_iters] of full grids."""
    L, ids, B = laplacian(p)
    alpha = p.k ** 2 if p.alpha is None else p.alpha
    c = alpha - p.k ** 2
    lu = spla.splu((L - c * sp.identity(L.shape[0], format="csc")).tocsc())
    full = fkmc.boundary_grid(p)
    f = source_grid(p).ravel()[ids]
    bterm = B @ full.ravel()
    u_int = np.zeros(len(ids), dtype=complex) if u0 is None else np.asarray(u0).ravel()[ids].astype(complex)
    out = []
    for _ in range(n_iters):
        rhs = f - complex(alpha, p.damping) * u_int - bterm
        u_int = lu.solve(rhs.real) + 1j * lu.solve(rhs.imag)
        g = full.copy()
        g.ravel()[ids] = u_int
        out.append(g)
    return out


def neumann_dst(p, n_iters):
    """``neumann`` for a plain rectangle by the DST-I, which diagonalises the
    interior 5-point Laplacian: mode (m, n) has eigenvalue
    -(4/dx^2 sin^2(m pi/(2(nx-1))) + 4/dy^2 sin^2(n pi/(2(ny-1))))."""
    from scipy.fft import dstn, idstn
    assert p.domain_kind == "rect"
    L, ids, B = laplacian(p)
    full = fkmc.boundary_grid(p)
    nxi, nyi = p.nx - 2, p.ny - 2
    dx = (p.x1 - p.x0) / (p.nx - 1)
    dy = (p.y1 - p.y0) / (p.ny - 1)
    mx = np.arange(1, nxi + 1)
    my = np.arange(1, nyi + 1)
    lam = -(4 / dx ** 2 * np.sin(mx[None, :] * np.pi / (2 * (p.nx - 1))) ** 2
            + 4 / dy ** 2 * np.sin(my[:, None] * np.pi / (2 * (p.ny - 1))) ** 2)
    f = source_grid(p)[1:-1, 1:-1]
    bterm = (B @ full.ravel()).reshape(nyi, nxi)
    u = np.zeros((nyi, nxi), dtype=complex)
    out = []
    for _ in range(n_iters):
        rhs = f - p.k ** 2 * u - bterm
        u = idstn(dstn(rhs.real, type=1) / lam, type=1) + 1j * idstn(dstn(rhs.imag, type=1) / lam, type=1)
        g = full.copy()
        g[1:-1, 1:-1] = u
        out.append(g)
    return out


def lambda1h(p) -> float:
    """Smallest eigenvalue of -Delta_h on the interior nodes (sparse
    eigensolver); k^2 / lambda1h is the spectral radius of G."""
    L, ids, B = laplacian(p)
    A = (-L).tocsc()
    vals = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)
    return float(vals[0])


def torsion(p) -> np.ndarray:
    """FD solution of Delta E = -1 with E = 0 on edge and hole nodes."""
    L, ids, B = laplacian(p)
    sol = spla.spsolve(L.tocsc(), -np.ones(len(ids)))
    out = np.zeros((p.ny, p.nx))
    out.ravel()[ids] = sol
    return out
