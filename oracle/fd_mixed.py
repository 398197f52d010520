"""Finite differences for the annular problems: an absorbing (Dirichlet) hole
inside a rectangle whose edge carries a Neumann or Robin condition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Two discretisations of the edge condition d_n u = g:

* ``ghost`` (second order): an edge node takes the 5-point Laplacian with the
  ghost value across the face set by the central difference,
  u_ghost = u_inner + 2 dx g; on a corner both faces do so.
* ``one_sided`` (the matrix A of Sec. 2.4): an edge node's row is the
  one-sided normal difference (u_edge - u_inner) / dx = g; a corner's row is
  the mean of its two faces' differences (a reading: the paper does not say
  how corners are treated).

Interior nodes take the 5-point Laplacian.  A neighbour in the hole is a
Dirichlet value: at the hole's boundary point on the grid line, with the
Shortley-Weller weights when that point falls short of the neighbour node
(the disc; a box whose edges lie between grid lines), else at the node.

Functions: ``exit_time`` (Delta E = -1, E = 0 on the hole, d_n E = 0: the
mean exit time of the reflected diffusion, Sec. 2.3), ``local_time``
(Delta L = 0, L = 0 on the hole, d_n L = 1: the mean local time on the edge,
the remark after Theorem 2.3), ``direct`` (Delta u + (k^2 + i p) u = f with
d_n u - i k u = g2), ``iterate`` (the partial sums U_n of the annular
iteration of Sec. 2.3), ``spectral_radius_G`` (the iteration matrix of
Sec. 2.4 with alpha = k^2).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fd, fkmc

# outward normals of the faces 0..3 (x = x0, x = x1, y = y0, y = y1)
_NORMALS = ((-1.0, 0.0), (1.0, 0.0), (0.0, -1.0), (0.0, 1.0))


def _steps(p):
    return (p.x1 - p.x0) / (p.nx - 1), (p.y1 - p.y0) / (p.ny - 1)


def _node_xy(p, i, j):
    dx, dy = _steps(p)
    return p.x0 + i * dx, p.y0 + j * dy


def _hole_distance(p, x, y, ex, ey, step):
    """Distance t in (0, step] from (x, y) along the unit direction (ex, ey)
    to the hole's boundary, given that the point at distance step is in the
    hole."""
    if p.domain_kind == "rect_minus_disc":
        # |(x, y) + t e - c| = r, the smaller root
        fx, fy = x - p.cx, y - p.cy
        b = fx * ex + fy * ey
        c = fx * fx + fy * fy - p.r * p.r
        disc = b * b - c
        t = -b - math.sqrt(max(disc, 0.0))
        return min(max(t, 1e-12 * step), step)
    bx0, bx1, by0, by1 = p.cx - p.r, p.cx + p.r, p.cy - p.ry, p.cy + p.ry
    if ex > 0:
        t = bx0 - x
    elif ex < 0:
        t = x - bx1
    elif ey > 0:
        t = by0 - y
    else:
        t = y - by1
    if t >= step * (1.0 - 1e-9):
        return step
    return min(max(t, 1e-12 * step), step)


def _faces(p, i, j):
    """Faces of the rectangle that node (i, j) lies on."""
    out = []
    if i == 0:
        out.append(0)
    if i == p.nx - 1:
        out.append(1)
    if j == 0:
        out.append(2)
    if j == p.ny - 1:
        out.append(3)
    return out


def system(p, scheme="ghost", phi=None):
    """Assembles the discrete operator over the unknown nodes (every node not
    in the hole) for a problem with a reflecting edge.

    Returns (A, ids, D, EF): A the operator (sparse), ids the unknown node
    ids (grid order), D the Dirichlet right-hand-side contribution (A u + D =
    the discrete Laplacian / edge operator applied to the full field), and EF
    (rows x 4) the weight with which the datum g_f of face f (= d_n u there)
    enters each row: the discrete row reads
    (A u)_r + D_r + sum_f EF_{r,f} g_{r,f} = rhs_r.

    ghost:     interior rows Delta_h u = f; edge rows Delta_h^ghost u + ... = f
               with EF = 2/dx on an x face, 2/dy on a y face;
    one_sided: interior rows as above; edge rows: the mean over the node's
               faces of (u_edge - u_inner)/step - g_f equals 0, i.e.
               EF = -1/(number of faces) and the right-hand side is 0.
    phi(x, y): the Dirichlet datum on the hole (complex), default 0.
    """
    assert p.reflect
    cls = fkmc.node_classes(p).ravel()
    ids = np.nonzero(cls == 0)[0]
    pos = -np.ones(p.nx * p.ny, dtype=np.int64)
    pos[ids] = np.arange(len(ids))
    dx, dy = _steps(p)
    n = len(ids)
    rows, cols, vals = [], [], []
    D = np.zeros(n, dtype=complex)
    EF = np.zeros((n, 4))
    for r, g in enumerate(ids):
        i, j = int(g % p.nx), int(g // p.nx)
        x, y = _node_xy(p, i, j)
        faces = _faces(p, i, j)
        if faces and scheme == "one_sided":
            # mean of the one-sided normal differences of the node's faces
            w = 1.0 / len(faces)
            for f in faces:
                st = dx if f < 2 else dy
                ii, jj = (i + 1, j) if f == 0 else (i - 1, j) if f == 1 else (i, j + 1) if f == 2 else (i, j - 1)
                rows += [r, r]
                cols += [r, pos[ii + p.nx * jj]]
                vals += [w / st, -w / st]
                EF[r, f] = -w
            continue
        diag = 0.0
        for axis, st in ((0, dx), (1, dy)):
            lo = (i - 1, j) if axis == 0 else (i, j - 1)
            hi = (i + 1, j) if axis == 0 else (i, j + 1)
            nodes = [lo, hi]
            # ghost: a node on a face mirrors its inner neighbour
            if axis == 0 and i == 0:
                nodes[0] = hi
            if axis == 0 and i == p.nx - 1:
                nodes[1] = lo
            if axis == 1 and j == 0:
                nodes[0] = hi
            if axis == 1 and j == p.ny - 1:
                nodes[1] = lo
            for f in faces:
                if (f < 2) == (axis == 0):
                    EF[r, f] = 2.0 / st
            # arm lengths and Dirichlet values (Shortley-Weller)
            arms = []
            for side, (ii, jj) in enumerate(nodes):
                nb = ii + p.nx * jj
                if pos[nb] >= 0:
                    arms.append((st, pos[nb], None))
                else:
                    sgn = -1.0 if side == 0 else 1.0
                    ex, ey = (sgn, 0.0) if axis == 0 else (0.0, sgn)
                    t = _hole_distance(p, x, y, ex, ey, st)
                    val = 0.0 if phi is None else phi(x + t * ex, y + t * ey)
                    arms.append((t, None, val))
            (h1, c1, v1), (h2, c2, v2) = arms
            w1 = 2.0 / (h1 * (h1 + h2))
            w2 = 2.0 / (h2 * (h1 + h2))
            diag -= 2.0 / (h1 * h2)
            for w, c, v in ((w1, c1, v1), (w2, c2, v2)):
                if c is not None:
                    rows.append(r)
                    cols.append(c)
                    vals.append(w)
                else:
                    D[r] += w * v
        rows.append(r)
        cols.append(r)
        vals.append(diag)
    A = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    return A, ids, D, EF


def _edge_mask(p, ids):
    i, j = ids % p.nx, ids // p.nx
    return (i == 0) | (i == p.nx - 1) | (j == 0) | (j == p.ny - 1)


def _full(p, ids, vals, phi=None):
    out = np.zeros((p.ny, p.nx), dtype=complex)
    if phi is not None:
        X, Y = fd._grid(p)
        out = np.asarray(phi(X, Y), dtype=complex) * np.ones((p.ny, p.nx))
    out.ravel()[ids] = vals
    return out


def exit_time(p, scheme="ghost"):
    """Mean exit time of the reflected diffusion: Delta E = -1, E = 0 on the
    hole, d_n E = 0 on the edge (Sec. 2.3; eq. (2.10) with a reflecting
    part).  Full real grid, 0 on hole nodes."""
    A, ids, D, EF = system(p, scheme)
    rhs = -np.ones(len(ids))
    if scheme == "one_sided":
        rhs[_edge_mask(p, ids)] = 0.0
    sol = spla.spsolve(A.tocsc(), rhs)
    return _full(p, ids, sol).real


def local_time(p, scheme="ghost"):
    """Mean local time on the edge: Delta L = 0, L = 0 on the hole,
    d_n L = 1 on the edge (the remark after Theorem 2.3)."""
    A, ids, D, EF = system(p, scheme)
    rhs = -EF.sum(axis=1)
    sol = spla.spsolve(A.tocsc(), rhs)
    return _full(p, ids, sol).real


def _phi_inner(p):
    """The inner (hole) Dirichlet datum as a numpy function."""
    bc = p.inner
    if bc.kind == "zero":
        return lambda X, Y: np.zeros(np.broadcast(X, Y).shape, dtype=complex)
    if bc.kind == "plane_wave":
        kappa = p.k if p.damping == 0.0 else complex(np.sqrt(complex(p.k * p.k, p.damping)))
        return lambda X, Y: complex(bc.amp) * np.exp(1j * kappa * (np.asarray(X) * math.cos(bc.theta)
                                                                  + np.asarray(Y) * math.sin(bc.theta)))
    raise ValueError(bc.kind)


def robin_datum(p, ids):
    """g2 per unknown node and face (rows x 4; 0 off the faces), from the
    outer datum: zero, or plane_wave_robin (the Robin datum
    i (kappa d.n - k) w of the plane wave w on each face)."""
    g = np.zeros((len(ids), 4), dtype=complex)
    bc = p.outer
    if bc.kind == "zero":
        return g
    if bc.kind != "plane_wave_robin":
        raise ValueError(bc.kind)
    kappa = p.k if p.damping == 0.0 else complex(np.sqrt(complex(p.k * p.k, p.damping)))
    d = (math.cos(bc.theta), math.sin(bc.theta))
    for r, nid in enumerate(ids):
        i, j = int(nid % p.nx), int(nid // p.nx)
        faces = _faces(p, i, j)
        if not faces:
            continue
        x, y = _node_xy(p, i, j)
        w = complex(bc.amp) * np.exp(1j * kappa * (x * d[0] + y * d[1]))
        for f in faces:
            dn = _NORMALS[f][0] * d[0] + _NORMALS[f][1] * d[1]
            g[r, f] = 1j * (kappa * dn - p.k) * w
    return g


def direct(p, scheme="ghost"):
    """Delta u + (k^2 + i p) u = f, u = phi on the hole, d_n u - i k u = g2 on
    the edge (ghost scheme: the edge datum d_n u = i k u + g2 enters the edge
    rows).  Full complex grid."""
    phi = _phi_inner(p)
    A, ids, D, EF = system(p, scheme, phi=lambda x, y: complex(phi(x, y)))
    f = fd.source_grid(p).ravel()[ids]
    E = EF.sum(axis=1)
    eg2 = (EF * robin_datum(p, ids)).sum(axis=1)
    edge = _edge_mask(p, ids)
    # rows: A u + D + E i k u + sum_f EF_f g2_f + (k^2 + i p) u = f   (ghost)
    #       A u + E i k u + sum_f EF_f g2_f = 0                        (one_sided, edge rows)
    M = A.astype(complex) + sp.diags(1j * p.k * E)
    rhs = f - D - eg2
    lam = complex(p.k ** 2, p.damping)
    if scheme == "one_sided":
        M = M + sp.diags(np.where(edge, 0.0, 1.0) * lam)
        rhs = np.where(edge, -eg2, rhs)
    else:
        M = M + lam * sp.identity(len(ids))
    sol = spla.spsolve(M.tocsc(), rhs)
    return _full(p, ids, sol, phi)


def iterate(p, n_iters, scheme="ghost"):
    """Partial sums U_1..U_n of the annular iteration (Sec. 2.3):
    Delta U_{n+1} - (alpha - k^2) U_{n+1} = f - (alpha + i p) U_n,
    U_{n+1} = phi on the hole, d_n U_{n+1} = i k U_n + g2 on the edge,
    U_0 = 0 (hole nodes carry phi from U_1 on).  Returns the list of full
    grids."""
    phi = _phi_inner(p)
    alpha = p.k ** 2 if p.alpha is None else p.alpha
    c = alpha - p.k ** 2
    A, ids, D, EF = system(p, scheme, phi=lambda x, y: complex(phi(x, y)))
    f = fd.source_grid(p).ravel()[ids]
    E = EF.sum(axis=1)
    eg2 = (EF * robin_datum(p, ids)).sum(axis=1)
    edge = _edge_mask(p, ids)
    if scheme == "one_sided":
        M = A - c * sp.diags(np.where(edge, 0.0, 1.0))
    else:
        M = A - c * sp.identity(len(ids))
    lu = spla.splu(M.tocsc())
    u = np.zeros(len(ids), dtype=complex)
    out = []
    for n in range(n_iters):
        eg = E * (1j * p.k * u) + eg2
        rhs = f - complex(alpha, p.damping) * u - D - eg
        if scheme == "one_sided":
            rhs = np.where(edge, -eg, rhs)
        u = lu.solve(rhs.real) + 1j * lu.solve(rhs.imag)
        out.append(_full(p, ids, u, phi))
    return out


def spectral_radius_G(p, k, scheme="one_sided"):
    """Spectral radius of the iteration matrix G = A^{-1} diag(-k^2 on PDE
    rows, +i k on edge rows) of Sec. 2.4 (alpha = k^2, zero data), dense."""
    A, ids, D, EF = system(p, scheme)
    E = EF.sum(axis=1)
    edge = _edge_mask(p, ids)
    if scheme == "one_sided":
        d = np.where(edge, 1j * k, -k * k)
        G = np.linalg.solve(A.toarray().astype(complex), np.diag(d))
    else:
        # ghost rows: A u + E (i k u_prev) = -k^2 u_prev
        G = np.linalg.solve(A.toarray().astype(complex), np.diag(-k * k - 1j * k * E))
    return float(np.max(np.abs(np.linalg.eigvals(G))))


def k_star_A(sup_tau, sup_xi):
    """k_*^A = (-E[xi] + sqrt(E[xi]^2 + 4 E[tau])) / (2 E[tau]) (the remark
    after Theorem 2.3), here from the suprema as in Table 1."""
    return (-sup_xi + math.sqrt(sup_xi ** 2 + 4.0 * sup_tau)) / (2.0 * sup_tau)
