"""Probabilistic domain decomposition of one Poisson step of the iteration.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The two-stage procedure of Sec. 3 (and the case for PDD in Sec. 1): first
the Poisson iterate is computed by Feynman-Kac only at the nodes on the
subdomain interfaces; then every subdomain, with those values (and the
boundary data) as Dirichlet condition, is solved on its own by finite
differences.

Reading taken: the interfaces are whole grid lines (x index in ``cuts_x``,
y index in ``cuts_y``), so the interface nodes are exactly the nodes the
subdomains' 5-point stencils reach across, and no interpolation between
interface values is needed.  The subdomains are the blocks of unknown nodes
between consecutive lines (or the rectangle's edge); each solves
(Delta_h - (alpha - k^2)) U_{n+1} = f - (alpha + i p) U_n with the same
5-point operator as ``fd.py``, here by sparse LU of the block's own matrix.

With a hole (the scattering problem's disc, or a box) a block that has a
hole node in it or on its frame holds part of the hole's boundary: it is
not the rectangle's Dirichlet problem any more.  Reading taken for those
blocks: their unknown nodes keep the Feynman-Kac estimator (they join the
interface in the first stage), and only the blocks clear of the hole are
solved in the second.  An absorbing edge only (a reflecting edge has no
Dirichlet frame).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fd, fkmc


def check(p, cuts_x, cuts_y):
    if getattr(p, "reflect", False):
        raise ValueError("PDD here needs an absorbing edge")
    for cuts, n in ((cuts_x, p.nx), (cuts_y, p.ny)):
        c = list(cuts)
        if any(not (1 <= v <= n - 2) for v in c) or any(b <= a for a, b in zip(c, c[1:])):
            raise ValueError("cuts must increase strictly within [1, n - 2]")
    if not len(cuts_x) and not len(cuts_y):
        raise ValueError("at least one cut")


def interface_ids(p, cuts_x, cuts_y) -> np.ndarray:
    """Unknown nodes on the cut lines, in grid order."""
    check(p, cuts_x, cuts_y)
    ids = fkmc.interior_ids(p)
    i, j = ids % p.nx, ids // p.nx
    on = np.isin(i, np.asarray(cuts_x, dtype=np.int64)) | np.isin(j, np.asarray(cuts_y, dtype=np.int64))
    return ids[on].astype(np.int32)


def all_blocks(p, cuts_x, cuts_y):
    """Every block between consecutive cut lines (or the edge), as index
    ranges [i0, i1) x [j0, j1)."""
    xs = [0] + list(cuts_x) + [p.nx - 1]
    ys = [0] + list(cuts_y) + [p.ny - 1]
    out = []
    for b in range(len(ys) - 1):
        for a in range(len(xs) - 1):
            i0, i1, j0, j1 = xs[a] + 1, xs[a + 1], ys[b] + 1, ys[b + 1]
            if i1 > i0 and j1 > j0:
                out.append((i0, i1, j0, j1))
    return out


def clear_of_hole(p, block) -> bool:
    """No node of the block or of its frame lies in the hole."""
    i0, i1, j0, j1 = block
    return not np.any(fkmc.node_classes(p)[j0 - 1:j1 + 1, i0 - 1:i1 + 1] == 2)


def blocks(p, cuts_x, cuts_y):
    """The subdomains solved by finite differences: the blocks clear of the
    hole (every block on a plain rectangle)."""
    return [b for b in all_blocks(p, cuts_x, cuts_y) if clear_of_hole(p, b)]


def mc_ids(p, cuts_x, cuts_y) -> np.ndarray:
    """The nodes of the Feynman-Kac stage: the interface, and the unknown
    nodes of the blocks that touch the hole; grid order."""
    ids = set(interface_ids(p, cuts_x, cuts_y).tolist())
    cls = fkmc.node_classes(p)
    for blk in all_blocks(p, cuts_x, cuts_y):
        if not clear_of_hole(p, blk):
            i0, i1, j0, j1 = blk
            for j in range(j0, j1):
                for i in range(i0, i1):
                    if cls[j, i] == 0:
                        ids.add(j * p.nx + i)
    return np.array(sorted(ids), dtype=np.int32)


def block_solve(p, u_prev, u_frame, block):
    """One block of the Poisson step: the 5-point system on the block's nodes
    with Dirichlet values from ``u_frame`` (the new iterate on the interface
    lines, g on the edge) and right-hand side f - (alpha + i p) u_prev.
    Returns the block's values, shape (j1 - j0, i1 - i0)."""
    i0, i1, j0, j1 = block
    mx, my = i1 - i0, j1 - j0
    dx = (p.x1 - p.x0) / (p.nx - 1)
    dy = (p.y1 - p.y0) / (p.ny - 1)
    alpha = p.k ** 2 if p.alpha is None else p.alpha
    c = alpha - p.k ** 2
    n = mx * my
    rows, cols, vals = [], [], []
    rhs = np.zeros(n, dtype=complex)
    f = fd.source_grid(p)
    for jj in range(my):
        for ii in range(mx):
            r = ii + mx * jj
            gi, gj = i0 + ii, j0 + jj
            rows.append(r); cols.append(r); vals.append(-2.0 / dx ** 2 - 2.0 / dy ** 2 - c)
            rhs[r] = f[gj, gi] - complex(alpha, p.damping) * (0.0 if u_prev is None else u_prev[gj, gi])
            for (di, dj, w) in ((-1, 0, 1 / dx ** 2), (1, 0, 1 / dx ** 2), (0, -1, 1 / dy ** 2), (0, 1, 1 / dy ** 2)):
                ni, nj = ii + di, jj + dj
                if 0 <= ni < mx and 0 <= nj < my:
                    rows.append(r); cols.append(ni + mx * nj); vals.append(w)
                else:
                    rhs[r] -= w * u_frame[gj + dj, gi + di]
    A = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    lu = spla.splu(A)
    sol = lu.solve(rhs.real) + 1j * lu.solve(rhs.imag)
    return sol.reshape(my, mx)


def fill_blocks(p, u_prev, u_frame, cuts_x, cuts_y):
    """The full new iterate: u_frame (interface and edge values) with every
    block solved from it."""
    out = np.array(u_frame, dtype=complex)
    for blk in blocks(p, cuts_x, cuts_y):
        i0, i1, j0, j1 = blk
        out[j0:j1, i0:i1] = block_solve(p, u_prev, u_frame, blk)
    return out


def pdd_step(p, u_prev, n, cuts_x, cuts_y, nthreads=0):
    """U_{n+1} by PDD from U_n (u_prev, full grid; None for U_0 = 0):
    Feynman-Kac at the interface nodes and at the nodes of blocks touching a
    hole (``fkmc.fk_nodes``), then the other blocks.  Returns (new full
    grid, the Feynman-Kac estimates)."""
    ids = mc_ids(p, cuts_x, cuts_y)
    est = fkmc.fk_nodes(p, u_prev, n, ids, nthreads)
    frame = fkmc.boundary_grid(p)
    frame.ravel()[ids] = est["mean"]
    return fill_blocks(p, u_prev, frame, cuts_x, cuts_y), est
