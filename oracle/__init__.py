"""FP64 CPU oracle for the Monte Carlo Feynman-Kac fixed-point Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
runs anything in this directory: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` do.  The oracle shares no code with
the HIP library; both are written from the paper (Bernal, Chen, dos Reis, "An
iterative method for Helmholtz boundary value problems arising in wave
propagation") and meet only in the seeded problem descriptions that the tests
hand to each.

Contents
--------
``fkmc.c`` / ``fkmc.py``
    The estimator itself, step by step: Philox4x32-10 normals, Euler-Maruyama
    paths of ``y + sqrt(2) W``, first exit, boundary datum at the nearest
    boundary point, left-point integral of ``f - k^2 u_n`` and per-node mean and
    variance (Sec. 2.1 eq. (2.3); Sec. 2.2; Remark 2.1), plus the fixed-point
    loop with its stopping and divergence rules (Sec. 3).  With a reflecting
    edge (Sec. 2.3): mirrored steps, the local time on the edge and the Robin
    coupling d_n U_{n+1} = i k U_n + g2.
``fd.py``
    Five-point finite differences: the direct Helmholtz solve and the
    Neumann-series iterate ``u_{n+1} = Delta_h^{-1}(f - k^2 u_n)`` whose
    convergence is governed by the spectral radius of ``G`` (Sec. 2.4).
``fd_mixed.py``
    Finite differences with a reflecting (Neumann / Robin) edge around an
    absorbing hole: mean exit time and mean local time (Table 1), the direct
    Robin solve, the annular iteration and the spectral radius of its matrix
    (Sec. 2.4).
``closed_forms.py``
    Exact solutions that pin the above: plane waves, the sound-soft disc
    series, the exit-time (torsion) series of Remark 2.5 and ``lambda_1``.

Parity status of each function is listed in its docstring; everything that is
not pinned by a closed form, a library routine or brute force says
"parity unpinned".
"""
