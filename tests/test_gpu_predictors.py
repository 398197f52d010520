"""GPU: the convergence predictors on the same kernels.  With k = 0, f = -1,
g = 0 one Feynman-Kac step estimates the mean exit time E[tau] (Remark 2.5);
its maximum gives k_*^C = (max E[tau])^(-1/2) (Remark 2.4), which must lie
below k_max = sqrt(lambda_1) (Sec. 3: a sufficient bound)."""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import fkmc
from paper_2308_11469_amd import fkh, serving
from paper_2308_11469_amd import workloads as W

from gpu_util import require_lib

pytestmark = pytest.mark.gpu


def test_exit_time_map_matches_shifted_torsion_and_kstar():
    require_lib()
    p = serving.exit_time_problem(W.cavity_65(k=2.0).replace(nx=33, ny=33, h=5e-4), M=4096)
    s = fkh.Solver(p)
    s.iterate(1)
    E, se = s.get()
    s.close()
    d = cf.bgk_beta() * math.sqrt(2 * p.h)
    xs = np.arange(33) / 32
    X, Y = np.meshgrid(xs, xs)
    T = cf.torsion_rect(1 + 2 * d, 1 + 2 * d, X + d, Y + d)
    ids = fkmc.interior_ids(p)
    err = np.abs(E.ravel()[ids].real - T.ravel()[ids])
    assert np.all(err <= 4.5 * np.abs(se.ravel()[ids]) + 0.015 * T.ravel()[ids])
    assert np.all(np.abs(E.imag) == 0)
    ks = serving.kstar_cavity(E.real)
    assert 3.3 < ks < math.pi * math.sqrt(2)
    # and it agrees with the oracle's estimate of the same quantity
    orc = fkmc.fk_nodes(p, None, 0, ids[::37])
    assert np.allclose(E.ravel()[ids[::37]].real, orc["mean"].real, rtol=1e-12, atol=1e-15)


def test_disc_domain_rho_prediction_brackets_divergence():
    require_lib()
    base = W.scatter_problem(k=3.0, theta=0.3, N=33, M=256, seed=3, precision=32, h=1e-3, table_len=2048)
    rho_ok = serving.predicted_rho(base)
    rho_bad = serving.predicted_rho(base.replace(k=4.0))
    assert rho_ok < 0.8 and rho_bad > 1.05
    s = fkh.Solver(base.replace(k=4.0, crn=True, max_iters=40))
    rep = s.solve()
    s.close()
    assert rep["status"] == "FK_EDIVERGED"
