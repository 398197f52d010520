"""GPU: the disc domains (the annular problems of Sec. 2.5 whose outer
boundary is a disc; Table 1's shape 2 as read here: the disc of radius 0.45
at (0.8, 0.5) minus the rhombus of diagonals 0.15 at its centre).  The
radially mirrored paths, their local time and the datum at the move's foot
against the oracle (exit steps bit for bit, scores and node estimates to
1e-12 in FP64): the exit-time and local-time solves (k = 0) and the
annular iteration at k > 0, whose iterate is read beyond the circle through
each exterior node's nearest unknown node; FP32 stepping within 0.1 SE of
FP64; Table 1's row for shape 2 (sup E[tau], sup E[xi], k_*^A, the
converging and diverging k) from the GPU."""
import math

import numpy as np
import pytest

from oracle import fkmc
from paper_2308_11469_amd import fkh, serving
from paper_2308_11469_amd import workloads as W

import paper_values as PV
from gpu_util import assert_fp64_node_parity, interior_values, require_lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    require_lib()


def concentric(h=1e-4, M=64, n=21):
    return W.Problem(name="concentric", domain_kind=W.DISC_MINUS_DISC, x0=0.0, x1=1.0, y0=0.0, y1=1.0,
                     cx=0.5, cy=0.5, r=0.15, reflect=True, nx=n, ny=n, k=0.0, h=h, M=M, seed=41,
                     jmax=int(math.ceil(60.0 / h)), outer=W.BC("zero"), inner=W.BC("zero"))


def _cases():
    s2 = W.annulus_shape2(n=21, M=64, h=1e-4)
    exit2 = serving.exit_time_problem(s2, M=64)
    local2 = serving.local_time_problem(s2, M=64)
    # a Robin datum that varies along the circle, a bilinear datum on the
    # rhombus and a Gaussian source: the foot's coordinates, the rhombus
    # projection and the source kernel (feature bits 0, 1, 3 and the curved
    # edge)
    mixed = s2.replace(outer=W.BC("bilinear", coeffs=(0.5 + 0.2j, 1.0 - 0.5j, -0.7 + 0.1j, 0.3 + 0.3j)),
                       inner=W.BC("bilinear", coeffs=(0.3 + 0.1j, 1.0 - 0.5j, 0.4j, -0.2 + 0j)),
                       src_kind="gaussian", src_amp=0.3 + 0.2j,
                       src_cx=0.7, src_cy=0.6, src_sigma=0.1, seed=43)
    conc = serving.exit_time_problem(concentric(), M=64)
    # the annular iteration at k > 0: the plane wave's own data, and a
    # shifted, damped iteration with a source on the disc hole
    wave = s2.replace(k=1.0, outer=W.BC("plane_wave_robin", 1.0, 0.4), inner=W.BC("plane_wave", 1.0, 0.4),
                      seed=44)
    general = concentric(M=64).replace(k=0.9, alpha=2.0, damping=0.5, src_kind="gaussian",
                                       src_amp=0.3 - 0.2j, src_cx=0.3, src_cy=0.6, src_sigma=0.1,
                                       outer=W.BC("bilinear", coeffs=(0.2j, 0.5, -0.3 + 0.1j, 0.1)),
                                       inner=W.BC("plane_wave", 1.0 - 0.5j, 1.1), seed=45)
    return {"shape2_exit_time": exit2, "shape2_local_time": local2, "shape2_mixed_data": mixed,
            "concentric_exit_time": conc, "shape2_k1_plane_wave": wave, "concentric_general_k09": general}


def plane_wave_iterate(p, theta=0.4):
    """A k > 0 iterate for the paths to read: the plane wave at the unknown
    nodes, the inner datum on the hole's nodes (as the iteration carries it
    from n = 1 on; the oracle's own fill), 1e3 at the exterior ones (which
    the library replaces by their nearest unknown node's value, and which
    the oracle reads through its remap)."""
    X, Y = np.meshgrid(np.linspace(p.x0, p.x1, p.nx), np.linspace(p.y0, p.y1, p.ny))
    u = np.exp(1j * p.k * (X * math.cos(theta) + Y * math.sin(theta)))
    cls = fkmc.node_classes(p).ravel()
    u.ravel()[cls == 2] = fkmc.boundary_grid(p).ravel()[cls == 2]
    u.ravel()[cls == 3] = 1e3
    return u


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_disc_paths_bit_exact_exit_steps(name):
    p = _cases()[name]
    say("disc paths", name)
    s = fkh.Solver(p)
    ids = fkmc.interior_ids(p)
    rng = np.random.default_rng(17)
    # the nodes nearest the circle (their paths mirror at once) and a sample
    X = p.x0 + (ids % p.nx) * ((p.x1 - p.x0) / (p.nx - 1))
    Y = p.y0 + (ids // p.nx) * ((p.y1 - p.y0) / (p.ny - 1))
    rad = np.hypot(X - 0.5 * (p.x0 + p.x1), Y - 0.5 * (p.y0 + p.y1))
    nodes = list(ids[np.argsort(-rad)[:8]]) + list(rng.choice(ids, size=16, replace=False))
    pairs = [(int(n), int(m)) for n in nodes for m in rng.integers(0, p.M, 6)]
    u, it = None, 0
    if p.k > 0:
        # the paths of iteration 2 read a given iterate
        u, it = plane_wave_iterate(p), 2
        s.set_iterate(u, it)
    J, sc, xj = s.debug_paths([a for a, _ in pairs], [b for _, b in pairs])
    for c, (n, m) in enumerate(pairs):
        so, Jo, capo, xo = fkmc.path(p, u, it, n, m)
        assert J[c] == Jo, (name, n, m, J[c], Jo)
        assert abs(sc[c] - so) <= 1e-12 * max(1.0, abs(so)), (name, n, m, sc[c], so)
        assert abs(xj[c][0] - xo[0]) < 1e-12 and abs(xj[c][1] - xo[1]) < 1e-12
    s.close()


@pytest.mark.parametrize("name", list(_cases().keys()))
def test_disc_node_estimates_fp64(name):
    p = _cases()[name].replace(M=160)
    say("disc nodes fp64", name)
    s = fkh.Solver(p)
    ids = fkmc.interior_ids(p)
    u = None
    for it in range(2):
        s.iterate(1)
        g, se = s.get()
        sj, cp = s.node_stats()
        orc = fkmc.fk_nodes(p, u, it)
        assert_fp64_node_parity(interior_values(p, g), sj[ids], orc, p.M, label="%s it %d" % (name, it))
        assert cp.sum() == 0
        # exterior nodes carry their nearest unknown node's new value (the
        # oracle's own remap table), and no standard error
        cls = fkmc.node_classes(p).ravel()
        ext = np.nonzero(cls == 3)[0]
        remap = fkmc.Handle(p)._remap
        assert len(ext) > 0 and np.array_equal(g.ravel()[ext], g.ravel()[remap[ext]])
        assert np.all(se.ravel()[ext] == 0)
        u = g
    s.close()


def test_disc_domain_rejected_by_the_engine():
    # the disc kernels mirror every path radially (they serve disc domains
    # alone) and an engine launch mixes instances, so the engine takes no
    # disc domain
    e = fkh.Engine(4, precision=64, max_grid_nodes=1 << 14, max_items=1 << 16, max_table=16,
                   max_instance_nodes=1024)
    with pytest.raises(ValueError):
        e.add(_cases()["shape2_mixed_data"])
    assert e.add(W.cavity_small().replace(M=96)) is not None
    e.close()


def test_table1_shape2_suprema_and_kstar_from_gpu():
    # the suprema lie on the circle (farthest from the hole); the nodes next
    # to it are within O(dx^2) of them (zero normal derivative there).  The
    # once-per-step exit test biases E by O(sqrt h): E_0 ~ 2 E(h/4) - E(h)
    est = {}
    for which in ("exit_time", "local_time"):
        vals = []
        for h in (4e-5, 1e-5):
            p = W.annulus_shape2(n=21, h=h)
            mk = serving.exit_time_problem if which == "exit_time" else serving.local_time_problem
            q = mk(p, M=1 << 17)
            s = fkh.Solver(q)
            s.iterate(1)
            u = s.get()[0].real
            s.close()
            ids = fkmc.interior_ids(q)
            vals.append(float(np.max(u.ravel()[ids])))
        est[which] = 2.0 * vals[1] - vals[0]
        say("shape2", which, "E(4e-5) %.5f E(1e-5) %.5f -> %.5f" % (vals[0], vals[1], est[which]))
    ks = float(serving.khat_annulus(est["exit_time"], est["local_time"]))
    t = PV.table1()[2]
    say("shape2 k_*^A %.4f (Table 1: %s %s %s)" % (ks, t["sup_tau"], t["sup_xi"], t["kstar_A"]))
    # sup E[tau] to the printed two digits
    assert round(est["exit_time"], 2) == t["sup_tau"]
    # For a centred hole both suprema sit on the circle, and the hole acts
    # nearly as a disc of some radius a: E[tau](R) = R^2/2 ln(R/a) -
    # (R^2 - a^2)/4 and E[xi](R) = R ln(R/a).  The a that gives sup E[tau]
    # = 0.15 gives sup E[xi] = 0.89, not the printed 0.91 (the printed
    # geometry is garbled: its hole lies outside the disc).  The GPU's pair
    # follows that relation; against the printed sup E[xi] and k_*^A it is
    # within 3%.
    R = 0.45
    a = 0.06
    for _ in range(60):   # fixed point of the E[tau] relation for a
        a = R * math.exp(-(est["exit_time"] + (R * R - a * a) / 4.0) / (R * R / 2.0))
    assert abs(est["local_time"] - R * math.log(R / a)) <= 0.01 * est["local_time"]
    assert abs(est["local_time"] - t["sup_xi"]) <= 0.03 * t["sup_xi"]
    assert abs(ks - t["kstar_A"]) <= 0.03 * t["kstar_A"]


def test_table1_shape2_convergence_outcomes():
    # Table 1's column for shape 2: the annular iteration (30 iterates of
    # fresh paths, the paper's inner datum -exp(-i k x) and g2 = 0) converges
    # at k = 0.70, 0.95, 0.96 and diverges at 1.12.  With common random
    # numbers the iteration is one fixed linear map, and the change shrinks
    # or grows by its spectral radius per iterate: below one at 0.96, above
    # at 1.12.
    t = PV.table1()[2]
    for k, converges in t["tested"]:
        p = W.annulus_shape2(k=k, n=46, M=4096, h=1e-4, seed=57)
        s = fkh.Solver(p)
        rows = [s.iterate(1) for _ in range(30)]
        s.close()
        du = [r["max_du"] for r in rows]
        sup = [r["sup"] for r in rows]
        say("shape2 k=%.2f sup at 10/20/30 %.3f %.3f %.3f, max change %.3g %.3g %.3g"
            % (k, sup[9], sup[19], sup[29], du[9], du[19], du[29]))
        if converges:
            assert sup[29] < 1.2 and du[29] < du[9]
        else:
            assert du[29] > du[19] > du[9] and sup[29] > 2.0 * sup[9]
    for k, above in ((0.96, False), (1.12, True)):
        s = fkh.Solver(W.annulus_shape2(k=k, n=46, M=4096, h=1e-4, seed=57).replace(crn=True))
        du = [s.iterate(1)["max_du"] for _ in range(30)]
        s.close()
        rate = (du[29] / du[19]) ** 0.1
        say("shape2 k=%.2f CRN change ratio per iterate %.4f" % (k, rate))
        assert (rate > 1.0) == above


def test_disc_checkpoint_resume_bit_identity():
    # resuming from a saved iterate (the host extends it to the exterior
    # nodes) continues exactly as the uninterrupted run (where the device
    # extends it after each update)
    p = _cases()["shape2_k1_plane_wave"].replace(M=128)
    s = fkh.Solver(p)
    s.iterate(2)
    saved, _ = s.get()
    s.iterate(2)
    ref, ref_se = s.get()
    s.close()
    r = fkh.Solver(p)
    r.set_iterate(saved, 2)
    r.iterate(2)
    got, got_se = r.get()
    r.close()
    say("disc checkpoint/resume")
    assert np.array_equal(got, ref) and np.array_equal(got_se, ref_se)


@pytest.mark.parametrize("name", ["shape2_k1_plane_wave", "concentric_general_k09", "shape2_mixed_data"])
def test_disc_fp32_within_tenth_se_of_fp64(name):
    # FP32 stepping on the disc domain (compensated position, the test and
    # the radial mirror at the circle formed in FP64) against FP64 on the
    # same streams and the same u_n: every unknown node within 0.1 SE
    p = _cases()[name].replace(M=1024)
    s64 = fkh.Solver(p)
    s32 = fkh.Solver(p.replace(precision=32))
    s64.iterate(1)
    s32.iterate(1)
    g64, _ = s64.get()
    s64.iterate(1)
    s32.set_iterate(g64, 1)
    s32.iterate(1)
    g64b, se64b = s64.get()
    g32b, _ = s32.get()
    s64.close()
    s32.close()
    d = np.abs(interior_values(p, g32b) - interior_values(p, g64b))
    se = np.abs(interior_values(p, se64b))
    say("disc fp32", name, "max %.4f SE" % (d / se).max())
    assert np.all(d <= 0.1 * se)
    # the exterior nodes carry their pairs' FP32-path values as well
    cls = fkmc.node_classes(p).ravel()
    ext = np.nonzero(cls == 3)[0]
    remap = fkmc.Handle(p)._remap
    assert np.array_equal(g32b.ravel()[ext], g32b.ravel()[remap[ext]])


def test_disc_fp32_bench_configuration_within_tenth_se():
    # the disc bench line's configuration (shape 2, 91 x 91, k = 0.5,
    # M = 4096, h = 1e-4): FP32 against FP64 from the same u_1
    p = W.annulus_shape2(k=0.5, n=91, M=4096, h=1e-4)
    s64 = fkh.Solver(p)
    s64.iterate(1)
    u1, _ = s64.get()
    s64.iterate(1)
    g64, se64 = s64.get()
    s64.close()
    s32 = fkh.Solver(p.replace(precision=32))
    s32.set_iterate(u1, 1)
    s32.iterate(1)
    g32, _ = s32.get()
    s32.close()
    r = np.abs(interior_values(p, g32) - interior_values(p, g64)) / np.abs(interior_values(p, se64))
    say("disc shape 2 91x91 FP32 vs FP64: max %.4f SE, rms %.4f SE over %d nodes"
        % (r.max(), np.sqrt(np.mean(r ** 2)), r.size))
    assert r.max() <= 0.1
