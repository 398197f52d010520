"""The C ABI library loads, exports every symbol that include/fk_helmholtz.h
declares, and rejects invalid problems on the host (no GPU needed: argument
validation runs before any device call)."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2308_11469_amd import build, fkh
from paper_2308_11469_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "fk_helmholtz.h")).read()
    return re.findall(r"^(?:fk_status|const char \*)\s*(\w+)\s*\(", txt, flags=re.M)


@pytest.fixture(scope="module")
def lib():
    if not build.is_built():
        build.build()
    return fkh.lib()


def test_header_and_binding_agree():
    assert sorted(header_functions()) == sorted(fkh.EXPORTS)


def test_every_declared_symbol_is_exported(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def arena_status(p):
    m = fkh.Marshalled(p)
    n = C.c_size_t()
    st = fkh.lib().fk_helmholtz_arena_bytes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params), C.byref(n))
    return st, n.value


@pytest.mark.parametrize("bad", [
    dict(nx=2), dict(ny=0), dict(x1=0.0), dict(h=0.0), dict(h=-1e-3), dict(M=1), dict(precision=16),
    dict(k=float("nan")), dict(k=-1.0), dict(paths_per_item=100),
])
def test_invalid_parameters_rejected(lib, bad):
    p = W.cavity_small()
    ppi = bad.pop("paths_per_item", 0)
    p = p.replace(**bad)
    m = fkh.Marshalled(p, ppi)
    n = C.c_size_t()
    st = lib.fk_helmholtz_arena_bytes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params), C.byref(n))
    assert st == fkh.FK_EINVAL
    assert lib.fk_helmholtz_last_error().decode()


def test_disc_must_be_inside(lib):
    p = W.scatter_problem(k=2.0, theta=0.0, N=33, M=64, seed=1, table_len=64).replace(r=1.5)
    assert arena_status(p)[0] == fkh.FK_EINVAL
    p = W.scatter_problem(k=2.0, theta=0.0, N=33, M=64, seed=1, table_len=64)
    st, nbytes = arena_status(p)
    assert st == fkh.FK_OK and nbytes > 33 * 33 * 16


def test_table_only_outside(lib):
    p = W.scatter_problem(k=2.0, theta=0.0, N=33, M=64, seed=1, table_len=64)
    p.inner = p.outer
    m = fkh.Marshalled(p)
    h = C.c_void_p()
    st = lib.fk_helmholtz_create(*m.args(), None, 0, None, C.byref(h))
    assert st == fkh.FK_EINVAL and not h.value


def test_arena_size_grows_with_grid_and_paths(lib):
    a = arena_status(W.cavity_small())[1]
    b = arena_status(W.cavity_65())[1]
    c = arena_status(W.cavity_source())[1]
    assert a < b < c


def test_work_items_guided_and_uniform(lib):
    # automatic item size: large items (a whole number of small ones, at most
    # three quarters of M) ahead of small ones, as long as 3 x 4096 large
    # items result; a fixed item size is uniform; small problems stay uniform
    def check(p, wi):
        a, b = wi["items_large"] * wi["paths_large"], wi["paths_small"]
        assert a <= 3 * p.M // 4 and (a == 0 or a % b == 0)
        assert a + (wi["items_small"] - 1) * b < p.M <= a + wi["items_small"] * b
    c3 = W.cavity_source(precision=64)
    wi = fkh.work_items(c3)
    assert (wi["paths_large"], wi["items_large"], wi["paths_small"], wi["items_small"]) == (12288, 1, 1024, 4)
    assert wi["n_items"] == 127 * 127 * 5
    check(c3, wi)
    c2 = W.cavity_65(precision=64)
    wi = fkh.work_items(c2)
    assert (wi["paths_large"], wi["items_large"], wi["paths_small"], wi["items_small"]) == (768, 4, 256, 4)
    check(c2, wi)
    for p in (W.rect_batch(256)[:24] + [W.annulus_shape3(k=0.5, nx=101, ny=161, M=4096, h=1e-4, precision=32)]):
        wi = fkh.work_items(p)
        check(p, wi)
        assert wi["items_large"] * (wi["n_items"] // (wi["items_large"] + wi["items_small"])) >= 3 * 4096 \
            or wi["items_large"] == 0
    # reflecting edge: uniform items
    assert fkh.work_items(W.annulus_shape3(k=0.5, nx=101, ny=161, M=4096, h=1e-4, precision=32))["items_large"] == 0
    wi = fkh.work_items(c3, paths_per_item=256)
    assert (wi["paths_large"], wi["items_large"], wi["paths_small"], wi["items_small"]) == (0, 0, 256, 64)
    wi = fkh.work_items(W.cavity_small())
    assert wi["items_large"] == 0 and wi["n_items"] == 49 * wi["items_small"]


def test_gather_layout_sizes_and_validation(lib):
    # FP32: cell-major copy is 32 B per cell instead of 8 B per node; FP64:
    # 64 B per cell, or no copy at all (row-major paths read the FP64 master)
    def size(p, layout):
        m = fkh.Marshalled(p, 0, layout)
        n = C.c_size_t()
        st = lib.fk_helmholtz_arena_bytes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params), C.byref(n))
        return st, n.value
    p32 = W.cavity_65(precision=32)
    st_n, nodes = size(p32, "nodes")
    st_c, cells = size(p32, "cells")
    assert st_n == st_c == fkh.FK_OK
    grow = 64 * 64 * 32 - 65 * 65 * 8
    assert abs((cells - nodes) - grow) <= 256
    assert size(p32, "auto")[1] == nodes            # 33.8 KB row-major copy fits L1
    # a single FP32 instance up to 152 KiB of row-major copy (139 x 139
    # nodes) is staged in LDS (the solver's automatic layout keeps it
    # row-major); above, cell-major
    for n in (129, 139):
        mid = p32.replace(nx=n, ny=n)
        assert size(mid, "auto")[1] == size(mid, "nodes")[1] != size(mid, "cells")[1]
    over = p32.replace(nx=140, ny=140)
    assert size(over, "auto")[1] == size(over, "cells")[1] != size(over, "nodes")[1]
    big = p32.replace(nx=257, ny=257)
    assert size(big, "auto")[1] == size(big, "cells")[1] != size(big, "nodes")[1]
    p64 = W.cavity_65(precision=64)
    assert abs((size(p64, "cells")[1] - size(p64, "nodes")[1]) - 64 * 64 * 64) <= 256
    assert size(p64, "auto")[1] == size(p64, "nodes")[1]      # 67.6 KB master fits the threshold
    assert size(p32, "nodes")[1] - size(p64, "nodes")[1] < 65 * 65 * 8 + 256   # FP64 rows: no copy
    for bad in (-1, 3):
        assert size(p32, bad)[0] == fkh.FK_EINVAL


@pytest.mark.parametrize("waves", [-4, 2, 6, 36])
def test_waves_per_cu_validated(lib, waves):
    m = fkh.Marshalled(W.cavity_small(), 0, "auto", waves)
    n = C.c_size_t()
    assert lib.fk_helmholtz_arena_bytes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params),
                                        C.byref(n)) == fkh.FK_EINVAL
    m = fkh.Marshalled(W.cavity_small(), 0, "auto", 8)
    assert lib.fk_helmholtz_arena_bytes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params),
                                        C.byref(n)) == fkh.FK_OK


def test_step_cap_overflow_rejected(lib):
    p = W.cavity_small().replace(h=1e-12)
    assert arena_status(p)[0] == fkh.FK_EINVAL


def test_engine_config_validation(lib):
    cfg = fkh.fk_engine_config()
    cfg.max_instances = 0
    cfg.precision = 32
    cfg.max_grid_nodes = 100
    cfg.max_items = 100
    h = C.c_void_p()
    assert lib.fk_engine_create(C.byref(cfg), None, C.byref(h)) == fkh.FK_EINVAL
    cfg.max_instances = 4
    cfg.precision = 48
    assert lib.fk_engine_create(C.byref(cfg), None, C.byref(h)) == fkh.FK_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(fkh, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(fkh, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        fkh.lib()


@pytest.mark.parametrize("bad", ["no_hole", "no_step_cap", "unprojected", "robin_on_absorbing_edge",
                                 "robin_inner", "box_outside", "box_flat", "sides_vs_step"])
def test_reflecting_edge_and_box_validation(lib, bad):
    p = W.annulus_shape3(nx=21, ny=33)
    if bad == "no_hole":
        p = p.replace(domain_kind="rect")
    elif bad == "no_step_cap":
        p = p.replace(jmax=0)
    elif bad == "unprojected":
        p = p.replace(g_unprojected=True)
    elif bad == "robin_on_absorbing_edge":
        p = p.replace(reflect=False, outer=W.BC("plane_wave_robin", 1.0, 0.3))
    elif bad == "robin_inner":
        p = p.replace(inner=W.BC("plane_wave_robin", 1.0, 0.3))
    elif bad == "box_outside":
        p = p.replace(ry=0.9)
    elif bad == "box_flat":
        p = p.replace(ry=0.0)
    elif bad == "sides_vs_step":
        # 6 sqrt(2 h) = 0.85 with h = 0.01: longer than the 0.8-wide side
        p = p.replace(h=0.01, x0=-0.4, x1=0.4)
    if bad == "robin_inner":
        # the inner datum is checked at create (validation precedes any device call)
        m = fkh.Marshalled(p)
        h = C.c_void_p()
        assert lib.fk_helmholtz_create(*m.args(), None, 0, None, C.byref(h)) == fkh.FK_EINVAL and not h.value
        return
    assert arena_status(p)[0] == fkh.FK_EINVAL, bad


def test_annulus_workloads_accepted(lib):
    for p in (W.annulus_shape1(), W.annulus_shape3(), W.annulus_fig2(),
              W.annulus_shape1().replace(outer=W.BC("plane_wave_robin", 1.0, 0.4),
                                         inner=W.BC("plane_wave", 1.0, 0.4), alpha=3.0, damping=0.5)):
        st, nbytes = arena_status(p)
        assert st == fkh.FK_OK, (p.name, fkh.lib().fk_helmholtz_last_error())


@pytest.mark.parametrize("bad", ["not_square", "absorbing", "hole_outside", "rhombus_flat", "small_disc"])
def test_disc_domain_validation(lib, bad):
    # the disc inscribed in a square box, reflecting; either precision, any
    # k, shift and damping
    p = W.annulus_shape2(n=21)
    assert arena_status(p)[0] == fkh.FK_OK
    assert arena_status(p.replace(precision=32))[0] == fkh.FK_OK
    assert arena_status(p.replace(domain_kind=W.DISC_MINUS_DISC, r=0.1))[0] == fkh.FK_OK
    assert arena_status(p.replace(k=1.12, alpha=2.0, damping=0.5,
                                  outer=W.BC("plane_wave_robin", 1.0, 0.4)))[0] == fkh.FK_OK
    if bad == "not_square":
        p = p.replace(y1=p.y1 + 0.1)
    elif bad == "absorbing":
        p = p.replace(reflect=False)
    elif bad == "hole_outside":
        p = p.replace(cx=0.0, cy=0.0)      # the printed centre of Table 1's shape 2
    elif bad == "rhombus_flat":
        p = p.replace(ry=0.0)
    elif bad == "small_disc":
        p = p.replace(h=0.01)
    assert arena_status(p)[0] == fkh.FK_EINVAL


@pytest.mark.parametrize("case", ["shape2_21", "shape2_46", "shape2_129", "shape2_33x41", "disc_hole_40",
                                  "thin_annulus_65", "rectangle"])
def test_exterior_nodes_are_the_oracles_nearest_unknown_nodes(lib, case):
    # the library's pairs (exterior node, the unknown node it reads) against
    # the oracle's own remap table, built by brute force over every unknown
    # node: bit-identical, ties included (the square grid of a disc centred in
    # its box has many equidistant candidates)
    from oracle import fkmc
    if case == "shape2_21":
        p = W.annulus_shape2(n=21)
    elif case == "shape2_46":
        p = W.annulus_shape2(n=46)
    elif case == "shape2_33x41":
        p = W.annulus_shape2(n=33).replace(ny=41)
    elif case == "shape2_129":
        p = W.annulus_shape2(n=129)
    elif case == "disc_hole_40":
        p = W.annulus_shape2(n=40).replace(domain_kind=W.DISC_MINUS_DISC, r=0.1)
    elif case == "thin_annulus_65":
        # the hole's rim a cell or two from the circle: both rims are frontier
        p = W.annulus_shape2(n=65).replace(domain_kind=W.DISC_MINUS_DISC, r=0.42)
    else:
        p = W.annulus_shape1(n=13)
    pairs = fkh.exterior_nodes(p)
    cls = fkmc.node_classes(p).ravel()
    ext = np.nonzero(cls == 3)[0]
    if case == "rectangle":
        assert len(pairs) == 0 and len(ext) == 0
        return
    assert np.array_equal(pairs[:, 0], ext)
    remap = fkmc.Handle(p)._remap
    assert np.array_equal(pairs[:, 1], remap[ext])
    assert np.all(cls[pairs[:, 1]] == 0)


def test_exterior_nodes_buffer_too_small(lib):
    p = W.annulus_shape2(n=21)
    m = fkh.Marshalled(p)
    n = C.c_int64()
    assert lib.fk_helmholtz_exterior_nodes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params), None, 0,
                                           C.byref(n)) == fkh.FK_OK and n.value > 0
    buf = (C.c_int32 * (2 * n.value))()
    assert lib.fk_helmholtz_exterior_nodes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params), buf,
                                           n.value - 1, C.byref(n)) == fkh.FK_EINVAL
    assert lib.fk_helmholtz_exterior_nodes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params), buf,
                                           n.value, None) == fkh.FK_EINVAL
