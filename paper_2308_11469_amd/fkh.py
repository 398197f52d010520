"""Python binding of ``libfk_helmholtz.so`` (argument marshalling only).

Every step of the path runs in the library's HIP kernels; this module only
converts problem descriptions to the C structs of ``include/fk_helmholtz.h``,
hands over device memory and the stream (both from PyTorch) and copies
results back.  It raises if the library is not built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfk_helmholtz.so")

FK_OK, FK_EINVAL, FK_ENOMEM, FK_EDEVICE, FK_EDIVERGED, FK_ENOTCONVERGED, FK_EBUSY, FK_ECANCELLED = range(8)
STATUS_NAMES = {0: "FK_OK", 1: "FK_EINVAL", 2: "FK_ENOMEM", 3: "FK_EDEVICE", 4: "FK_EDIVERGED",
                5: "FK_ENOTCONVERGED", 6: "FK_EBUSY", 7: "FK_ECANCELLED"}

_DOMAIN = {"rect": 0, "rect_minus_disc": 1, "rect_minus_box": 2, "disc_minus_rhombus": 3, "disc_minus_disc": 4}
_SRC = {"zero": 0, "const": 1, "gaussian": 2}
_BC = {"zero": 0, "plane_wave": 1, "bilinear": 2, "table": 3, "plane_wave_robin": 4}
GATHER = {"auto": 0, "nodes": 1, "cells": 2}   # layout of the gathered copy of u_n (fk_gather_layout)


class FkError(RuntimeError):
    """A status other than FK_OK from the library (FK_EINVAL also raises
    ValueError subclasses: see FkInvalid)."""

    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class fk_domain(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("edge", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("r", C.c_double), ("ry", C.c_double)]


class fk_source(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("amp_re", C.c_double), ("amp_im", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("sigma", C.c_double)]


class fk_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("c", C.c_double * 8),
                ("table", C.POINTER(C.c_double)), ("table_len", C.c_int64)]


class fk_params(C.Structure):
    _fields_ = [("k", C.c_double), ("h", C.c_double), ("M", C.c_int64), ("seed", C.c_uint64),
                ("precision", C.c_int32), ("max_iters", C.c_int32), ("tol", C.c_double),
                ("max_steps", C.c_int64), ("crn", C.c_int32), ("g_unprojected", C.c_int32),
                ("paths_per_item", C.c_int32), ("gather_layout", C.c_int32),
                ("waves_per_cu", C.c_int32), ("reserved", C.c_int32),
                ("alpha", C.c_double), ("damping", C.c_double)]


class fk_iter_report(C.Structure):
    _fields_ = [("n", C.c_int32), ("diverging", C.c_int32), ("max_du", C.c_double), ("sup", C.c_double),
                ("max_se", C.c_double), ("noise_floor", C.c_double), ("path_steps", C.c_int64),
                ("capped", C.c_int64), ("nonfinite", C.c_int64), ("step_ms", C.c_double),
                ("noise_ratio", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class fk_engine_config(C.Structure):
    _fields_ = [("max_instances", C.c_int32), ("precision", C.c_int32), ("max_grid_nodes", C.c_int64),
                ("max_items", C.c_int64), ("max_table", C.c_int64), ("waves_per_cu", C.c_int32),
                ("max_instance_nodes", C.c_int32)]


# every entry point of include/fk_helmholtz.h
EXPORTS = ["fk_helmholtz_arena_bytes", "fk_helmholtz_work_items", "fk_helmholtz_exterior_nodes",
           "fk_helmholtz_create", "fk_helmholtz_iterate", "fk_helmholtz_solve",
           "fk_helmholtz_get", "fk_helmholtz_node_stats", "fk_helmholtz_set_iterate", "fk_helmholtz_set_pdd",
           "fk_helmholtz_cancel", "fk_engine_node_stats", "fk_engine_set_iterate", "fk_engine_set_pdd",
           "fk_helmholtz_timing", "fk_helmholtz_step_static",
           "fk_helmholtz_destroy", "fk_helmholtz_last_error", "fk_debug_philox", "fk_debug_normals",
           "fk_helmholtz_debug_paths", "fk_engine_create", "fk_engine_add", "fk_engine_tick", "fk_engine_get",
           "fk_engine_remove", "fk_engine_timing", "fk_engine_destroy"]

_lib = None


def lib():
    """Loads the in-tree HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfk_helmholtz.so is not built (run paper_2308_11469_amd/build.py); "
                               "there is no fallback path")
        # PyTorch first: its HIP runtime must be the one the library binds to
        # (device pointers and stream handles come from PyTorch); loading the
        # library first would bring in a second HIP runtime.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        i32p, i64p, u32p = C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.POINTER(C.c_uint32)
        P = C.POINTER
        sig = {
            "fk_helmholtz_arena_bytes": [P(fk_domain), P(fk_bc), P(fk_params), P(C.c_size_t)],
            "fk_helmholtz_work_items": [P(fk_domain), P(fk_bc), P(fk_params), i64p, i32p, i32p, i32p, i32p],
            "fk_helmholtz_exterior_nodes": [P(fk_domain), P(fk_bc), P(fk_params), i32p, C.c_int64, i64p],
            "fk_helmholtz_create": [P(fk_domain), P(fk_source), P(fk_bc), P(fk_bc), P(fk_params), vp, C.c_size_t,
                                    vp, P(vp)],
            "fk_helmholtz_iterate": [vp, C.c_int32, P(fk_iter_report)],
            "fk_helmholtz_solve": [vp, P(fk_iter_report)],
            "fk_helmholtz_get": [vp, vp, vp, C.c_int32],
            "fk_helmholtz_node_stats": [vp, i64p, i64p],
            "fk_helmholtz_set_iterate": [vp, vp, C.c_int32, C.c_int32],
            "fk_helmholtz_set_pdd": [vp, i32p, C.c_int32, i32p, C.c_int32],
            "fk_helmholtz_timing": [vp, dp, i64p, C.c_int32],
            "fk_helmholtz_step_static": [P(fk_domain), P(fk_source), P(fk_bc), P(fk_bc), P(fk_params), vp,
                                         C.c_int32, vp, vp, vp, P(fk_iter_report)],
            "fk_helmholtz_destroy": [vp],
            "fk_helmholtz_cancel": [vp],
            "fk_engine_node_stats": [vp, C.c_int32, i64p, i64p],
            "fk_engine_set_iterate": [vp, C.c_int32, vp, C.c_int32, C.c_int32],
            "fk_engine_set_pdd": [vp, C.c_int32, i32p, C.c_int32, i32p, C.c_int32],
            "fk_debug_philox": [C.c_uint64, u32p, C.c_int64, u32p],
            "fk_debug_normals": [C.c_int32, u32p, C.c_int64, dp],
            "fk_helmholtz_debug_paths": [vp, i32p, i64p, C.c_int64, i64p, dp, dp],
            "fk_engine_create": [P(fk_engine_config), vp, P(vp)],
            "fk_engine_add": [vp, P(fk_domain), P(fk_source), P(fk_bc), P(fk_bc), P(fk_params), i32p],
            "fk_engine_tick": [vp, P(fk_iter_report), P(C.c_uint8)],
            "fk_engine_get": [vp, C.c_int32, dp, dp],
            "fk_engine_remove": [vp, C.c_int32],
            "fk_engine_timing": [vp, dp, i64p, C.c_int32],
            "fk_engine_destroy": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.fk_helmholtz_last_error.argtypes = []
        L.fk_helmholtz_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class FkInvalid(FkError, ValueError):
    """FK_EINVAL: the problem description or an argument is invalid."""


def _check(st, allow=()):
    if st != FK_OK and st not in allow:
        cls = FkInvalid if st == FK_EINVAL else FkError
        raise cls(st, lib().fk_helmholtz_last_error().decode())
    return st


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------- marshalling

class Marshalled:
    """C structs for one problem description (keeps the table alive)."""

    def __init__(self, p, paths_per_item=0, gather_layout="auto", waves_per_cu=0):
        d = fk_domain()
        d.kind = _DOMAIN[p.domain_kind]
        d.nx, d.ny = int(p.nx), int(p.ny)
        d.x0, d.x1, d.y0, d.y1 = p.x0, p.x1, p.y0, p.y1
        d.cx, d.cy, d.r = p.cx, p.cy, p.r
        d.ry = float(getattr(p, "ry", 0.0))
        d.edge = 1 if getattr(p, "reflect", False) else 0
        f = fk_source()
        f.kind = _SRC[p.src_kind]
        a = complex(p.src_amp)
        f.amp_re, f.amp_im, f.cx, f.cy, f.sigma = a.real, a.imag, p.src_cx, p.src_cy, p.src_sigma
        self._keep = []
        bcs = []
        for bc in (p.outer, p.inner):
            b = fk_bc()
            b.kind = _BC[bc.kind]
            if bc.kind in ("plane_wave", "plane_wave_robin"):
                amp = complex(bc.amp)
                b.c[0], b.c[1], b.c[2] = amp.real, amp.imag, bc.theta
            elif bc.kind == "bilinear":
                for i, z in enumerate(bc.coeffs):
                    b.c[2 * i], b.c[2 * i + 1] = complex(z).real, complex(z).imag
            elif bc.kind == "table":
                t = np.ascontiguousarray(np.asarray(bc.table, dtype=np.complex128)).view(np.float64)
                self._keep.append(t)
                b.table = _dptr(t)
                b.table_len = len(t) // 2
            bcs.append(b)
        par = fk_params()
        par.k, par.h, par.M, par.seed = p.k, p.h, int(p.M), int(p.seed)
        par.precision = int(p.precision)
        par.max_iters = int(p.max_iters)
        par.tol = float(p.tol)
        par.max_steps = int(p.jmax)
        par.crn = 1 if p.crn else 0
        par.g_unprojected = 1 if getattr(p, "g_unprojected", False) else 0
        par.paths_per_item = int(paths_per_item)
        par.gather_layout = GATHER[gather_layout] if isinstance(gather_layout, str) else int(gather_layout)
        par.waves_per_cu = int(waves_per_cu)
        par.alpha = 0.0 if getattr(p, "alpha", None) is None else float(p.alpha)
        par.damping = float(getattr(p, "damping", 0.0))
        self.domain, self.source, self.outer, self.inner, self.params = d, f, bcs[0], bcs[1], par

    def args(self):
        return (C.byref(self.domain), C.byref(self.source), C.byref(self.outer), C.byref(self.inner),
                C.byref(self.params))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible to PyTorch")
    return torch


def current_stream_handle():
    return _torch().cuda.current_stream().cuda_stream


# ------------------------------------------------------------- solver

class Solver:
    """One Helmholtz instance on the GPU (the C ABI's fk_solver).  Device
    memory is a PyTorch uint8 tensor (the arena); work runs on PyTorch's
    current HIP stream unless ``stream`` is given."""

    def __init__(self, problem, paths_per_item=0, stream=None, gather_layout="auto", waves_per_cu=0):
        torch = _torch()
        self.problem = problem
        self.m = Marshalled(problem, paths_per_item, gather_layout, waves_per_cu)
        nbytes = C.c_size_t()
        _check(lib().fk_helmholtz_arena_bytes(C.byref(self.m.domain), C.byref(self.m.outer),
                                              C.byref(self.m.params), C.byref(nbytes)))
        self.arena_bytes = int(nbytes.value)
        raw = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device="cuda")
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.arena = raw[off:off + self.arena_bytes]
        self.stream = stream if stream is not None else current_stream_handle()
        h = C.c_void_p()
        _check(lib().fk_helmholtz_create(*self.m.args(), C.c_void_p(self.arena.data_ptr()),
                                         self.arena_bytes, C.c_void_p(self.stream), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().fk_helmholtz_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def iterate(self, n=1):
        """Runs n iterations; returns the last report (dict).  A fired
        divergence rule is reported as ``diverging`` (not raised); a cancelled
        call raises FkError with status FK_ECANCELLED."""
        r = fk_iter_report()
        _check(lib().fk_helmholtz_iterate(self.h, int(n), C.byref(r)), allow=(FK_EDIVERGED,))
        return r.as_dict()

    def solve(self):
        """Iterates to the stopping rule; the report carries ``status``
        (FK_OK, FK_ENOTCONVERGED, FK_EDIVERGED or FK_ECANCELLED)."""
        r = fk_iter_report()
        st = _check(lib().fk_helmholtz_solve(self.h, C.byref(r)),
                    allow=(FK_EDIVERGED, FK_ENOTCONVERGED, FK_ECANCELLED))
        d = r.as_dict()
        d["status"] = STATUS_NAMES[st]
        return d

    def cancel(self):
        """Stops the iterate / solve call running on this solver in another
        thread (or the next one) before its next iteration."""
        _check(lib().fk_helmholtz_cancel(self.h))

    def get(self):
        p = self.problem
        u = np.zeros((p.ny, p.nx), dtype=np.complex128)
        se = np.zeros((p.ny, p.nx), dtype=np.complex128)
        _check(lib().fk_helmholtz_get(self.h, u.ctypes.data_as(C.c_void_p), se.ctypes.data_as(C.c_void_p), 0))
        return u, se

    def get_device(self, out_u, out_se=None):
        """Copies the iterate (and SE) into device tensors (complex128 or
        float64 with 2 * nx * ny elements)."""
        _check(lib().fk_helmholtz_get(self.h, C.c_void_p(out_u.data_ptr()),
                                      C.c_void_p(out_se.data_ptr()) if out_se is not None else None, 1))

    def node_stats(self):
        p = self.problem
        sj = np.zeros(p.nx * p.ny, dtype=np.int64)
        cp = np.zeros(p.nx * p.ny, dtype=np.int64)
        _check(lib().fk_helmholtz_node_stats(self.h, sj.ctypes.data_as(C.POINTER(C.c_int64)),
                                             cp.ctypes.data_as(C.POINTER(C.c_int64))))
        return sj, cp

    def set_iterate(self, u, n):
        ub = np.ascontiguousarray(np.asarray(u, dtype=np.complex128))
        _check(lib().fk_helmholtz_set_iterate(self.h, ub.ctypes.data_as(C.c_void_p), int(n), 0))

    def set_pdd(self, cuts_x, cuts_y):
        """Probabilistic domain decomposition from the next iteration on:
        paths only from the nodes on the grid lines x index in cuts_x,
        y index in cuts_y; the blocks between them solved on the device."""
        cx = np.ascontiguousarray(np.asarray(cuts_x, dtype=np.int32))
        cy = np.ascontiguousarray(np.asarray(cuts_y, dtype=np.int32))
        i32p = C.POINTER(C.c_int32)
        _check(lib().fk_helmholtz_set_pdd(self.h, cx.ctypes.data_as(i32p), len(cx), cy.ctypes.data_as(i32p), len(cy)))

    def timing(self, reset=False):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().fk_helmholtz_timing(self.h, C.byref(ms), C.byref(n), 1 if reset else 0))
        return float(ms.value), int(n.value)

    def debug_paths(self, node_ids, ms):
        node_ids = np.ascontiguousarray(np.asarray(node_ids, dtype=np.int32))
        ms = np.ascontiguousarray(np.asarray(ms, dtype=np.int64))
        n = len(node_ids)
        J = np.zeros(n, dtype=np.int64)
        s = np.zeros(2 * n)
        x = np.zeros(2 * n)
        _check(lib().fk_helmholtz_debug_paths(self.h, node_ids.ctypes.data_as(C.POINTER(C.c_int32)),
                                              ms.ctypes.data_as(C.POINTER(C.c_int64)), n,
                                              J.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(s), _dptr(x)))
        return J, s[0::2] + 1j * s[1::2], x.reshape(-1, 2)


STATIC_SCRATCH_BYTES = 16 * 1024 * 1024   # FK_STATIC_SCRATCH_BYTES


def work_items(problem, paths_per_item=0, gather_layout="auto"):
    """The work items of a solver launch (fk_helmholtz_work_items): large
    items first, then small ones, per unknown node."""
    m = Marshalled(problem, paths_per_item, gather_layout)
    n = C.c_int64()
    pl, il, ps, is_ = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().fk_helmholtz_work_items(C.byref(m.domain), C.byref(m.outer), C.byref(m.params), C.byref(n),
                                         C.byref(pl), C.byref(il), C.byref(ps), C.byref(is_)))
    return dict(n_items=n.value, paths_large=pl.value, items_large=il.value, paths_small=ps.value,
                items_small=is_.value)


def exterior_nodes(problem):
    """Disc domains (fk_helmholtz_exterior_nodes): an (n, 2) int32 array of
    (exterior node, the unknown node whose value it carries)."""
    m = Marshalled(problem)
    n = C.c_int64()
    _check(lib().fk_helmholtz_exterior_nodes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params), None, 0,
                                             C.byref(n)))
    out = np.zeros((max(n.value, 1), 2), dtype=np.int32)
    _check(lib().fk_helmholtz_exterior_nodes(C.byref(m.domain), C.byref(m.outer), C.byref(m.params),
                                             out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, C.byref(n)))
    return out[:n.value]


def step_static(problem, u_n, n, u_next, se=None, stream=None, paths_per_item=0, gather_layout="auto"):
    """One fixed-point iteration without any device allocation in the library
    (fk_helmholtz_step_static): u_n and u_next (and se) are device tensors of
    nx * ny complex128 (or 2 nx ny float64) that the caller owns; u_n None
    means u_0 = 0.  Returns the report; a non-finite iterate is reported as
    ``diverging`` (not raised)."""
    m = Marshalled(problem, paths_per_item, gather_layout)
    r = fk_iter_report()
    st = lib().fk_helmholtz_step_static(
        *m.args(), C.c_void_p(u_n.data_ptr()) if u_n is not None else None, int(n),
        C.c_void_p(u_next.data_ptr()), C.c_void_p(se.data_ptr()) if se is not None else None,
        C.c_void_p(stream if stream is not None else current_stream_handle()), C.byref(r))
    _check(st, allow=(FK_EDIVERGED,))
    return r.as_dict()


def debug_philox(seed, ctrs):
    ctrs = np.ascontiguousarray(np.asarray(ctrs, dtype=np.uint32).reshape(-1, 4))
    out = np.zeros_like(ctrs)
    u32p = C.POINTER(C.c_uint32)
    _check(lib().fk_debug_philox(int(seed), ctrs.ctypes.data_as(u32p), ctrs.shape[0], out.ctypes.data_as(u32p)))
    return out


def debug_normals(precision, words):
    words = np.ascontiguousarray(np.asarray(words, dtype=np.uint32).reshape(-1, 2))
    z = np.zeros(2 * words.shape[0])
    _check(lib().fk_debug_normals(int(precision), words.ctypes.data_as(C.POINTER(C.c_uint32)), words.shape[0],
                                  _dptr(z)))
    return z.reshape(-1, 2)


# ------------------------------------------------------------- engine

class Engine:
    """Batched engine (the C ABI's fk_engine): instances are added into slots,
    every tick advances all of them by one iteration in one persistent launch."""

    def __init__(self, max_instances, precision=32, max_grid_nodes=1 << 22, max_items=1 << 22,
                 max_table=1 << 20, waves_per_cu=0, max_instance_nodes=0, stream=None):
        cfg = fk_engine_config()
        self.max_instances = int(max_instances)
        cfg.max_instances = int(max_instances)
        cfg.precision = int(precision)
        cfg.max_grid_nodes = int(max_grid_nodes)
        cfg.max_items = int(max_items)
        cfg.max_table = int(max_table)
        cfg.waves_per_cu = int(waves_per_cu)
        cfg.max_instance_nodes = int(max_instance_nodes)
        self.cfg = cfg
        self.stream = stream if stream is not None else current_stream_handle()
        h = C.c_void_p()
        _check(lib().fk_engine_create(C.byref(cfg), C.c_void_p(self.stream), C.byref(h)))
        self.h = h
        self.problems = {}
        self._marsh = {}

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().fk_engine_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, problem, paths_per_item=0, gather_layout="auto"):
        """Admits an instance; returns its slot, or None when no slot or no
        memory is free right now (FK_EBUSY / FK_ENOMEM)."""
        m = Marshalled(problem, paths_per_item, gather_layout)
        slot = C.c_int32(-1)
        st = _check(lib().fk_engine_add(self.h, *m.args(), C.byref(slot)), allow=(FK_EBUSY, FK_ENOMEM))
        if st != FK_OK:
            return None
        self.problems[slot.value] = problem
        self._marsh[slot.value] = m
        return slot.value

    def tick(self):
        n = self.cfg.max_instances
        reps = (fk_iter_report * n)()
        mask = (C.c_uint8 * n)()
        _check(lib().fk_engine_tick(self.h, reps, mask))
        return {i: reps[i].as_dict() for i in range(n) if mask[i]}

    def get(self, slot):
        p = self.problems[slot]
        u = np.zeros((p.ny, p.nx), dtype=np.complex128)
        se = np.zeros((p.ny, p.nx), dtype=np.complex128)
        _check(lib().fk_engine_get(self.h, int(slot), _dptr(u.view(np.float64)), _dptr(se.view(np.float64))))
        return u, se

    def node_stats(self, slot):
        p = self.problems[slot]
        sj = np.zeros(p.nx * p.ny, dtype=np.int64)
        cp = np.zeros(p.nx * p.ny, dtype=np.int64)
        _check(lib().fk_engine_node_stats(self.h, int(slot), sj.ctypes.data_as(C.POINTER(C.c_int64)),
                                          cp.ctypes.data_as(C.POINTER(C.c_int64))))
        return sj, cp

    def set_iterate(self, slot, u, n):
        ub = np.ascontiguousarray(np.asarray(u, dtype=np.complex128))
        _check(lib().fk_engine_set_iterate(self.h, int(slot), ub.ctypes.data_as(C.c_void_p), int(n), 0))

    def set_pdd(self, slot, cuts_x, cuts_y):
        """Probabilistic domain decomposition of a resident instance before
        its first tick (as Solver.set_pdd).  Returns False when the engine
        cannot hold it now (FK_ENOMEM)."""
        cx = np.ascontiguousarray(np.asarray(cuts_x, dtype=np.int32))
        cy = np.ascontiguousarray(np.asarray(cuts_y, dtype=np.int32))
        i32p = C.POINTER(C.c_int32)
        st = _check(lib().fk_engine_set_pdd(self.h, int(slot), cx.ctypes.data_as(i32p), len(cx),
                                            cy.ctypes.data_as(i32p), len(cy)), allow=(FK_ENOMEM,))
        return st == FK_OK

    def remove(self, slot):
        _check(lib().fk_engine_remove(self.h, int(slot)))
        self.problems.pop(slot, None)
        self._marsh.pop(slot, None)

    def timing(self, reset=False):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().fk_engine_timing(self.h, C.byref(ms), C.byref(n), 1 if reset else 0))
        return float(ms.value), int(n.value)
