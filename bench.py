"""Benchmark of the Feynman-Kac fixed-point Helmholtz path on one MI355X.

Default workload (the headline line): the 129x129 unit-square cavity with the
complex Gaussian source f = (1 + 0.5i) exp(-|x - (0.3, 0.6)|^2 / (2 0.05^2)),
plane-wave data theta = pi/6, k = 3.5, M = 16384 paths per node, h = 5e-5,
FP64 stepping, one instance through the single-instance solver (the largest
single-instance configuration: 1.9e11 path-steps per iteration).  A step is
one fixed-point iteration: Philox normals, Euler-Maruyama paths with exit test
and boundary datum, the left-point integral of f - k^2 u_n with u_n
interpolated from the device-resident grid, per-node reduction and the update
of the iterate.

Prints one JSON line: path-steps/s (value), ms per iteration, the roofline of
the path kernel (device time from HIP events recorded on the stream the
kernel runs on), the CPU oracle timed on a bounded sample on this host, and
extra figures: the same configuration on the FP32 path, the 65x65 cavity
(FP64 and its solves/s and RMS error against the exact plane wave), one full
tick of the 256-rectangle batch on the FP32 engine, served batched FP32
solves/s (with and without the domain decomposition) against the plain FP64
path on a subset of it, the 400-arrival scattering request window,
the reflecting kernels on the shape-3 annulus and the domain-decomposed
cavity.  ``--only NAME`` runs one of those parts alone and prints its line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks (vector ALU, non-sparse)
PEAK_TFLOPS = {64: 78.6, 32: 157.3}
# Algorithmic floating-point operations per path-step (FMA = 2, compare,
# conversion and transcendental = 1) of the stepping loop with f = 0 and u_n
# interpolated: two uniforms 4 (FP64: convert and scale each) or 2 (FP32: one
# subtraction each), Box-Muller 7 (log, sqrt, cos, sin and 3 mul for one pair
# of normals), step 4, exit test 4, cell location 10, complex bilinear lerps
# 18, integrand 2, left-point sum 1 (FP64) or 1.5 (FP32: half an FP32 add for
# the trip's two values, then half a conversion and half an FP64 add).
FLOPS_PER_STEP = {64: 50.0, 32: 48.5}
# A Gaussian source adds, per left point: two differences to its centre, the
# squared distance (a multiply and a multiply-add), the scale by -1/(2 sigma^2),
# the exponential, the two amplitude products and the two additions into the
# integrand.
FLOPS_GAUSSIAN_SOURCE = 10.0
# HBM bytes per launch of the path kernels from FETCH_SIZE / WRITE_SIZE
# counters (scaled by a plain copy of known size), valid only for the kernel
# sources they were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fk_stream_traffic.json")
# the path kernels and the host code that picks their launch (item size,
# gather layout, LDS staging): counter figures hold for these sources only
KERNEL_SOURCES = ["fk_kernels.hip", "fk_device.hpp", "fk_internal.hpp", "fk_problem.cpp", "fk_problem.hpp",
                  "fk_solver.cpp"]

HEADLINE_WORKLOAD = ("unit-square cavity 129x129, Gaussian source (1+0.5i) at (0.3,0.6) sigma=0.05, "
                     "plane wave theta=pi/6, k=3.5, M=16384, h=5e-5, single instance")
CAVITY65_WORKLOAD = "unit-square cavity 65x65, plane wave theta=pi/6, k=%g, M=4096, h=1e-4, single instance"


def flops_per_step(precision, source=False):
    return FLOPS_PER_STEP[precision] + (FLOPS_GAUSSIAN_SOURCE if source else 0.0)


def path_kernel_name(precision, features, row_major, lds=False):
    """The path kernel the single-instance solver launches (the library's
    choice in launch_stream)."""
    if precision == 64 and features == 0 and row_major:
        return "fk_stream_f64_l1"
    if precision == 32 and lds:
        return "fk_stream_f32_lds<%d>" % features
    return "fk_stream_f%d<%d>" % (precision, features)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2308_11469_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_counters(kernel, workload):
    """The counter record of the kernel on this workload (HBM bytes per
    launch, VALU issue figures), or None when no measurement exists for these
    kernel sources and this workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_hash():
        return None
    for k in t.get("records", []):
        if k.get("kernel") == kernel and k.get("workload") == workload:
            return k
    return None


def measured_traffic(kernel, workload):
    """Counter-derived HBM bytes per launch, or None (see measured_counters)."""
    k = measured_counters(kernel, workload)
    return None if k is None else k["bytes_per_launch"]


def _issue(k):
    if k is None or "valu_busy" not in k:
        return None
    return {"busy": k["valu_busy"], "lane_utilisation": k["valu_lane_utilisation"],
            "instructions_per_path_step": k["valu_instructions_per_path_step"]}


ONLY = ("headline", "fp32_same_config", "cavity65", "batch256_tick", "served_vs_plain", "scatter_served_vs_plain",
        "serving", "serving_pdd", "serving_sweep", "annulus", "disc_annulus", "pdd", "tuned_tick")


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", type=int, default=64, choices=[32, 64],
                    help="stepping precision of the headline line")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the extra figures")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--only", choices=ONLY, default=None,
                    help="run one part alone and print its line (headline: no extras, no CPU baseline)")
    ap.add_argument("--k", type=float, default=2.0, help="k of the 65x65 cavity line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (the reference kernel for "
                         "scaling HBM byte counters) and exit")
    return ap.parse_args(argv)


def calibrate_copy(mib):
    """Three plain device copies of mib MiB each: a profiler's FETCH_SIZE and
    WRITE_SIZE for this copy kernel, against the mib MiB it must move each
    way, give the factor that turns those counters into bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "copies": 3, "bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4}))


def _log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ------------------------------------------------------------- CPU oracle

def cpu_baseline(target_s):
    """The CPU oracle, as it is, on bounded samples of the headline workload
    and in full on the 9x9 cavity:

    - one Feynman-Kac step (all M = 16384 paths) at a growing set of
      interior nodes of the 129x129 source cavity spread over the grid, with
      u_n = the plane wave of the boundary data on the grid (a closed-form
      input; the work per path does not depend on the values), on all host
      threads for about target_s seconds, then on one thread for about a
      quarter of that;
    - the 9x9 cavity (M = 500, h = 2e-3) for all 10 iterations, all threads.
    """
    import numpy as np
    from oracle import fkmc
    from paper_2308_11469_amd import workloads as W
    p = W.cavity_source(precision=64)
    xs = p.x0 + np.arange(p.nx) * ((p.x1 - p.x0) / (p.nx - 1))
    ys = p.y0 + np.arange(p.ny) * ((p.y1 - p.y0) / (p.ny - 1))
    X, Y = np.meshgrid(xs, ys)
    u = W.plane_wave(p.k, p.outer.theta, X, Y)
    ids = fkmc.interior_ids(p)
    order = np.random.default_rng(0).permutation(ids)
    threads = len(os.sched_getaffinity(0))

    def run(nthreads, budget, start):
        done, steps, t_used = 0, 0, 0.0
        batch = nthreads
        while t_used < budget and start + done < len(order):
            sel = order[start + done:start + done + batch]
            t0 = time.perf_counter()
            est = fkmc.fk_nodes(p, u, 1, sel, nthreads=nthreads)
            t_used += time.perf_counter() - t0
            steps += int(est["sumJ"].sum())
            done += len(sel)
        return done, steps, t_used

    done, steps, t_used = run(threads, target_s, 0)
    done1, steps1, t1 = run(1, target_s / 4, done)
    c1 = W.cavity_small()
    t0 = time.perf_counter()
    r1 = fkmc.solve(c1, max_iters=10, tol=0.0, nthreads=threads)
    tc1 = time.perf_counter() - t0
    c1_steps = sum(h["sumJ"] for h in r1["history"])
    return dict(value=steps / t_used, unit="path-steps/s", cores=threads, kind="oracle",
                sample="%d of %d interior nodes of the 129x129 source cavity x M=%d paths, one iteration "
                       "(u_n = the boundary plane wave on the grid), %.3g path-steps in %.1f s on %d threads"
                       % (done, len(ids), p.M, steps, t_used, threads),
                single_thread=dict(value=steps1 / t1, unit="path-steps/s", cores=1,
                                   sample="%d further nodes, %.3g path-steps in %.1f s" % (done1, steps1, t1)),
                cavity9_full=dict(iterations=10, path_steps=int(c1_steps), seconds=tc1,
                                  value=c1_steps / tc1, unit="path-steps/s", cores=threads,
                                  solves_per_s=1.0 / tc1))


# ------------------------------------------------------------- GPU parts

def _timed_solver(p, steps, warmup, **kw):
    """Iterates a single-instance solver: warm-up iterations, then `steps`
    timed ones between device synchronisations.  Returns the reports (all),
    the timed wall time, the path kernel's HIP-event time and launch count
    over the timed iterations, and the final iterate and SE."""
    import torch
    from paper_2308_11469_amd import fkh
    s = fkh.Solver(p, **kw)
    reports = [s.iterate(1) for _ in range(warmup)]
    s.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed = [s.iterate(1) for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, launches = s.timing()
    u, se = s.get()
    s.close()
    # the library keeps the gather copy row-major while it fits 80 KiB
    # (automatic layout): FP32 8 bytes per node, FP64 16; a single FP32
    # instance without a reflecting edge whose row-major copy fits 156 KiB has
    # it staged in LDS
    layout = kw.get("gather_layout", "auto")
    node_bytes = 8 if p.precision == 32 else 16
    lds = p.precision == 32 and not p.reflect and layout != "cells" and p.nx * p.ny * 8 <= 156 * 1024
    row_major = layout == "nodes" or (layout == "auto" and (p.nx * p.ny * node_bytes <= 80 * 1024 or lds))
    return dict(reports=reports + timed, timed=timed, wall=wall, kern_ms=kern_ms, launches=launches, u=u, se=se,
                row_major=row_major, lds=lds)


def _features(p):
    return ((1 if p.domain_kind != "rect" else 0) | (2 if p.src_kind != "zero" else 0)
            | (4 if (p.alpha is not None and p.alpha != p.k * p.k) or p.damping != 0.0 else 0)
            | (8 if p.reflect else 0) | (64 if p.domain_kind in ("disc_minus_rhombus", "disc_minus_disc") else 0))


def _roofline(p, run, workload):
    steps_total = sum(r["path_steps"] for r in run["timed"])
    launches = max(run["launches"], 1)
    avg_kernel_s = run["kern_ms"] / 1e3 / launches
    fl = flops_per_step(p.precision, p.src_kind == "gaussian")
    achieved = fl * steps_total / launches / avg_kernel_s / 1e12
    peak = PEAK_TFLOPS[p.precision]
    kernel = path_kernel_name(p.precision, _features(p), run["row_major"], run["lds"])
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": measured_traffic(kernel, workload), "kernel": kernel,
            "kernel_ms_avg": avg_kernel_s * 1e3, "flops_per_path_step": fl,
            "path_steps_per_launch": steps_total / launches,
            # the ALU bound in issue terms, from the committed counter profile
            # of these kernel sources (None once they change): VALU-active
            # cycles at four per instruction over the dispatch, lanes active
            # per instruction, instructions per path-step
            "valu_issue": _issue(measured_counters(kernel, workload))}


def _settle(reports):
    from paper_2308_11469_amd import serving
    return next((r["n"] for r in reports if serving.settled(r)), None)


def headline(steps, warmup, precision):
    from paper_2308_11469_amd import workloads as W
    p = W.cavity_source(precision=precision)
    _log("headline: 129x129 source cavity, FP%d, %d warm-up + %d timed iterations" % (precision, warmup, steps))
    run = _timed_solver(p, steps, warmup)
    steps_total = sum(r["path_steps"] for r in run["timed"])
    ms_per_step = run["wall"] / steps * 1e3
    settle = _settle(run["reports"])
    return p, run, {
        "value": steps_total / run["wall"],
        "ms_per_step": ms_per_step,
        "roofline": _roofline(p, run, HEADLINE_WORKLOAD),
        "extra": {"path_steps_per_iteration": steps_total / steps,
                  # iterations to the first settled iteration (the change is
                  # Monte Carlo noise: noise ratio below 9/8), None if not
                  # reached in this run
                  "iterations_per_solve": settle,
                  "solves_per_s": (1e3 / (ms_per_step * settle)) if settle else None,
                  "capped_paths": int(sum(r["capped"] for r in run["reports"])),
                  "max_se_last": run["reports"][-1]["max_se"]},
    }


def fp32_same_config(steps=3):
    """The headline configuration on the FP32 path."""
    from paper_2308_11469_amd import workloads as W
    p = W.cavity_source(precision=32)
    _log("fp32_same_config")
    run = _timed_solver(p, steps, 1)
    total = sum(r["path_steps"] for r in run["timed"])
    rf = _roofline(p, run, HEADLINE_WORKLOAD)
    return dict(value=total / run["wall"], unit="path-steps/s", ms_per_step=run["wall"] / steps * 1e3,
                kernel=rf["kernel"], kernel_ms_avg=rf["kernel_ms_avg"], roofline_frac=rf["frac"],
                path_steps_per_launch=rf["path_steps_per_launch"], flops_per_path_step=rf["flops_per_path_step"],
                traffic=rf["traffic"], valu_issue=rf["valu_issue"])


def cavity65(k, steps=5, warmup=2):
    """The 65x65 cavity (FP64 and FP32): path-steps/s, solves/s (iterations
    to the first settled iteration) and the RMS error against the exact plane
    wave."""
    import numpy as np
    from paper_2308_11469_amd import workloads as W
    out = {"workload": CAVITY65_WORKLOAD % k}
    for prec in (64, 32):
        p = W.cavity_65(k=k, precision=prec)
        _log("cavity65 FP%d" % prec)
        run = _timed_solver(p, steps, warmup)
        total = sum(r["path_steps"] for r in run["timed"])
        ms = run["wall"] / steps * 1e3
        settle = _settle(run["reports"])
        ex = W.exact_solution(p)
        ids = np.nonzero(np.abs(run["se"].ravel()) > 0)[0]
        rf = _roofline(p, run, out["workload"])
        out["fp%d" % prec] = dict(
            value=total / run["wall"], unit="path-steps/s", ms_per_step=ms, kernel=rf["kernel"],
            kernel_ms_avg=rf["kernel_ms_avg"], roofline_frac=rf["frac"], traffic=rf["traffic"],
            path_steps_per_launch=rf["path_steps_per_launch"],
            valu_issue=rf["valu_issue"], iterations_per_solve=settle,
            solves_per_s=(1e3 / (ms * settle)) if settle else None,
            rms_error_vs_exact=float(np.sqrt(np.mean(np.abs(run["u"].ravel()[ids] - ex.ravel()[ids]) ** 2))))
    return out


def batch256_tick():
    """One tick of the full 256-rectangle batch on the FP32 engine: every
    instance advanced by one fixed-point iteration in one persistent launch
    (the first iteration: the gathers of u_n run, with coefficient zero)."""
    import torch
    from paper_2308_11469_amd import fkh
    from paper_2308_11469_amd import workloads as W
    probs = W.rect_batch(256)
    nodes = sum(p.nx * p.ny for p in probs)
    _log("batch256_tick: %d instances, %d grid nodes" % (len(probs), nodes))
    t0 = time.perf_counter()
    eng = fkh.Engine(len(probs), precision=32, max_grid_nodes=nodes + 4096, max_items=1 << 31,
                     max_table=16, max_instance_nodes=max(p.nx * p.ny for p in probs))
    slots = [eng.add(p) for p in probs]
    t_add = time.perf_counter() - t0
    assert all(s is not None for s in slots)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = eng.tick()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, _ = eng.timing()
    eng.close()
    steps = sum(r["path_steps"] for r in reps.values())
    return dict(instances=len(reps), grid_nodes=nodes, admit_s=t_add, tick_s=wall, kernel_ms=kern_ms,
                path_steps=int(steps), value=steps / wall, unit="path-steps/s",
                capped_paths=int(sum(r["capped"] for r in reps.values())),
                kernel="fk_stream_f32<0>",
                roofline_frac=FLOPS_PER_STEP[32] * steps / (kern_ms / 1e3) / 1e12 / PEAK_TFLOPS[32])


def tuned_tick(n_sub=16):
    """Every 16th rectangle of the 256-rectangle workload in one FP32 engine:
    one tick (after a warm-up tick) with the library's own launch choice and
    one with the autotuner's per-instance item size and gather layout
    (proxy of 256 paths, item sizes 128-1024, both layouts, each proxy winner
    checked at the full M against the library's choice; cached per shape in
    a temporary file).  Launch parameters never change results, which is
    checked here too; the tuning time is reported beside."""
    import tempfile

    import numpy as np
    import torch
    from paper_2308_11469_amd import autotune, fkh
    from paper_2308_11469_amd import workloads as W
    probs = W.rect_batch(256)[::n_sub]
    nodes = sum(p.nx * p.ny for p in probs)
    _log("tuned_tick: tuning %d shapes" % len(probs))
    with tempfile.TemporaryDirectory() as d:
        tuner = autotune.Tuner(cache_path=os.path.join(d, "tune.json"), proxy_paths=256,
                               ppi=(128, 256, 512, 1024), waves=(16,))
        t0 = time.perf_counter()
        cfgs = [tuner.instance_config(p) for p in probs]
        tune_s = time.perf_counter() - t0
    out = {"instances": len(probs), "tune_s": tune_s, "timed_runs": tuner.timed,
           "tuned_configs": sum(1 for c in cfgs if c["paths_per_item"] != 0)}
    us = {}
    for mode in ("auto", "tuned"):
        _log("tuned_tick: %s" % mode)
        eng = fkh.Engine(len(probs), precision=32, max_grid_nodes=nodes + 4096, max_items=1 << 31,
                         max_table=16, max_instance_nodes=max(p.nx * p.ny for p in probs))
        slots = [eng.add(p, **(c if mode == "tuned" else {})) for p, c in zip(probs, cfgs)]
        assert all(s is not None for s in slots)
        eng.tick()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = eng.tick()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        us[mode] = [eng.get(s)[0] for s in slots]
        eng.close()
        steps = sum(r["path_steps"] for r in reps.values())
        out[mode] = {"tick_s": wall, "path_steps": int(steps), "value": steps / wall, "unit": "path-steps/s"}
    out["tuned_over_auto"] = out["tuned"]["value"] / out["auto"]["value"]
    out["bit_identical"] = all(np.array_equal(a, b) for a, b in zip(us["auto"], us["tuned"]))
    return out


def _served_comparison(probs, spacing, unknown_mask, max_table, tag):
    """Solves/s at the stopping rule (settled, max |du| < tol or max_iters)
    of the given requests:

    - plain: the FP64 single-instance solver with paths from every unknown
      node, the instances one after another;
    - served: the same requests all arriving at once at the continuous-
      batching loop over the FP32 engine (one persistent launch per tick),
      with paths from every node, and with the probabilistic domain
      decomposition (interface lines every `spacing` nodes, the blocks between
      them solved on the device in the same tick; Sec. 3's two-stage
      procedure).

    RMS error of each result against the exact solution over the unknown
    nodes (mean over the instances) beside each rate."""
    import numpy as np
    import torch
    from paper_2308_11469_amd import fkh, serving
    from paper_2308_11469_amd import workloads as W
    nodes = sum(p.nx * p.ny for p in probs)

    def rms(p, u):
        m = unknown_mask(p)
        return float(np.sqrt(np.mean(np.abs(u - W.exact_solution(p))[m] ** 2)))

    _log("%s: plain FP64" % tag)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    err_p, its_p = [], []
    for p in probs:
        q = p.replace(precision=64)
        s = fkh.Solver(q)
        while True:
            rep = s.iterate(1)
            if rep["diverging"] or rep["max_du"] < q.tol or serving.settled(rep) or rep["n"] >= q.max_iters:
                break
        err_p.append(rms(q, s.get()[0]))
        its_p.append(rep["n"])
        s.close()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    out = {"instances": len(probs), "pdd_spacing": spacing,
           "plain_fp64": dict(wall_s=t_plain, solves_per_s=len(probs) / t_plain,
                              rms_error=float(np.mean(err_p)), iterations_mean=float(np.mean(its_p)))}
    for name, pdd in (("served_fp32", False), ("served_fp32_pdd", True)):
        _log("%s: %s" % (tag, name))
        eng = fkh.Engine(len(probs), precision=32, max_grid_nodes=nodes + 4096, max_items=1 << 28,
                         max_table=max_table, max_instance_nodes=max(p.nx * p.ny for p in probs))
        reqs = []
        for i, p in enumerate(probs):
            cx, cy = serving.grid_cuts(p.nx, spacing), serving.grid_cuts(p.ny, spacing)
            reqs.append(serving.Request(i, 0.0, p, pdd=(cx, cy) if pdd and (cx or cy) else None))
        srv = serving.Server(eng, keep_results=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.run(reqs)
        wall = time.perf_counter() - t0
        eng.close()
        done = [r for r in res.values() if r.outcome in ("converged", "max_iters", "diverged")]
        out[name] = dict(wall_s=wall, solves_per_s=len(done) / wall, completed=len(done),
                         rms_error=float(np.mean([rms(probs[r.rid], r.u) for r in done])),
                         iterations_mean=float(np.mean([r.iterations for r in done])),
                         path_steps=int(sum(r.path_steps for r in done)), ticks=srv.ticks)
    out["ratio_served_fp32_vs_plain_fp64"] = out["served_fp32"]["solves_per_s"] / out["plain_fp64"]["solves_per_s"]
    out["ratio_served_fp32_pdd_vs_plain_fp64"] = (out["served_fp32_pdd"]["solves_per_s"]
                                                  / out["plain_fp64"]["solves_per_s"])
    out["rms_ratio_pdd_vs_plain"] = out["served_fp32_pdd"]["rms_error"] / out["plain_fp64"]["rms_error"]
    return out


def served_vs_plain(n_sub=16, spacing=32):
    """The served-vs-plain comparison (see _served_comparison) on every 16th
    instance of the 256-rectangle workload, errors against the exact plane
    wave."""
    from paper_2308_11469_amd import workloads as W
    probs = W.rect_batch(256)[::256 // n_sub]

    def interior(p):
        import numpy as np
        m = np.zeros((p.ny, p.nx), bool)
        m[1:-1, 1:-1] = True
        return m
    return _served_comparison(probs, spacing, interior, 16, "served_vs_plain")


def scatter_served_vs_plain(n_sub=16, spacing=32):
    """The same comparison on the scattering stream's requests: the first 16
    of every 12th of the 400 arrivals that the server's predicted-contraction
    rule admits,
    grids 33..257 on [-1, 1]^2 around the sound-soft disc, errors against the
    exact disc series.  With the decomposition, the blocks touching the disc
    keep their own paths and the others are solved."""
    import numpy as np
    from paper_2308_11469_amd import serving
    from paper_2308_11469_amd import workloads as W
    _, params = W.scatter_stream(400, 200.0, 5)
    probs = []
    for q in params[::12]:
        p = W.scatter_problem(q["k"], q["theta"], q["N"], q["M"], q["seed"], precision=32)
        if serving.predicted_rho(p) < 0.98:
            probs.append(p)
    probs = probs[:n_sub]

    def unknown(p):
        xs = p.x0 + np.arange(p.nx) * ((p.x1 - p.x0) / (p.nx - 1))
        ys = p.y0 + np.arange(p.ny) * ((p.y1 - p.y0) / (p.ny - 1))
        X, Y = np.meshgrid(xs, ys)
        m = (X - p.cx) ** 2 + (Y - p.cy) ** 2 > p.r ** 2
        m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = False
        return m
    return _served_comparison(probs, spacing, unknown, len(probs) * 4 * 8192, "scatter_served_vs_plain")


def _scatter_requests(n, rate, seed=5, pdd_spacing=None):
    """The scattering stream's requests; each problem (with its boundary
    table from the disc series) is built when the server first looks at the
    request, so requests turned away at a full queue cost nothing.  With
    pdd_spacing, requests carry decomposition lines every pdd_spacing nodes
    (grids too small for a line run without)."""
    from paper_2308_11469_amd import serving
    from paper_2308_11469_amd import workloads as W
    arrivals, params = W.scatter_stream(n, rate, seed)
    reqs = []
    for r, (t, q) in enumerate(zip(arrivals, params)):
        make = (lambda q=q: W.scatter_problem(q["k"], q["theta"], q["N"], q["M"], q["seed"], precision=32))
        cuts = serving.grid_cuts(q["N"], pdd_spacing) if pdd_spacing else []
        reqs.append(serving.Request(r, float(t), None, make=make, pdd=(cuts, cuts) if cuts else None))
    return reqs


def serving_window(n_requests=400, rate=200.0, max_queue=32, slots=8, pdd_spacing=None):
    """The scattering request stream (Poisson arrivals, k ~ U[1, 4], grids
    33..257, M 1024..8192, h = 1e-4, FP32) through the continuous-batching
    loop with a bounded waiting queue: completed solves/s, p50 / p99 latency
    of the completed requests, turned-away requests by reason, queue growth.
    With pdd_spacing, every request carries decomposition lines."""
    import numpy as np
    from paper_2308_11469_amd import fkh, serving
    reqs = _scatter_requests(n_requests, rate, pdd_spacing=pdd_spacing)
    eng = fkh.Engine(slots, precision=32, max_grid_nodes=slots * 257 * 257, max_items=1 << 26,
                     max_table=slots * 4 * 8192, max_instance_nodes=257 * 257)
    last = [time.perf_counter()]

    def progress(entry):
        now = time.perf_counter()
        if now - last[0] > 10.0:
            last[0] = now
            _log("serving tick %d t=%.1fs resident=%d queued=%d arrived=%d" % (
                entry["tick"], entry["t"], entry["resident"], entry["queued"], entry["arrived"]))

    srv = serving.Server(eng, keep_results=False, max_queue=max_queue, on_tick=progress)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    eng.close()
    out = serving.latency_summary(res, wall, srv.tick_log)
    its = [r.iterations for r in res.values() if r.outcome in ("converged", "max_iters")]
    out.update(requests=n_requests, offered_rate_per_s=rate, max_queue=max_queue, slots=slots, wall_s=wall,
               pdd_spacing=pdd_spacing,
               ticks=srv.ticks, max_resident=max((t["resident"] for t in srv.tick_log), default=0),
               iterations_per_solve_median=float(np.median(its)) if its else None)
    return out


def serving_sweep(capacity, fractions=(0.25, 0.5, 0.8), n_requests=20):
    """The stream offered at fractions of a measured capacity (solves/s):
    the latency / throughput curve below saturation."""
    out = []
    for f in fractions:
        _log("serving sweep at %.2f of capacity" % f)
        r = serving_window(n_requests, f * capacity)
        r.update(capacity_fraction=f, capacity_solves_per_s=capacity)
        out.append(r)
    return out


def annulus_shape3(steps=3):
    """The annular problem of Sec. 2.3 on the paper's shape 3 (rectangle
    [-0.5, 0.5] x [-0.8, 0.8] with the box hole [-0.05, 0.05] x [-0.4, 0.4],
    reflecting Robin edge) at the grid step 0.01 of its FE mesh (101 x 161
    nodes), k = 0.5, M = 4096, h = 1e-4: path-steps/s of the reflecting
    kernels in both precisions, one iteration per step after two warm-up
    iterations."""
    from paper_2308_11469_amd import workloads as W
    out = {"workload": "annulus shape 3, 101x161, k=0.5, M=4096, h=1e-4, reflecting edge"}
    for prec in (64, 32):
        _log("annulus FP%d" % prec)
        p = W.annulus_shape3(k=0.5, nx=101, ny=161, M=4096, h=1e-4, precision=prec)
        run = _timed_solver(p, steps, 2)
        total = sum(r["path_steps"] for r in run["timed"])
        rf = _roofline(p, run, out["workload"])
        out["fp%d" % prec] = dict(value=total / run["wall"], unit="path-steps/s",
                                  ms_per_step=run["wall"] / steps * 1e3, kernel=rf["kernel"],
                                  kernel_ms_avg=rf["kernel_ms_avg"], path_steps_per_iteration=total / steps,
                                  path_steps_per_launch=rf["path_steps_per_launch"],
                                  roofline_frac=rf["frac"], traffic=rf["traffic"], valu_issue=rf["valu_issue"])
    return out


def disc_annulus_shape2(steps=3):
    """The annular problem of Sec. 2.3 on the paper's shape 2 as read here
    (the disc of radius 0.45 minus the centred rhombus of diagonals 0.15,
    reflecting curved edge) at the grid step 0.01 of its FE mesh (91 x 91
    nodes on the disc's square), k = 0.5, M = 4096, h = 1e-4: path-steps/s of
    the disc kernels in both precisions, one iteration per step after two
    warm-up iterations."""
    from paper_2308_11469_amd import workloads as W
    out = {"workload": "annulus shape 2, 91x91, k=0.5, M=4096, h=1e-4, reflecting disc edge"}
    for prec in (64, 32):
        _log("disc annulus FP%d" % prec)
        p = W.annulus_shape2(k=0.5, n=91, M=4096, h=1e-4, precision=prec)
        run = _timed_solver(p, steps, 2)
        total = sum(r["path_steps"] for r in run["timed"])
        rf = _roofline(p, run, out["workload"])
        out["fp%d" % prec] = dict(value=total / run["wall"], unit="path-steps/s",
                                  ms_per_step=run["wall"] / steps * 1e3, kernel=rf["kernel"],
                                  kernel_ms_avg=rf["kernel_ms_avg"], path_steps_per_iteration=total / steps,
                                  path_steps_per_launch=rf["path_steps_per_launch"], roofline_frac=rf["frac"],
                                  traffic=rf["traffic"], valu_issue=rf["valu_issue"])
    return out


def pdd_cavity65(k, n_iters=12):
    """The 65x65 cavity (FP64, M = 4096, h = 1e-4) by probabilistic domain
    decomposition: paths from the nodes on the grid lines 16, 32, 48 in x
    and y only (369 of 3969 unknowns), the 16 blocks of 15 x 15 nodes solved
    on the device.  Wall time per iteration, path-steps per iteration,
    iterations to the first settled iteration, RMS error against the plane
    wave at that iteration and after n_iters iterations."""
    import numpy as np
    import torch
    from paper_2308_11469_amd import fkh, serving
    from paper_2308_11469_amd import workloads as W
    _log("pdd")
    p = W.cavity_65(k=k, precision=64)
    ex = W.exact_solution(p)
    inner = (slice(1, -1), slice(1, -1))

    def rms(u):
        return float(np.sqrt(np.mean(np.abs(u[inner] - ex[inner]) ** 2)))

    s = fkh.Solver(p)
    s.set_pdd([16, 32, 48], [16, 32, 48])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [s.iterate(1) for _ in range(n_iters)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    u, _ = s.get()
    s.close()
    settle = next((r["n"] for r in reps if serving.settled(r)), None)
    rms_settle = None
    if settle:
        s = fkh.Solver(p)
        s.set_pdd([16, 32, 48], [16, 32, 48])
        s.iterate(settle)
        rms_settle = rms(s.get()[0])
        s.close()
    ms = wall / n_iters * 1e3
    return {"workload": "cavity 65x65, k=%g, M=4096, h=1e-4, FP64, interfaces x,y in {16,32,48}" % k,
            "ms_per_iteration": ms, "path_steps_per_iteration": sum(r["path_steps"] for r in reps) / n_iters,
            "iterations_per_solve": settle,
            "solves_per_s": (1e3 / (ms * settle)) if settle else None,
            "rms_error_at_settle": rms_settle,
            "rms_error_after_%d" % n_iters: rms(u)}


def main(argv=None):
    a = parse(argv)
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    import torch
    from paper_2308_11469_amd import build

    if not build.is_built():
        build.build()
    torch.cuda.set_device(0)
    parts = {
        "fp32_same_config": lambda: fp32_same_config(),
        "cavity65": lambda: cavity65(a.k),
        "batch256_tick": batch256_tick,
        "served_vs_plain": served_vs_plain,
        "scatter_served_vs_plain": scatter_served_vs_plain,
        "serving": serving_window,
        "serving_pdd": lambda: serving_window(pdd_spacing=32),
        "annulus": annulus_shape3,
        "disc_annulus": disc_annulus_shape2,
        "pdd": lambda: pdd_cavity65(a.k),
        "tuned_tick": tuned_tick,
    }
    if a.only == "serving_sweep":
        cap = serving_window()["solves_per_s"]
        print(json.dumps({"serving_sweep": serving_sweep(cap)}), flush=True)
        return
    if a.only and a.only != "headline":
        print(json.dumps({a.only: parts[a.only]()}), flush=True)
        return
    p, run, h = headline(a.steps, a.warmup, a.precision)
    out = {
        "metric": "Brownian path-steps/s (Helmholtz solves/s at fixed RMS error, p50/p99 latency "
                  "reported alongside)",
        "value": h["value"],
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": HEADLINE_WORKLOAD, "grid": [129, 129], "M": 16384, "h": 5e-5, "k": 3.5,
                   "precision": a.precision},
        "roofline": h["roofline"],
        "extra": h["extra"],
    }
    if not a.no_extras and a.only is None:
        for name in ("fp32_same_config", "cavity65", "served_vs_plain", "scatter_served_vs_plain", "annulus",
                     "disc_annulus", "pdd", "batch256_tick", "serving", "serving_pdd"):
            out["extra"][name] = parts[name]()
    if not a.no_cpu and a.only is None:
        _log("cpu_baseline")
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
