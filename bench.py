"""Benchmark of the Feynman-Kac fixed-point Helmholtz path on one MI355X.

Default workload (one GPU): the 65x65 unit-square cavity, plane-wave data
theta = pi/6, k = 2, M = 4096 paths per node, h = 1e-4, FP64, one instance
(the single-instance solver, no batching).  A step is one fixed-point
iteration: Philox normals, Euler-Maruyama paths with exit test and boundary
datum, the left-point integral of f - k^2 u_n with u_n interpolated from the
device-resident grid, per-node reduction and the update of the iterate.

Prints one JSON line: path-steps/s (value), ms per iteration, the roofline
of the path kernel (device time from HIP events recorded on the stream the
kernel runs on), the CPU oracle timed on a bounded sample on this host, and
extra figures (solves/s, RMS error against the exact plane wave).
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
KERNEL = {64: "fk_stream_f64_l1", 32: "fk_stream_f32"}
# HBM bytes per launch of the path kernels from FETCH_SIZE / WRITE_SIZE
# counters (scaled by a plain copy of known size), valid only for the kernel
# sources they were taken on
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fk_stream_traffic.json")
KERNEL_SOURCES = ["fk_kernels.hip", "fk_device.hpp", "fk_internal.hpp"]


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
    k = t.get("kernels", {}).get(kernel)
    if t.get("source_sha") != kernel_source_hash() or not k or k.get("workload") != workload:
        return None
    return k


def measured_traffic(kernel, workload):
    """Counter-derived HBM bytes per launch, or None (see measured_counters)."""
    k = measured_counters(kernel, workload)
    return None if k is None else k["bytes_per_launch"]


def _issue(k):
    if k is None or "valu_busy" not in k:
        return None
    return {"busy": k["valu_busy"], "lane_utilisation": k["valu_lane_utilisation"],
            "instructions_per_path_step": k["valu_instructions_per_path_step"]}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=float, default=2.0)
    ap.add_argument("--precision", type=int, default=64, choices=[32, 64])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP32, batched and serving figures")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--annulus-only", action="store_true",
                    help="only time the reflecting-edge kernels on the shape-3 annulus and print that line")
    ap.add_argument("--pdd-only", action="store_true",
                    help="only run the domain-decomposed bench cavity and print that line")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (the reference kernel for "
                         "scaling HBM byte counters) and exit")
    return ap.parse_args()


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


def cpu_baseline(p, target_s):
    """The CPU oracle, as it is, on a bounded sample of the same workload:
    one Feynman-Kac step (all M paths) at a growing set of interior nodes
    spread over the grid, with u_n = the exact plane wave on the grid (a
    closed-form input), until about target_s seconds of work."""
    import numpy as np
    from oracle import fkmc
    ids = fkmc.interior_ids(p)
    rng = np.random.default_rng(0)
    order = rng.permutation(ids)
    u = None
    from paper_2308_11469_amd import workloads as W
    u = W.exact_solution(p)
    threads = len(os.sched_getaffinity(0))
    done, steps, t_used = 0, 0, 0.0
    batch = max(threads, 4)
    while t_used < target_s and done < len(order):
        sel = order[done:done + batch]
        t0 = time.perf_counter()
        est = fkmc.fk_nodes(p, u, 1, sel, nthreads=threads)
        t_used += time.perf_counter() - t0
        steps += int(est["sumJ"].sum())
        done += len(sel)
        if t_used < target_s / 4:
            batch *= 2
    return dict(value=steps / t_used, unit="path-steps/s", cores=threads, kind="oracle",
                sample="%d of %d interior nodes x M=%d paths, one iteration (u_n = exact wave), "
                       "%.3g path-steps in %.1f s" % (done, len(ids), p.M, steps, t_used))


def fp32_same_config(k, steps):
    """The same cavity on the FP32 path: path-steps/s and kernel time."""
    import torch
    from paper_2308_11469_amd import fkh
    from paper_2308_11469_amd import workloads as W
    s = fkh.Solver(W.cavity_65(k=k, precision=32))
    s.iterate(2)
    s.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [s.iterate(1) for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, n = s.timing()
    s.close()
    steps_total = sum(r["path_steps"] for r in reps)
    return dict(value=steps_total / wall, unit="path-steps/s", ms_per_step=wall / steps * 1e3,
                kernel_ms_avg=ms / max(n, 1),
                roofline_frac=FLOPS_PER_STEP[32] * steps_total / (ms / 1e3) / 1e12 / PEAK_TFLOPS[32])


def annulus_shape3(steps=3):
    """The annular problem of Sec. 2.3 on the paper's shape 3 (rectangle
    [-0.5, 0.5] x [-0.8, 0.8] with the box hole [-0.05, 0.05] x [-0.4, 0.4],
    reflecting Robin edge) at the grid step 0.01 of its FE mesh (101 x 161
    nodes), k = 0.5, M = 4096, h = 1e-4: path-steps/s of the reflecting
    kernels in both precisions, one iteration per step after two warm-up
    iterations."""
    import torch
    from paper_2308_11469_amd import fkh
    from paper_2308_11469_amd import workloads as W
    out = {"workload": "annulus shape 3, 101x161, k=0.5, M=4096, h=1e-4, reflecting edge"}
    for prec in (64, 32):
        s = fkh.Solver(W.annulus_shape3(k=0.5, nx=101, ny=161, M=4096, h=1e-4, precision=prec))
        s.iterate(2)
        s.timing(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = [s.iterate(1) for _ in range(steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms, n = s.timing()
        s.close()
        total = sum(r["path_steps"] for r in reps)
        out["fp%d" % prec] = dict(value=total / wall, unit="path-steps/s", ms_per_step=wall / steps * 1e3,
                                  kernel_ms_avg=ms / max(n, 1), path_steps_per_iteration=total / steps,
                                  roofline_frac=FLOPS_PER_STEP[prec] * total / (ms / 1e3) / 1e12
                                  / PEAK_TFLOPS[prec])
    return out


def pdd_cavity65(k, n_iters=12):
    """The bench cavity (FP64, M = 4096, h = 1e-4) by probabilistic domain
    decomposition: paths from the nodes on the grid lines 16, 32, 48 in x
    and y only (369 of 3969 unknowns), the 16 blocks of 15 x 15 nodes solved
    on the device.  Wall time per iteration, path-steps per iteration,
    iterations to the first settled iteration, RMS error against the plane
    wave after n_iters iterations."""
    import numpy as np
    import torch
    from paper_2308_11469_amd import fkh, serving
    from paper_2308_11469_amd import workloads as W
    p = W.cavity_65(k=k, precision=64)
    s = fkh.Solver(p)
    s.set_pdd([16, 32, 48], [16, 32, 48])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [s.iterate(1) for _ in range(n_iters)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    u, _ = s.get()
    s.close()
    ex = W.exact_solution(p)
    ids = np.nonzero((np.arange(p.nx * p.ny) % p.nx > 0) & (np.arange(p.nx * p.ny) % p.nx < p.nx - 1)
                     & (np.arange(p.nx * p.ny) // p.nx > 0) & (np.arange(p.nx * p.ny) // p.nx < p.ny - 1))[0]
    settle = next((r["n"] for r in reps if serving.settled(r)), None)
    ms = wall / n_iters * 1e3
    return {"workload": "cavity 65x65, k=%g, M=4096, h=1e-4, FP64, interfaces x,y in {16,32,48}" % k,
            "ms_per_iteration": ms, "path_steps_per_iteration": sum(r["path_steps"] for r in reps) / n_iters,
            "iterations_per_solve": settle,
            "solves_per_s": (1e3 / (ms * settle)) if settle else None,
            "rms_error_vs_exact": float(np.sqrt(np.mean(np.abs(u.ravel()[ids] - ex.ravel()[ids]) ** 2)))}


def batched_vs_plain(n_sub=16, ticks=2):
    """Solves/s of the batched FP32 engine (one persistent launch per tick for
    all instances) against the plain FP64 single-instance path (instances one
    after another), on every 16th instance of the 256-rectangle workload, at
    the same iterations (so the same estimator and RMS error up to FP32
    rounding, which stays below 0.1 SE).  Timed: iterations 1..ticks after
    the first (iteration 0 has no interpolation)."""
    import numpy as np
    import torch
    from paper_2308_11469_amd import fkh
    from paper_2308_11469_amd import workloads as W
    probs = W.rect_batch(256)[::256 // n_sub]
    nodes = sum(p.nx * p.ny for p in probs)
    eng = fkh.Engine(len(probs), precision=32, max_grid_nodes=nodes + 4096, max_items=1 << 26,
                     max_table=16, max_instance_nodes=max(p.nx * p.ny for p in probs))
    slots = [eng.add(p) for p in probs]
    eng.tick()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_b = 0
    for _ in range(ticks):
        reps = eng.tick()
        steps_b += sum(r["path_steps"] for r in reps.values())
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / ticks
    err_b = []
    for p, sl in zip(probs, slots):
        u, _ = eng.get(sl)
        err_b.append(np.sqrt(np.mean(np.abs(u - W.exact_solution(p))[1:-1, 1:-1] ** 2)))
    eng.close()
    t_plain = 0.0
    steps_p = 0
    err_p = []
    for p in probs:
        s = fkh.Solver(p.replace(precision=64))
        s.iterate(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(ticks):
            steps_p += s.iterate(1)["path_steps"]
        torch.cuda.synchronize()
        t_plain += (time.perf_counter() - t0) / ticks
        u, _ = s.get()
        err_p.append(np.sqrt(np.mean(np.abs(u - W.exact_solution(p))[1:-1, 1:-1] ** 2)))
        s.close()
    return dict(instances=len(probs), ticks_timed=ticks,
                batched_fp32_s_per_iteration=t_batched, plain_fp64_s_per_iteration=t_plain,
                solves_per_s_ratio=t_plain / t_batched,
                batched_path_steps_per_s=steps_b / ticks / t_batched,
                plain_path_steps_per_s=steps_p / ticks / t_plain,
                rms_error_batched=float(np.mean(err_b)), rms_error_plain=float(np.mean(err_p)),
                note="same iteration counts; iterations per solve are equal on both sides")


def serving_window(n_requests=12):
    """The scattering request stream (Poisson arrivals at 200/s, k ~ U[1,4],
    grids 33..257, M 1024..8192, h = 1e-4, FP32) for its first n_requests
    arrivals, through the continuous-batching loop; p50/p99 latency of the
    completed requests and solves/s over the window."""
    from paper_2308_11469_amd import fkh, serving
    from paper_2308_11469_amd import workloads as W
    arrivals, params = W.scatter_stream(n_requests)
    reqs = []
    for r, (t, q) in enumerate(zip(arrivals, params)):
        p = W.scatter_problem(q["k"], q["theta"], q["N"], q["M"], q["seed"], precision=32)
        reqs.append(serving.Request(r, t, p.replace(max_iters=12, tol=1e-3)))
    eng = fkh.Engine(8, precision=32, max_grid_nodes=8 * 257 * 257, max_items=1 << 26,
                     max_table=8 * 4 * 8192, max_instance_nodes=257 * 257)
    srv = serving.Server(eng, keep_results=False)
    t0 = time.perf_counter()
    res = srv.run(reqs)
    wall = time.perf_counter() - t0
    eng.close()
    out = serving.latency_summary(res, wall)
    out.update(requests=n_requests, wall_s=wall, offered_rate_per_s=200.0,
               ticks=srv.ticks, max_resident=max((t["resident"] for t in srv.tick_log), default=0))
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.annulus_only:
        print(json.dumps(annulus_shape3(a.steps)), flush=True)
        return
    if a.pdd_only:
        print(json.dumps(pdd_cavity65(a.k)), flush=True)
        return
    import numpy as np
    import torch
    from paper_2308_11469_amd import build, fkh
    from paper_2308_11469_amd import workloads as W

    if not build.is_built():
        build.build()
    torch.cuda.set_device(0)
    p = W.cavity_65(k=a.k, precision=a.precision)
    s = fkh.Solver(p)
    reports = []
    for _ in range(a.warmup):
        reports.append(s.iterate(1))
    s.timing(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timed = []
    for _ in range(a.steps):
        timed.append(s.iterate(1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    reports += timed
    kern_ms, launches = s.timing()
    steps_total = sum(r["path_steps"] for r in timed)
    value = steps_total / wall
    avg_kernel_s = kern_ms / 1e3 / max(launches, 1)
    steps_per_launch = steps_total / max(launches, 1)
    achieved = FLOPS_PER_STEP[a.precision] * steps_per_launch / avg_kernel_s / 1e12
    peak = PEAK_TFLOPS[a.precision]

    u, se = s.get()
    ex = W.exact_solution(p)
    ids = np.nonzero(np.abs(se.ravel()) > 0)[0]
    rms = float(np.sqrt(np.mean(np.abs(u.ravel()[ids] - ex.ravel()[ids]) ** 2)))
    from paper_2308_11469_amd import serving
    floor_iter = next((r["n"] for r in reports if serving.settled(r)), None)
    s.close()
    ms_per_step = wall / a.steps * 1e3
    solve_iters = floor_iter if floor_iter else len(reports)

    workload = ("unit-square cavity 65x65, plane wave theta=pi/6, k=%g, M=4096, h=1e-4, single instance"
                % a.k)
    out = {
        "metric": "Brownian path-steps/s (Helmholtz solves/s at fixed RMS error reported alongside)",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": workload,
                   "grid": [65, 65], "M": 4096, "h": 1e-4, "k": a.k, "precision": a.precision},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": measured_traffic(KERNEL[a.precision], workload),
                     "kernel": KERNEL[a.precision],
                     "kernel_ms_avg": avg_kernel_s * 1e3, "flops_per_path_step": FLOPS_PER_STEP[a.precision],
                     # the ALU bound in issue terms, from the committed counter
                     # profile of these kernel sources (None once they change):
                     # VALU-active cycles at four per instruction over the
                     # dispatch, lanes active per instruction, instructions
                     # per path-step
                     "valu_issue": _issue(measured_counters(KERNEL[a.precision], workload))},
        "extra": {"solves_per_s": 1.0 / (ms_per_step / 1e3 * solve_iters),
                  "iterations_per_solve": solve_iters,
                  "rms_error_vs_exact": rms,
                  "path_steps_per_iteration": steps_total / a.steps},
    }
    if not a.no_extras:
        out["extra"]["fp32_same_config"] = fp32_same_config(a.k, 5)
        out["extra"]["batched_fp32_vs_plain_fp64"] = batched_vs_plain()
        out["extra"]["serving_scatter_window"] = serving_window()
        out["extra"]["annulus_shape3_reflecting"] = annulus_shape3()
        out["extra"]["pdd_same_cavity"] = pdd_cavity65(a.k)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
