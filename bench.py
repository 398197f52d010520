"""Benchmark of the Feynman-Kac fixed-point Helmholtz path on one MI355X.

Default workload (one GPU): the 65x65 unit-square cavity, plane-wave data
theta = pi/6, k = 2, M = 4096 paths per node, h = 1e-4, FP64, one instance
on the plain (non-persistent) path kernel.  A step is one fixed-point
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
# Algorithmic floating-point operations per path-step (FMA = 2, compare and
# transcendental = 1) of the stepping loop with f = 0 and u_n interpolated:
# uniforms 2, Box-Muller 3.5 (2 transcendentals + 1.5 mul), step 4, exit test
# 4, cell location 8, complex bilinear lerps 18, integrand and accumulation 4;
# the FP32 path adds 6 for the compensated (Kahan) integral.
FLOPS_PER_STEP = {64: 44.0, 32: 50.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--k", type=float, default=2.0)
    ap.add_argument("--precision", type=int, default=64, choices=[32, 64])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


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


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
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
    floor_iter = next((r["n"] for r in reports if r["max_du"] < r["noise_floor"]), None)
    s.close()
    ms_per_step = wall / a.steps * 1e3
    solve_iters = floor_iter if floor_iter else len(reports)

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
        "config": {"workload": "unit-square cavity 65x65, plane wave theta=pi/6, k=%g, M=4096, h=1e-4, "
                               "single instance, plain path kernel" % a.k,
                   "grid": [65, 65], "M": 4096, "h": 1e-4, "k": a.k, "precision": a.precision},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": None,
                     "kernel": "fk_paths_kernel<%s>" % ("double" if a.precision == 64 else "float"),
                     "kernel_ms_avg": avg_kernel_s * 1e3, "flops_per_path_step": FLOPS_PER_STEP[a.precision]},
        "extra": {"solves_per_s": 1.0 / (ms_per_step / 1e3 * solve_iters),
                  "iterations_per_solve": solve_iters,
                  "rms_error_vs_exact": rms,
                  "path_steps_per_iteration": steps_total / a.steps},
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
