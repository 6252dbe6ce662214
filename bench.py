#!/usr/bin/env python3
"""Benchmark of the phonon BTE time step on one MI355X.

Workload: 2D 128 x 128 cells, 400 directions (20 polar x 20 azimuthal),
55 band entries (40 frequency bands, 15 of them with a transverse branch),
strip heater on the top wall, implicit backward-Euler steps of 1 ps with
point-Jacobi inner sweeps to a 1e-4 step-relative residual, FP64.  A "step" is
one time step: every inner sweep, energy reduction, temperature inversion and
convergence test of that step.  Inputs are seeded and synthetic (Si-like band
tables), resident in HBM before timing starts.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_bytes(inst, real_bytes):
    """Algorithmic HBM bytes of one sweep launch: read I^k and I^n, write I^{k+1}
    for every (cell, direction, band), plus per-(band, cell) equilibrium read
    and energy-partial write."""
    per_update = 3 * real_bytes
    per_band_cell = 8 + 8
    return inst.n_dof * per_update + inst.n_bands * inst.n_cells * per_band_cell


def measured_traffic(kernel_file, counters_file):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    if it was measured on the kernel source as it is now; else None."""
    import hashlib
    try:
        with open(counters_file) as f:
            c = json.load(f)
        with open(kernel_file, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256") != sha:
        return None
    return c.get("traffic_bytes_per_launch")


def cpu_baseline(inst, log_fn):
    """Oracle (plain FP64 C, OpenMP over cells) on the host cores: the first
    time step of the same workload, all of its inner sweeps."""
    from oracle import Oracle
    from oracle import oracle as om
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", threads))
    om.set_threads(threads)
    log_fn(f"cpu baseline: oracle, first time step of {inst.name}, {threads} threads")
    o = Oracle(inst)
    t0 = time.perf_counter()
    st = o.step()
    dt = time.perf_counter() - t0
    updates = st["inner"] * inst.n_dof
    return {"value": updates / dt, "unit": "updates/s", "cores": om.get_threads(),
            "kind": "oracle",
            "sample": f"first time step of {inst.name} ({st['inner']} inner sweeps, "
                      f"{updates:.3e} updates) in {dt:.1f} s"}


def copy_probe():
    """A plain copy kernel of known size: reads 1 GiB and writes 1 GiB once, so
    the HBM byte counters of a profiler can be scaled against known traffic."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: {4 * n} bytes read, {4 * n} bytes written")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--workload", choices=["c2", "c3", "c4"], default="c2",
                    help="c2 (default, the benchmarked 2D case) or the 3D cases")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the band-sharded design is described, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2305_19400_amd import bte, inputs

    inst = inputs.CONFIGS[args.workload]()
    prec = bte.BTE_FP64 if args.precision == "fp64" else bte.BTE_FP32_MIXED
    real_bytes = 8 if prec == bte.BTE_FP64 else 4
    dev = torch.device("cuda:0")
    log(f"workload {inst.name}: {inst.n} cells, {inst.n_dirs} dirs, {inst.n_bands} bands, "
        f"N_dof={inst.n_dof:.3e}, precision={args.precision}")

    if args.warmup > 0:
        with bte.Solver(inst, device="cuda:0", precision=prec) as sol:
            sol.step(args.warmup)
        log(f"warmup: {args.warmup} steps done")

    sol = bte.Solver(inst, device="cuda:0", precision=prec, timing=True)
    torch.cuda.synchronize(dev)
    sol.sweep_time()  # reset accumulators
    t0 = time.perf_counter()
    stats = []
    chunk = 20
    done = 0
    while done < args.steps:
        n = min(chunk, args.steps - done)
        stats += sol.step(n)
        done += n
        log(f"steps {done}/{args.steps}, inner last={stats[-1]['inner']}")
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    sweep_ms, nsweeps = sol.sweep_time()
    T = sol.temperature()
    sol.close()

    sweeps = sum(s["inner"] for s in stats)
    updates = sweeps * inst.n_dof
    avg_sweep_s = sweep_ms / 1e3 / max(nsweeps, 1)
    achieved = sweep_bytes(inst, real_bytes) / avg_sweep_s / 1e9
    out = {
        "metric": "cell-dir-band updates/s (implicit point-Jacobi sweeps)",
        "value": updates / wall,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if prec == bte.BTE_FP64 else "f32+f64",
        "data": "synthetic (seeded Si-like band tables, strip heater)",
        "config": {"workload": inst.name, "mesh": "x".join(str(v) for v in inst.n[:inst.dim]),
                   "dirs": inst.n_dirs,
                   "bands": inst.n_bands, "dt_s": inst.dt, "tol": inst.tol,
                   "scheme": "implicit backward Euler, point-Jacobi",
                   "time_steps": args.steps},
        "time_to_solution_s": wall,
        "inner_sweeps": sweeps,
        "inner_per_step": {"min": min(s["inner"] for s in stats),
                           "max": max(s["inner"] for s in stats)},
        "T_max_K": float(T.max()),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sweep_kernel", "avg_ms": avg_sweep_s * 1e3,
                     "bytes_per_launch": sweep_bytes(inst, real_bytes)},
    }
    if prec == bte.BTE_FP64 and args.workload == "c2":
        out["roofline"]["traffic"] = measured_traffic(
            os.path.join(ROOT, "paper_2305_19400_amd", "csrc", "bte_kernels.hip"),
            os.path.join(ROOT, "profiles", "sweep2d_c2_fp64_counters.json"))
    if not args.no_cpu_baseline and args.workload == "c2":
        out["cpu_baseline"] = cpu_baseline(inst, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
