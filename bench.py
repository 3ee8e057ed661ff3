#!/usr/bin/env python3
"""Throughput of the fused MRT-LBM step on one MI355X.

Workload: periodic 8192 x 8192 D2Q9 spinodal decomposition in FP32 (phi0 =
U(-0.05, 0.05) from seed 5, alpha = 0.2, m = 4, Willmore eps = 0.03,
M = 0.1, interface eps_w = 1.5 -> D = 2 sqrt(2) eps_w, sigma = 0.01).
One "step" is one time step of lbch_step: pull-stream + phi + all stencils +
anisotropic chemical potential + equilibrium + source + MRT collision.  By
default one kernel launch advances two time steps (temporal blocking).

Prints ONE JSON line: MLUPS (whole job), the roofline of the step kernel
(algorithmic 72 B per lattice update in FP32 = 9 populations read + 9
written, times the updates of one launch; the launch's own minimum traffic,
one read and one write of the state, is reported beside it) and the
oracle's CPU throughput on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic(n_nodes: int, precision: str, depth: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source at this size and depth; else None."""
    from paper_2501_03759_amd.profiling import STEP_KERNELS, kernel_hash
    side = int(round(n_nodes ** 0.5))
    path = os.path.join(ROOT, "profiles", f"{STEP_KERNELS[depth]}_spinodal{side}_{precision}.json")
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if (rec.get("kernel_sha256_16") != kernel_hash() or rec.get("nodes") != n_nodes
            or rec.get("precision") != precision or rec.get("depth", 1) != depth):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(seconds_target: float = 15.0):
    """The oracle (NumPy, FP64, single thread) on a bounded sample of the same workload:
    a 256 x 256 periodic window of the spinodal field with the workload's parameters."""
    from threadpoolctl import threadpool_limits

    from oracle import lbm
    from paper_2501_03759_amd import inputs
    d = inputs.C5
    n = 256
    width = inputs.width_from_eps(d["eps_w"])
    kappa, beta = lbm.kappa_beta_from_sigma_width(inputs.SIGMA_PAPER, width)
    p = lbm.Params(nx=n, ny=n, kappa=kappa, beta=beta, mobility=d["mobility"], alpha=d["alpha"],
                   aniso_m=d["m"], eps_reg=d["eps_reg"])
    phi0 = inputs.spinodal(d["n"], d["n"], seed=d["seed"], amp=d["amp"])[:n, :n].copy()
    with threadpool_limits(limits=1):
        f = lbm.initial_populations(phi0, p)
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds_target:
            f = lbm.step(f, p)
            steps += 1
        dt = time.perf_counter() - t0
    return {"value": n * n * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of a {n}x{n} window of the workload (FP64 NumPy oracle, 1 thread)"}


def copy_ceiling(torch, lbch, stream, nbytes=1 << 30, reps=5):
    """Practical HBM copy bandwidth (read + write bytes / time) of the library's plain copy kernel."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").uniform_()
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    lbch.diag_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        lbch.diag_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream)
    b.record(stream)
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    ok = bool(torch.equal(src, dst))
    del src, dst
    torch.cuda.empty_cache()
    return {"GBs": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "bytes_per_launch": 2 * nbytes, "ms": round(ms, 4),
            "verified": ok}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=8192, help="grid side (default: the 8192^2 workload)")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--depth", type=int, default=2, choices=[1, 2], help="time steps per kernel launch")
    ap.add_argument("--tiling", type=str, default="", help="block_threads,rows_per_block")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2501_03759_amd import inputs, lbch

    d = inputs.C5
    n = args.n
    prec = lbch.FP32 if args.precision == "fp32" else lbch.FP64
    esize = 4 if prec == lbch.FP32 else 8
    p = lbch.default_params(nx=n, ny=n, precision=prec, sigma_width=(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"])),
                            mobility=d["mobility"], alpha=d["alpha"], aniso_m=d["m"], eps_reg=d["eps_reg"])
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    copy = copy_ceiling(torch, lbch, stream)
    sim = lbch.Sim(p, stream)
    sim.set_time_blocking(args.depth)
    if args.tiling:
        bt, rows = (int(v) for v in args.tiling.split(","))
        sim.set_tiling(bt, rows)
    phi0 = inputs.spinodal(n, n, seed=d["seed"], amp=d["amp"])
    sim.init(phi0)
    del phi0
    sim.step(args.warmup)
    sim.synchronize()

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(args.steps)
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(end)
    ms_step = ms_total / args.steps
    _, mass, lo, hi = sim.moments(want_phi=False)
    tiling = sim.tiling()
    sim.close()

    nodes = n * n
    mlups = nodes * args.steps / (ms_total * 1e-3) / 1e6
    depth = args.depth
    # every launch advances `depth` steps (an odd tail step, if any, is one
    # single-step launch of about half the time: the average below counts it
    # as half a launch)
    launch_ms = ms_step * depth
    bytes_per_update = 18 * esize                      # 9 populations read + 9 written
    alg_bytes = bytes_per_update * nodes * depth       # per launch
    min_bytes = bytes_per_update * nodes               # one read + one write of the state per launch
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(nodes, args.precision, depth),
                "kernel": "step2_fused" if depth == 2 else "step_fused",
                "launch_ms": round(launch_ms, 4), "updates_per_launch": depth * nodes,
                "bytes_per_update": bytes_per_update, "algorithmic_bytes_per_launch": alg_bytes,
                "min_bytes_per_launch": min_bytes,
                "min_bytes_GBs": round(min_bytes / (launch_ms * 1e-3) / 1e9, 1),
                "min_bytes_frac": round(min_bytes / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out = {
        "metric": "MLUPS & % HBM peak (1 GPU)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == lbch.FP32 else "f64",
        "data": "synthetic (seeded spinodal noise U(-0.05,0.05), seed 5)",
        "config": {"workload": f"spinodal-{n}x{n}-{args.precision}", "grid": [n, n], "lattice": "D2Q9",
                   "alpha": d["alpha"], "m": d["m"], "regularization": "willmore", "eps_reg": d["eps_reg"],
                   "mobility": d["mobility"], "time_steps_per_launch": depth, "tiling": list(tiling)},
        "roofline": roofline,
        "checks": {"mass": mass, "phi_min": lo, "phi_max": hi},
        "hbm_copy": copy,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
