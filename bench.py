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


def measured_traffic(n_nodes: int, precision: str, depth: int, lattice: str = "d2q9", path: str = "",
                     tiling=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source at this size, depth (and launch shape, when given); else None."""
    from paper_2501_03759_amd.profiling import STEP_KERNEL_3D, STEP_KERNELS, kernel_hash
    if not path and lattice == "d3q15":
        side = int(round(n_nodes ** (1.0 / 3.0)))
        path = os.path.join(ROOT, "profiles", f"{STEP_KERNEL_3D}_spinodal{side}_{precision}.json")
    elif not path:
        side = int(round(n_nodes ** 0.5))
        path = os.path.join(ROOT, "profiles", f"{STEP_KERNELS[depth]}_spinodal{side}_{precision}.json")
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if (rec.get("kernel_sha256_16") != kernel_hash(lattice) or rec.get("nodes") != n_nodes
            or rec.get("precision") != precision or rec.get("depth", 1) != depth
            or (tiling is not None and rec.get("tiling") != list(tiling))):
        return None
    return rec.get("bytes_per_launch")


def host_info():
    """The host the CPU figures were taken on: usable cores (the process's affinity, what
    `nproc` prints without OMP variables), online CPUs and the CPU model (as `lscpu`)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "online_cpus": os.cpu_count(), "cpu_model": model}


def _oracle_window_worker(args):
    """One process: the oracle (NumPy FP64, one thread) stepping one periodic window for
    about seconds_target; returns (lattice updates, seconds)."""
    phi0, prm, seconds_target = args
    from threadpoolctl import threadpool_limits

    from oracle import lbm
    p = lbm.Params(**prm)
    with threadpool_limits(limits=1):
        f = lbm.initial_populations(phi0, p)
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds_target:
            f = lbm.step(f, p)
            steps += 1
        dt = time.perf_counter() - t0
    return phi0.size * steps, dt


def cpu_baseline(seconds_target: float = 12.0, max_procs: int = 16):
    """The oracle (NumPy, FP64) on a bounded sample of the same workload, on every usable host
    core: one single-threaded oracle process per 256 x 256 window of the 8192^2 spinodal field
    (the workload's parameters), all running at once for about seconds_target.  Called before
    the GPU is initialised (the worker processes are forked)."""
    import multiprocessing as mp

    from oracle import lbm
    from paper_2501_03759_amd import inputs
    d = inputs.C5
    n = 256
    width = inputs.width_from_eps(d["eps_w"])
    kappa, beta = lbm.kappa_beta_from_sigma_width(inputs.SIGMA_PAPER, width)
    prm = dict(nx=n, ny=n, kappa=kappa, beta=beta, mobility=d["mobility"], alpha=d["alpha"], aniso_m=d["m"],
               eps_reg=d["eps_reg"])
    procs = max(1, min(max_procs, len(os.sched_getaffinity(0))))
    field = inputs.spinodal(d["n"], d["n"], seed=d["seed"], amp=d["amp"])
    per_row = d["n"] // n
    wins = [field[(q // per_row) * n:(q // per_row + 1) * n, (q % per_row) * n:(q % per_row + 1) * n].copy()
            for q in range(procs)]
    del field
    with mp.get_context("fork").Pool(procs) as pool:
        res = pool.map(_oracle_window_worker, [(w, prm, seconds_target) for w in wins])
    updates = sum(u for u, _ in res)
    wall = max(t for _, t in res)
    steps = [u // (n * n) for u, _ in res]
    return {"value": updates / wall / 1e6, "unit": "MLUPS", "cores": procs, "kind": "oracle",
            "sample": f"{procs} processes, one per core, each stepping its own {n}x{n} periodic window of the "
                      f"workload's field ({min(steps)}-{max(steps)} steps in {wall:.1f} s; FP64 NumPy oracle, "
                      f"1 thread each)",
            "host": host_info()}


def cpu_baseline_3d(seconds_target: float = 10.0):
    """The D3Q15 oracle (NumPy, FP64, one thread) on a 32^3 periodic window of the 3D workload."""
    from threadpoolctl import threadpool_limits

    from oracle import lbm, lbm3
    from paper_2501_03759_amd import inputs
    d = inputs.C5
    n = 32
    kappa, beta = lbm.kappa_beta_from_sigma_width(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"]))
    p = lbm3.Params(nx=n, ny=n, nz=n, kappa=kappa, beta=beta, mobility=d["mobility"], alpha=d["alpha"],
                    eps_reg=d["eps_reg"])
    phi0 = inputs.spinodal3(n, n, n, seed=d["seed"], amp=d["amp"])
    with threadpool_limits(limits=1):
        f = lbm3.initial_populations(phi0, p)
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < seconds_target:
            f = lbm3.step(f, p)
            steps += 1
        dt = time.perf_counter() - t0
    return {"value": n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of a {n}^3 box of the workload's recipe (FP64 NumPy D3Q15 oracle, 1 thread)"}


def cpu_baseline_ensemble(members, seconds_target: float = 10.0):
    """The oracle stepping ensemble members one after another (FP64, one thread): the first
    members of the list in order, as many whole steps over them as fit."""
    from threadpoolctl import threadpool_limits

    from oracle import lbm
    from paper_2501_03759_amd import inputs
    kappa, beta = lbm.kappa_beta_from_sigma_width(inputs.SIGMA_PAPER, inputs.width_from_eps(1.5))
    sims = []
    for m in members[:8]:
        p = lbm.Params(nx=m["side"], ny=m["side"], kappa=kappa, beta=beta, mobility=0.1, alpha=m["alpha"],
                       aniso_m=m["m"], eps_reg=0.03)
        sims.append((p, lbm.initial_populations(inputs.member_phi0(m), p)))
    nodes = sum(p.nx * p.ny for p, _ in sims)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        sweeps = 0
        while time.perf_counter() - t0 < seconds_target:
            sims = [(p, lbm.step(f, p)) for p, f in sims]
            sweeps += 1
        dt = time.perf_counter() - t0
    return {"value": nodes * sweeps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} steps of the first {len(sims)} members ({nodes} nodes; FP64 NumPy oracle, 1 thread)"}


def cpu_baseline_unet(chans, c_in, seconds_target: float = 10.0):
    """The float64 U-Net oracle's forward on one 64 x 64 patch, FLOPs counted as on the GPU."""
    from threadpoolctl import threadpool_limits

    from oracle import unet
    hw = 64
    params = unet.init_params(len(chans), chans, c_in, seed=0)
    x = np.random.default_rng(0).standard_normal((1, hw, hw, c_in))
    flops = 0.0
    prev = c_in
    for l, c in enumerate(chans):
        flops += 18.0 * (prev * c + c * c) * (hw >> l) ** 2
        prev = c
    for l in range(len(chans) - 2, -1, -1):
        flops += 18.0 * ((chans[l + 1] + chans[l]) * chans[l] + chans[l] * chans[l]) * (hw >> l) ** 2
    flops += 2.0 * chans[0] * hw * hw
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < seconds_target:
            unet.forward(params, x, len(chans), chans)
            reps += 1
        dt = time.perf_counter() - t0
    return {"value": flops * reps / dt / 1e12, "unit": "TFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{reps} forwards of one {hw}x{hw} patch (float64 NumPy U-Net oracle, 1 thread)"}


def copy_ceiling(torch, lbch, stream, nbytes=1 << 30, reps=300):
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


def time_to_t(stream, n, steps, warm, K, NC, inner, chunk, net=None, cond=(), note=None, extrapolate=1,
              plain_until=0):
    """Wall time to advance the 8192^2-recipe FP32 spinodal run (alpha 0.2, seed 5; side n)
    by `steps` steps after `warm` untimed plain steps, twice on the same GPU: with the plain
    scheme, and with the jump + correction + rejection schedule (jumps of K steps, NC correction
    steps, inner projective cycles `inner`; extrapolate = 1: rate-extrapolated jumps, plus the
    network's residual when `net` is given; extrapolate = 0: the network's own jump).  The free energy of both runs is sampled every `chunk` steps (rounded
    to whole cycles); the hybrid's cycles are counted per chunk so that rejections can be told
    apart by phase (spinodal growth, coarsening).  plain_until: the hybrid run advances
    plainly (timed) up to that step before its first jump."""
    import torch

    from paper_2501_03759_amd import inputs, lbch

    note = note or (lambda m: None)
    d = inputs.C5
    p = lbch.default_params(nx=n, ny=n, precision=lbch.FP32,
                            sigma_width=(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"])),
                            mobility=d["mobility"], alpha=d["alpha"], aniso_m=d["m"], eps_reg=d["eps_reg"])
    cyc = K + NC
    chunk = max(cyc, chunk // cyc * cyc)
    with torch.cuda.stream(stream):
        phi0 = inputs.spinodal(n, n, seed=d["seed"], amp=d["amp"])
        plain = lbch.Sim(p, stream)
        plain.init(phi0)
        for k in range(0, warm, 20000):
            plain.step(min(20000, warm - k))
            plain.synchronize()
            note(f"warm-up: step {plain.nstep}")
        hyb = lbch.Sim(p, stream)
        if warm:
            blob = plain.save_state()
            hyb.load_state(blob)
            del blob
        else:
            hyb.init(phi0)
        del phi0

        def run(advance):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done = 0
            while done < steps:
                k = min(chunk, steps - done)
                done += advance(k) or k
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        e_plain, e_hyb = [plain.free_energy()[0]], [hyb.free_energy()[0]]
        o = lbch.hybrid_opts(jump=K, correct_steps=NC, windows=4, window_interior=192, window_margin=64,
                             tol_window=1e-2, tol_energy=0.0, check_every=4, extrapolate=extrapolate,
                             cond=list(cond), inner_steps=inner[0], inner_jump=inner[1])
        totals, phases = {}, []

        def adv_plain(k):
            plain.step(k)
            e_plain.append(plain.free_energy()[0])
            note(f"plain: step {plain.nstep}, E = {e_plain[-1]:.6f}")

        def adv_hyb(k):
            st_ = lbch.hybrid_advance(hyb, net, o, k)
            for f, _ in st_._fields_:
                v = getattr(st_, f)
                if f == "max_window_err":
                    totals[f] = max(totals.get(f, 0.0), v)
                elif f != "last_energy":
                    totals[f] = totals.get(f, 0) + v
            phases.append([int(hyb.nstep), int(st_.cycles), int(st_.accepted), int(st_.rejected_energy),
                           int(st_.rejected_window)])
            e_hyb.append(hyb.free_energy()[0])
            note(f"hybrid: step {hyb.nstep}, E = {e_hyb[-1]:.6f}, accepted {st_.accepted}/{st_.cycles}")

        def adv_mixed(k):
            # plain steps up to plain_until, then the schedule (chunks never straddle it)
            if hyb.nstep - warm < plain_until:
                k = min(k, plain_until - (hyb.nstep - warm))
                hyb.step(k)
                e_hyb.append(hyb.free_energy()[0])
                note(f"hybrid (plain prefix): step {hyb.nstep}, E = {e_hyb[-1]:.6f}")
                return k
            adv_hyb(k)
            return k

        t_plain = run(adv_plain)
        t_hyb = run(adv_mixed)
        pa, ph = plain.phi(), hyb.phi()
        plain.close()
        hyb.close()
    rel = float(np.linalg.norm(ph - pa) / np.linalg.norm(pa))
    return {
        "workload": f"spinodal-{n}x{n}-fp32", "from_step": warm, "steps": steps, "plain_prefix": plain_until,
        "plain_s": round(t_plain, 3), "hybrid_s": round(t_hyb, 3), "speedup": round(t_plain / t_hyb, 3),
        "rel_l2": rel, "rel_l2_ok": rel <= 1e-2,
        "energy_nonincreasing": {"plain": bool(np.all(np.diff(e_plain) <= 0)),
                                 "hybrid": bool(np.all(np.diff(e_hyb) <= 0)), "samples": len(e_hyb)},
        "energy_final": {"plain": e_plain[-1], "hybrid": e_hyb[-1]},
        "jump_form": ("rate extrapolation" + (" + network residual" if net is not None else "")) if extrapolate
                     else "network",
        "jump": K, "correct_steps": NC, "inner_steps": inner[0], "inner_jump": inner[1], "windows": 4,
        "check_every": 4, "tol_energy": 0.0, "tol_window": 1e-2,
        "cycles": int(totals.get("cycles", 0)), "accepted": int(totals.get("accepted", 0)),
        "rejected_energy": int(totals.get("rejected_energy", 0)),
        "rejected_window": int(totals.get("rejected_window", 0)),
        "max_window_err": totals.get("max_window_err", 0.0),
        "ms_split": {k: round(totals.get(k, 0.0), 1) for k in ("ms_surrogate", "ms_correct", "ms_checks", "ms_plain")},
        "per_chunk": {"columns": ["end_step", "cycles", "accepted", "rejected_energy", "rejected_window"],
                      "rows": phases},
    }


def hybrid_workload(args):
    """Time-to-t of the jump + correction schedule against the plain scheme on the same GPU
    (the 8192^2 FP32 spinodal run, alpha 0.2): --hybrid-warm untimed plain steps, then
    --hybrid-steps steps timed twice (see time_to_t), optionally with a trained network's
    residual added to the rate-extrapolated jump (--surrogate)."""
    import torch

    from paper_2501_03759_amd import inputs

    d = inputs.C5
    n = args.n
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    K, NC = args.hybrid_jump, args.hybrid_correct
    net, cond = None, []
    train_s = 0.0

    def note(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.surrogate:
        from paper_2501_03759_amd import lbsg, surrogate_train as st
        with torch.cuda.stream(stream):
            t0 = time.time()
            runs = st.draw_runs(64, seed=1)
            X, Y = st.generate(runs, 256, 60000, 300000, 4000, K, 256, 1, seed=7, stream=stream, log=note,
                               extrapolate=True)
            tr = lbsg.Surrogate((32, 32), 1 + st.N_COND, 16, 256, 256, train=True, seed=0, stream=stream,
                                out_scale=0.02)
            st.train(tr, X, Y, epochs=8, batch=16, lr=1e-3, margin=0, log=lambda m: None)
            w = tr.get_params()
            tr.close()
            del X, Y
            torch.cuda.empty_cache()
            net = lbsg.Surrogate((32, 32), 1 + st.N_COND, 1, n, n, train=False, seed=0, stream=stream,
                                 out_scale=0.02)
            net.set_params(w)
            cond = list(st.conditioning(d["alpha"], d["m"], 0.0))
            train_s = time.time() - t0
    inner = [int(v) for v in args.hybrid_inner.split(",")]
    r = time_to_t(stream, n, args.hybrid_steps, args.hybrid_warm, K, args.hybrid_correct, inner,
                  args.hybrid_chunk, net=net, cond=cond, note=note)
    out = {
        "metric": "time-to-t speedup of the jump + correction schedule over the plain scheme (1 GPU)",
        "value": r["speedup"], "unit": "x", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32", "data": "synthetic (seeded spinodal noise U(-0.05,0.05), seed 5)",
        "config": {"workload": f"spinodal-{n}x{n}-fp32-time-to-t", "warm_steps": args.hybrid_warm,
                   "timed_steps": args.hybrid_steps, "jump": K, "correct_steps": NC, "windows": 4,
                   "check_every": 4, "jump_form": r["jump_form"], "inner_steps": inner[0], "inner_jump": inner[1]},
        "time_to_t": r, "surrogate_train_s": round(train_s, 1),
    }
    print(json.dumps(out), flush=True)


def learned_workload(args):
    """The learned surrogate at its stated configuration: the 5-level periodic U-Net (32, 64, 128,
    256, 256 channels; phi plus alpha, cos / sin(m theta0), m / 6 planes; BF16 storage, FP32
    accumulation) trained on the GPU by the library's kernels to predict phi(t + 200) on 256^2
    crops of 1024^2 FP32 spinodal runs (one ensemble of --c4-runs runs, snapshots every 1000
    steps up to 50000, 8 crops each; alpha ~ U[0, 0.3], m in {4, 6}, theta0 ~ U[0, 2 pi)), then
    measured on held-out runs (other seeds) against the plain scheme, beside the jump without the
    network and the rate-extrapolated jump.  Reports the 8192^2 inference time and, with
    --c4-hybrid, the time-to-t of the schedule whose jump is the network's."""
    import torch

    from paper_2501_03759_amd import inputs, lbsg, surrogate_train as st

    def note(msg):
        print(msg, file=sys.stderr, flush=True)

    chans, K, crop, margin = (32, 64, 128, 256, 256), 200, 256, 32
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    out = {"metric": "surrogate held-out relative L2 of phi(t + 200) (1 GPU)", "unit": "rel-L2", "n_gpus": 1,
           "higher_is_better": False, "dtype": "bf16", "data": "synthetic (seeded 1024^2 spinodal runs)",
           "config": {"workload": "unet5-32-256-c4", "chans": list(chans), "jump": K, "crop": crop,
                      "loss_margin": margin, "runs": args.c4_runs, "heldout_runs": 6, "epochs": args.c4_epochs}}
    with torch.cuda.stream(stream):
        t0 = time.time()
        if args.c4_weights:
            w = np.load(args.c4_weights)
            hist = []
        else:
            runs = st.draw_runs(args.c4_runs, seed=1)
            X, Y = st.generate(runs, 1024, 1000, 50000, 1000, K, crop, 8, seed=7, stream=stream, log=note)
            out["config"]["pairs"] = int(X.shape[0])
            net = lbsg.Surrogate(chans, 1 + st.N_COND, 16, crop, crop, train=True, seed=0, stream=stream,
                                 out_scale=0.02)
            t1 = time.time()
            hist = st.train(net, X, Y, epochs=args.c4_epochs, batch=16, lr=args.c4_lr, margin=margin, log=note)
            torch.cuda.synchronize()
            out["train_s"] = round(time.time() - t1, 1)
            w = net.get_params()
            net.close()
            del X, Y
            torch.cuda.empty_cache()
            if args.c4_save:
                np.save(args.c4_save, w)
        out["loss_history"] = [float(v) for v in hist]
        held = st.draw_runs(6, seed=2)
        Xh, Yh, Rh, Th = st.generate(held, 1024, 1000, 50000, 7000, K, crop, 8, seed=8, stream=stream, log=note,
                                     with_rate=True)
        ev = lbsg.Surrogate(chans, 1 + st.N_COND, 8, crop, crop, train=False, seed=0, stream=stream, out_scale=0.02)
        ev.set_params(w)
        out["heldout"] = st.evaluate_jumps(ev, Xh, Yh, Rh, K, Th, split=10000, margin=margin)
        ev.close()
        del Xh, Yh, Rh
        torch.cuda.empty_cache()
        out["value"] = round(out["heldout"]["all"]["network"], 6)
        # inference on the whole 8192^2 periodic field (the hybrid's jump)
        n = args.n
        inf = lbsg.Surrogate(chans, 1 + st.N_COND, 1, n, n, train=False, seed=0, stream=stream, out_scale=0.02)
        inf.set_params(w)
        phi = torch.empty((n, n), dtype=torch.float32, device="cuda").uniform_(-1, 1)
        o = torch.empty_like(phi)
        cond = list(st.conditioning(inputs.C5["alpha"], inputs.C5["m"], 0.0))
        for _ in range(2):
            inf.predict(phi.data_ptr(), cond, n, n, o.data_ptr())
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(5):
            inf.predict(phi.data_ptr(), cond, n, n, o.data_ptr())
        e.record(stream)
        e.synchronize()
        out["inference_ms_8192"] = round(a.elapsed_time(e) / 5, 2)
        del phi, o
        if args.c4_hybrid:
            inner = [int(v) for v in args.c4_hybrid_inner.split(",")]
            out["time_to_t"] = time_to_t(stream, n, args.time_to_t_steps, args.hybrid_warm, K, args.c4_correct,
                                         inner, args.hybrid_chunk, net=inf, cond=cond, note=note,
                                         extrapolate=0, plain_until=args.time_to_t_plain)
        inf.close()
    out["wall_s"] = round(time.time() - t0, 1)
    print(json.dumps(out), flush=True)


def droplet_workload(args):
    """The droplet workload in FP64 (64 x 64 periodic, centred tanh disc of radius 16 with
    eps_w = 2, alpha = 0.05, m = 4, tau_phi = 1, Willmore 0.03; 2000 steps): MLUPS of the HIP
    path (one launch per step at this size; launch-bound), the oracle timed on the same
    workload on one host core, and the two results compared node by node."""
    import torch

    from oracle import lbm
    from paper_2501_03759_amd import inputs, lbch

    d = inputs.C1
    n, steps = d["n"], d["steps"]
    p = lbch.default_params(nx=n, ny=n, precision=lbch.FP64,
                            sigma_width=(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"])),
                            mobility=d["mobility"], alpha=d["alpha"], aniso_m=d["m"], eps_reg=d["eps_reg"])
    phi0 = inputs.droplet(n, n, d["radius"], d["eps_w"])
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    sim = lbch.Sim(p, stream)
    sim.init(phi0)
    sim.step(args.warmup)
    sim.init(phi0)
    sim.synchronize()
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    sim.step(steps)
    e.record(stream)
    e.synchronize()
    ms = a.elapsed_time(e)
    got = sim.phi()
    sim.close()
    out = {"metric": "MLUPS, droplet 64^2 FP64 (1 GPU)", "value": round(n * n * steps / (ms * 1e-3) / 1e6, 2),
           "unit": "MLUPS", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
           "ms_per_step": round(ms / steps, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic (centred tanh droplet, deterministic)",
           "config": {"workload": "droplet-64x64-fp64", "alpha": d["alpha"], "m": d["m"], "steps": steps}}
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        kappa, beta = lbm.kappa_beta_from_sigma_width(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"]))
        op = lbm.Params(nx=n, ny=n, kappa=kappa, beta=beta, mobility=d["mobility"], alpha=d["alpha"],
                        aniso_m=d["m"], eps_reg=d["eps_reg"])
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            want = lbm.phi_of(lbm.run(phi0, op, steps))
            dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n * n * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
                               "sample": f"the whole workload ({steps} steps of {n}x{n}; FP64 NumPy oracle, 1 thread)",
                               "host": host_info()}
        out["max_abs_dphi_vs_oracle"] = float(np.abs(got - want).max())
    print(json.dumps(out), flush=True)


def c2_workload(args):
    """The 1024^2 FP32 spinodal workload (phi0 = U(-0.05, 0.05) from seed 0, eps_w = 1.5,
    alpha = 0.3, m = 4, Willmore 0.03, M = 0.1): 50 000 steps with phi and the free energy
    checkpointed every 1000 steps (phi copied to the host).  Reports MLUPS over the whole
    run, checkpoints included, the energy series' monotonicity and the growth of phi's rms.
    The 75 MB working set fits the GPU's 256 MB last-level cache: an on-chip figure, not an
    HBM one."""
    import torch

    from paper_2501_03759_amd import inputs, lbch

    d = inputs.C2
    n, steps, every = d["n"], d["steps"], 1000
    p = lbch.default_params(nx=n, ny=n, precision=lbch.FP32,
                            sigma_width=(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"])),
                            mobility=d["mobility"], alpha=d["alpha"], aniso_m=d["m"], eps_reg=d["eps_reg"])
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    sim = lbch.Sim(p, stream)
    sim.init(inputs.spinodal(n, n, seed=d["seed"], amp=d["amp"]))
    sim.step(args.warmup)
    sim.init(inputs.spinodal(n, n, seed=d["seed"], amp=d["amp"]))
    sim.synchronize()
    energy, rms = [sim.free_energy()[0]], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(0, steps, every):
        sim.step(every)
        phi, mass, lo, hi = sim.moments()
        energy.append(sim.free_energy()[0])
        rms.append(float(np.sqrt(np.mean(phi * phi))))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.close()
    out = {"metric": "MLUPS, 1024^2 spinodal with checkpoints every 1000 steps (1 GPU)",
           "value": round(n * n * steps / wall / 1e6, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": round(wall * 1e3 / steps, 5), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded spinodal noise U(-0.05,0.05), seed 0)",
           "config": {"workload": "spinodal-1024x1024-fp32-checkpointed", "alpha": d["alpha"], "m": d["m"],
                      "checkpoint_every": every, "residency": "last-level cache (75 MB working set)"},
           "energy_nonincreasing": bool(np.all(np.diff(energy) <= 0)),
           "energy": {"start": energy[0], "end": energy[-1], "samples": len(energy)},
           "phi_rms": {"after_10k": rms[9], "after_25k": rms[24], "after_50k": rms[-1]}}
    print(json.dumps(out), flush=True)


def ensemble_workload(args):
    """Throughput of the ragged ensemble: 512 periodic members (side log-uniform in [64, 512],
    alpha ~ U[0, 0.3], m in {4, 6}, spinodal / droplet 50/50, seed 3), FP32, advanced by one
    persistent launch per two steps (graphs of 16 launches), launch shape from the autotuner."""
    import torch

    from paper_2501_03759_amd import inputs, lbch

    mems = inputs.ensemble_members(512, seed=3)
    params = [lbch.default_params(nx=m["side"], ny=m["side"], precision=lbch.FP32,
                                  sigma_width=(inputs.SIGMA_PAPER, inputs.width_from_eps(1.5)), mobility=0.1,
                                  alpha=m["alpha"], aniso_m=m["m"], eps_reg=0.03) for m in mems]
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    b = lbch.Batch(params, stream)
    for k, m in enumerate(mems):
        b.init(k, inputs.member_phi0(m))
    if args.tiling:                                  # block_threads,rows_per_block[,depth]: a fixed shape
        v = [int(x) for x in args.tiling.split(",")]
        b.set_time_blocking(v[2] if len(v) > 2 else 2)
        b.set_tiling(v[0], v[1])
        nt, hc = v[0], v[1]
    else:
        nt, hc, _ = b.autotune(3)
    depth = b.time_blocking()
    nodes = b.nodes
    b.step(args.warmup)
    b.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    b.step(args.steps)
    end.record(stream)
    end.synchronize()
    ms_step = start.elapsed_time(end) / args.steps
    b.close()
    copy = copy_ceiling(torch, lbch, stream)
    launch_ms = ms_step * depth
    alg = 72 * nodes * depth
    traffic = measured_traffic(nodes, "fp32", depth,
                               path=os.path.join(ROOT, "profiles", "batch_step_ensemble512_fp32.json"),
                               tiling=(nt, hc))
    achieved = alg / (launch_ms * 1e-3) / 1e9
    out = {
        "metric": "MLUPS, 512-member ragged ensemble (1 GPU)", "value": round(nodes / (ms_step * 1e-3) / 1e6, 1),
        "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded ragged spinodal / droplet members, seed 3)",
        "config": {"workload": "ensemble-512-ragged-fp32", "members": len(mems), "nodes": nodes,
                   "time_steps_per_launch": depth, "tiling": [nt, hc]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "batch_step",
                     "launch_ms": round(launch_ms, 4), "bytes_per_update": 72,
                     "min_bytes_GBs": round(72 * nodes / (launch_ms * 1e-3) / 1e9, 1)},
        "hbm_copy": copy,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_ensemble(mems)
    print(json.dumps(out), flush=True)


def step3d_workload(args):
    """Throughput of the D3Q15 step (eq 21): a periodic n^3 box (default 256^3) of spinodal noise
    U(-0.05, 0.05) from seed 5 with the parameters of the two-dimensional workload (alpha = 0.2,
    Willmore eps = 0.03, M = 0.1, D = 2 sqrt(2) 1.5, sigma = 0.01), one launch per step, tile
    shape and z-sweep length from the autotuner unless --tiling is given.
    Algorithmic bytes per update: 15 populations read + 15 written."""
    import torch

    from paper_2501_03759_amd import inputs, lbch

    d = inputs.C5
    n = args.n3
    prec = lbch.FP32 if args.precision == "fp32" else lbch.FP64
    esize = 4 if prec == lbch.FP32 else 8
    p = lbch.default_params(nx=n, ny=n, nz=n, lattice=lbch.D3Q15, precision=prec,
                            sigma_width=(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"])),
                            mobility=d["mobility"], alpha=d["alpha"], eps_reg=d["eps_reg"])
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    copy = copy_ceiling(torch, lbch, stream)
    sim = lbch.Sim(p, stream)
    if args.tiling:
        sim.set_tiling(*(int(v) for v in args.tiling.split(",")))
    phi0 = inputs.spinodal3(n, n, n, seed=d["seed"], amp=d["amp"])
    sim.init(phi0)
    del phi0
    tuned = None
    if not args.tiling:
        # tile shape and z-sweep length from the library's autotuner (trials on the live state,
        # which they leave untouched)
        t_at = time.perf_counter()
        bt_, hz_, ms_ = sim.autotune(args.autotune_steps)
        tuned = {"block_threads": bt_, "z_slabs": hz_, "ms_per_step": round(ms_, 4),
                 "launches_per_trial": args.autotune_steps, "seconds": round(time.perf_counter() - t_at, 2)}
    sim.step(args.warmup)
    sim.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(args.steps)
    end.record(stream)
    end.synchronize()
    ms_step = start.elapsed_time(end) / args.steps
    _, mass, lo, hi = sim.moments(want_phi=False)
    tiling = sim.tiling()
    sim.close()
    nodes = n ** 3
    bytes_per_update = 30 * esize
    achieved = bytes_per_update * nodes / (ms_step * 1e-3) / 1e9
    out = {
        "metric": "MLUPS & % HBM peak, D3Q15 (1 GPU)", "value": round(nodes / (ms_step * 1e-3) / 1e6, 1),
        "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if prec == lbch.FP32 else "f64",
        "data": "synthetic (seeded spinodal noise U(-0.05,0.05), seed 5)",
        "config": {"workload": f"spinodal-{n}^3-d3q15-{args.precision}", "grid": [n, n, n], "lattice": "D3Q15",
                   "alpha": d["alpha"], "regularization": "willmore", "eps_reg": d["eps_reg"],
                   "mobility": d["mobility"], "time_steps_per_launch": 1, "tiling": list(tiling),
                   "autotuned": tuned},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(nodes, args.precision, 1, "d3q15", tiling=tiling),
                     "kernel": "step3_fused",
                     "launch_ms": round(ms_step, 4), "updates_per_launch": nodes,
                     "bytes_per_update": bytes_per_update},
        "checks": {"mass": mass, "phi_min": lo, "phi_max": hi},
        "hbm_copy": copy,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_3d()
    print(json.dumps(out), flush=True)


def surrogate_workload(args):
    """Throughput of the surrogate network's forward and training step on 16 periodic 256 x 256
    patches: the 5-level U-Net (32, 64, 128, 256, 256 channels), inputs phi plus 4 conditioning
    planes, BF16 MFMA with FP32 accumulation.  FLOPs are the network's own 3x3 and 1x1
    convolutions (2 per multiply-add, real input channels); a training step counts 3x forward.
    Also times inference on one whole --n x --n field (the hybrid's jump, default 8192^2)."""
    import torch

    from paper_2501_03759_amd import lbsg

    chans, c_in, B, hw = (32, 64, 128, 256, 256), 5, 16, 256
    flops = 0.0
    prev = c_in
    for l, c in enumerate(chans):
        flops += 18.0 * (prev * c + c * c) * (hw >> l) ** 2
        prev = c
    for l in range(len(chans) - 2, -1, -1):
        flops += 18.0 * ((chans[l + 1] + chans[l]) * chans[l] + chans[l] * chans[l]) * (hw >> l) ** 2
    flops = (flops + 2.0 * chans[0] * hw * hw) * B
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn((B, hw, hw, c_in), device="cuda", generator=g)
    t = torch.randn((B, hw, hw), device="cuda", generator=g)
    out = torch.empty((B, hw, hw), device="cuda")
    net = lbsg.Surrogate(chans, c_in, B, hw, hw, train=True, seed=0, stream=stream, out_scale=0.02)
    torch.cuda.synchronize()
    res = {}
    for what, fn, mult in [("forward", lambda: net.forward(x.data_ptr(), B, hw, hw, out.data_ptr()), 1.0),
                           ("train_step", lambda: net.train_step(x.data_ptr(), t.data_ptr(), B, hw, hw, 0, 1e-4,
                                                                 want_loss=False), 3.0)]:
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        e.record(stream)
        e.synchronize()
        ms = a.elapsed_time(e) / args.steps
        res[what] = (ms, mult * flops / (ms * 1e-3) / 1e12)
    net.close()
    # inference on one whole n x n periodic field (the hybrid's jump; weights do not change the time)
    n = args.n
    inf_flops = 0.0
    prev = c_in
    for l, c in enumerate(chans):
        inf_flops += 18.0 * (prev * c + c * c) * (n >> l) ** 2
        prev = c
    for l in range(len(chans) - 2, -1, -1):
        inf_flops += 18.0 * ((chans[l + 1] + chans[l]) * chans[l] + chans[l] * chans[l]) * (n >> l) ** 2
    inf_flops += 2.0 * chans[0] * n * n
    inf = lbsg.Surrogate(chans, c_in, 1, n, n, train=False, seed=0, stream=stream, out_scale=0.02)
    phi = torch.empty((n, n), dtype=torch.float32, device="cuda").uniform_(-1, 1, generator=g)
    o = torch.empty_like(phi)
    cond = [0.2, 1.0, 0.0, 4.0 / 6.0][: c_in - 1]
    for _ in range(2):
        inf.predict(phi.data_ptr(), cond, n, n, o.data_ptr())
    a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(5):
        inf.predict(phi.data_ptr(), cond, n, n, o.data_ptr())
    e.record(stream)
    e.synchronize()
    inf_ms = a.elapsed_time(e) / 5
    inf.close()
    del phi, o
    fwd_ms, fwd_tf = res["forward"]
    out_line = {
        "metric": "surrogate forward TFLOP/s, 16 x 256^2 patches (1 GPU)", "value": round(fwd_tf, 1),
        "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(fwd_ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded normal inputs)",
        "config": {"workload": "unet5-32-256-b16x256x256", "chans": list(chans), "in_ch": c_in,
                   "flop_per_forward": flops},
        "roofline": {"bound": "mfma", "achieved": round(fwd_tf, 1), "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": round(fwd_tf / 2500.0, 4), "traffic": None, "kernel": "conv3_fwd_k (all layers)"},
        "train_step": {"ms": round(res["train_step"][0], 3), "TFLOP/s": round(res["train_step"][1], 1)},
        "inference": {"field": [n, n], "ms": round(inf_ms, 2), "TFLOP/s": round(inf_flops / (inf_ms * 1e-3) / 1e12, 1)},
    }
    if not args.no_cpu_baseline:
        out_line["cpu_baseline"] = cpu_baseline_unet(chans, c_in)
    print(json.dumps(out_line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=8192, help="grid side (default: the 8192^2 workload)")
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--depth", type=int, default=0, choices=[0, 1, 2],
                    help="time steps per kernel launch (0: the autotuner's choice with its launch shape)")
    ap.add_argument("--autotune-steps", type=int, default=40, help="launches per autotuner trial (default line)")
    ap.add_argument("--tiling", type=str, default="", help="block_threads,rows_per_block (ensemble: [,depth], a fixed shape instead of the autotuner)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n3", type=int, default=256, help="box side of the D3Q15 workload")
    ap.add_argument("--workload", choices=["step", "step3d", "hybrid", "ensemble", "surrogate", "learned", "droplet",
                                           "c2"],
                    default="step",
                    help="step: throughput of lbch_step (the default line); hybrid: time-to-t of the jump "
                         "schedule; ensemble: the 512-member batch; surrogate: the network's MFMA throughput; "
                         "learned: the 5-level network trained and measured on held-out runs; droplet: the "
                         "64^2 FP64 droplet against the oracle; c2: the 1024^2 run with checkpoints")
    ap.add_argument("--hybrid-warm", type=int, default=80000)
    ap.add_argument("--hybrid-steps", type=int, default=200000)
    ap.add_argument("--hybrid-jump", type=int, default=400)
    ap.add_argument("--hybrid-correct", type=int, default=128)
    ap.add_argument("--hybrid-chunk", type=int, default=10000)
    ap.add_argument("--hybrid-inner", type=str, default="4,16",
                    help="inner_steps,inner_jump: projective steps of the populations inside the correction phase")
    ap.add_argument("--surrogate", action="store_true", help="hybrid: add the trained network's residual")
    ap.add_argument("--c4-runs", type=int, default=50, help="learned: training runs (50 x 50 snapshots x 8 crops)")
    ap.add_argument("--c4-epochs", type=int, default=40)
    ap.add_argument("--c4-lr", type=float, default=1e-3)
    ap.add_argument("--c4-save", type=str, default="", help="learned: write the trained parameters (.npy)")
    ap.add_argument("--c4-weights", type=str, default="", help="learned: load parameters instead of training")
    ap.add_argument("--c4-hybrid", action="store_true", help="learned: also the time-to-t with the network's jump")
    ap.add_argument("--c4-correct", type=int, default=10, help="learned hybrid: correction steps per jump")
    ap.add_argument("--c4-hybrid-inner", type=str, default="0,0")
    ap.add_argument("--time-to-t-plain", type=int, default=15000,
                    help="default line: plain steps of the hybrid run before its first jump (the spinodal "
                         "growth amplifies early jump errors)")
    ap.add_argument("--time-to-t-steps", type=int, default=200000,
                    help="default line: steps of the plain / hybrid time-to-t comparison from the initial field "
                         "(0 = skip)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "hybrid":
        hybrid_workload(args)
        return
    if args.workload == "ensemble":
        ensemble_workload(args)
        return
    if args.workload == "surrogate":
        surrogate_workload(args)
        return
    if args.workload == "learned":
        learned_workload(args)
        return
    if args.workload == "droplet":
        droplet_workload(args)
        return
    if args.workload == "c2":
        c2_workload(args)
        return
    if args.workload == "step3d":
        step3d_workload(args)
        return

    # the oracle's CPU figure first: its worker processes are forked before the GPU is touched
    cpu = None if args.no_cpu_baseline else cpu_baseline()

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
    sim = lbch.Sim(p, stream)
    if args.depth:
        sim.set_time_blocking(args.depth)
    if args.tiling:
        bt, rows = (int(v) for v in args.tiling.split(","))
        sim.set_tiling(bt, rows)
    phi0 = inputs.spinodal(n, n, seed=d["seed"], amp=d["amp"])
    sim.init(phi0)
    del phi0
    copy = copy_ceiling(torch, lbch, stream)
    tuned = None
    if not args.depth and not args.tiling:
        # launch shape (steps per launch, lanes, rows per workgroup) from the library's autotuner,
        # which times every candidate for --autotune-steps launches on the live state without
        # changing it.  Long trials also leave the GPU in the power state the step kernel runs
        # in: after a pause the first ~20 launches of the step kernel run up to 40 % slower
        # (kernel trace in the committed profile)
        t_at = time.perf_counter()
        nt_, hc_, ms_ = sim.autotune(args.autotune_steps)
        tuned = {"block_threads": nt_, "rows_per_block": hc_, "ms_per_step": round(ms_, 4),
                 "launches_per_trial": args.autotune_steps, "seconds": round(time.perf_counter() - t_at, 2)}
    depth = sim.time_blocking()
    sim.step(args.warmup)
    sim.synchronize()

    # the K timed steps, in up to five windows of whole launches (HIP events on the step's
    # stream between them); value and roofline come from the whole region
    nwin = 5 if args.steps >= 5 * depth else 1
    sizes = [args.steps // nwin // depth * depth] * nwin
    sizes[-1] += args.steps - sum(sizes)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nwin + 1)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev[0].record(stream)
    for w in range(nwin):
        sim.step(sizes[w])
        ev[w + 1].record(stream)
    ev[-1].synchronize()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t_wall) * 1e3
    ms_total = ev[0].elapsed_time(ev[-1])
    ms_step = ms_total / args.steps
    win_ms = [ev[w].elapsed_time(ev[w + 1]) / sizes[w] for w in range(nwin)]
    _, mass, lo, hi = sim.moments(want_phi=False)
    tiling = sim.tiling()
    sim.close()

    nodes = n * n
    mlups = nodes * args.steps / (ms_total * 1e-3) / 1e6
    # every launch advances `depth` steps (an odd tail step, if any, is one
    # single-step launch of about half the time: the average below counts it
    # as half a launch)
    launch_ms = ms_step * depth
    bytes_per_update = 18 * esize                      # 9 populations read + 9 written
    alg_bytes = bytes_per_update * nodes * depth       # per launch
    min_bytes = bytes_per_update * nodes               # one read + one write of the state per launch
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(nodes, args.precision, depth)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "basis": f"algorithmic: {bytes_per_update} B per lattice update x {depth} updates per node per "
                         "launch (effective bandwidth; a launch moves the state once per launch)",
                "kernel": "step2_fused" if depth == 2 else "step_fused",
                "launch_ms": round(launch_ms, 4), "updates_per_launch": depth * nodes,
                "bytes_per_update": bytes_per_update, "algorithmic_bytes_per_launch": alg_bytes,
                "min_bytes_per_launch": min_bytes,
                "min_bytes_GBs": round(min_bytes / (launch_ms * 1e-3) / 1e9, 1),
                "min_bytes_frac": round(min_bytes / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if traffic:
        # the HBM bytes the counters saw per launch, over this run's launch time
        roofline["traffic_GBs"] = round(traffic / (launch_ms * 1e-3) / 1e9, 1)
        roofline["traffic_frac"] = round(traffic / (launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    med = float(np.median(win_ms))
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
                   "mobility": d["mobility"], "time_steps_per_launch": depth, "tiling": list(tiling),
                   "autotuned": tuned},
        "roofline": roofline,
        "windows": {"count": nwin, "steps": sizes, "ms_per_step": [round(v, 4) for v in win_ms],
                    "median_ms_per_step": round(med, 4), "median_MLUPS": round(nodes / (med * 1e-3) / 1e6, 1),
                    "spread": round((max(win_ms) - min(win_ms)) / med, 4), "wall_ms": round(wall_ms, 3)},
        "checks": {"mass": mass, "phi_min": lo, "phi_max": hi},
        "hbm_copy": copy,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if args.time_to_t_steps > 0 and args.precision == "fp32":
        # the second half of the metric: time to the workload's final step, plain against the
        # jump + correction schedule, both from the initial field
        def note(msg):
            print(msg, file=sys.stderr, flush=True)
        try:
            out["time_to_t"] = time_to_t(stream, n, args.time_to_t_steps, 0, args.hybrid_jump, args.hybrid_correct,
                                         [int(v) for v in args.hybrid_inner.split(",")], args.hybrid_chunk,
                                         note=note, plain_until=args.time_to_t_plain)
        except Exception as exc:                  # the throughput line stands on its own
            out["time_to_t"] = {"error": f"{type(exc).__name__}: {exc}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
