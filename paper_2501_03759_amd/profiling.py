"""Turns rocprofv3 output of bench.py runs into the committed summaries under profiles/.

Usage (after the three profiled runs named in the summary header):
    python -m paper_2501_03759_amd.profiling --trace DIR --fetch DIR --write DIR \
        --nodes N --precision fp32 --command "..." --out profiles/<name>

FETCH_SIZE / WRITE_SIZE are read per dispatch (KiB) and scaled by what the
same counter reads for the library's plain copy kernel, which moves a known
number of bytes in the same process (read = write = its buffer size).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_2501_03759_amd", "csrc", "lbch_kernels.hip")
KERNEL_SRC_3D = os.path.join(ROOT, "paper_2501_03759_amd", "csrc", "lbch3_kernels.hip")
STEP_KERNELS = {1: "step_fused", 2: "step2_fused"}   # by time steps per launch
STEP_KERNEL_3D = "step3_fused"
COPY_KERNEL = "copy16_k"
COPY_BYTES = 1 << 30          # bench.py's copy_ceiling buffer


def kernel_hash(lattice: str = "d2q9") -> str:
    src = KERNEL_SRC_3D if lattice == "d3q15" else KERNEL_SRC
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def _one(pattern):
    files = glob.glob(pattern, recursive=True)
    if not files:
        raise FileNotFoundError(pattern)
    return files[0]


def counter_values(d, counter, kernel_substr):
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    vals = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and kernel_substr in r["Kernel_Name"]:
            vals.append((int(r.get("Dispatch_Id") or 0), float(r["Counter_Value"])))
    vals = [v for _, v in sorted(vals, key=lambda dv: dv[0])]       # dispatch order
    return vals


def last_dispatches(d, kernel_substr, last):
    """Name and durations (ns) of the last `last` dispatches of a kernel, from the run's kernel trace."""
    path = _one(os.path.join(d, "**", "*kernel_trace.csv"))
    rows = [r for r in csv.DictReader(open(path)) if kernel_substr in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    rows = rows[-last:]
    names = {r["Kernel_Name"] for r in rows}
    if len(names) != 1:
        raise ValueError(f"the last {last} dispatches of {kernel_substr} are not one kernel: {sorted(names)}")
    return names.pop()[:120], [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows]


def kernel_stats(d):
    path = _one(os.path.join(d, "**", "*kernel_stats.csv"))
    out = []
    for r in csv.DictReader(open(path)):
        out.append({"name": r["Name"][:120], "calls": int(r["Calls"]), "avg_ns": float(r["AverageNs"]),
                    "pct": float(r["Percentage"])})
    return out


def stats_only(args):
    """Kernel statistics of one traced run, as a short Markdown table."""
    stats = kernel_stats(args.trace)
    lines = [f"# rocprofv3 summary: {args.title}", "", "Command:", ""]
    lines += ["    " + c for c in args.command.split(";;")]
    lines += ["", "Kernel statistics (--kernel-trace --stats):", "",
              "| kernel | calls | avg ms | % time |", "|---|---|---|---|"]
    for st in stats[:12]:
        lines.append(f"| {st['name'][:100]} | {st['calls']} | {st['avg_ns'] / 1e6:.4f} | {st['pct']:.1f} |")
    with open(args.out + ".md", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def shader_counters(dirs, kernel_substr, last=0):
    """Mean per dispatch of every counter collected in the given --pmc runs for the kernel
    (its last `last` dispatches when given)."""
    out = {}
    for d in dirs:
        path = _one(os.path.join(d, "**", "*counter_collection.csv"))
        per = {}
        for r in csv.DictReader(open(path)):
            if kernel_substr in r["Kernel_Name"]:
                per.setdefault(r["Counter_Name"], []).append((int(r.get("Dispatch_Id") or 0),
                                                             float(r["Counter_Value"])))
        for name, vals in per.items():
            vals = [v for _, v in sorted(vals)]
            if last:
                vals = vals[-last:]
            out[name] = statistics.mean(vals)
    return out


def shader_lines(c):
    """Markdown lines of the shader counters and the ratios derived from them (counter units:
    SQ_*_CYCLES, SQ_WAIT_* and SQ_ACTIVE_INST_* in quad-cycles summed over the waves of every
    SIMD; VALUBusy = 100 sum SQ_ACTIVE_INST_VALU / CUs / GRBM_GUI_ACTIVE)."""
    lines = ["| counter | mean per dispatch |", "|---|---|"]
    for k in sorted(c):
        lines.append(f"| {k} | {c[k]:.6g} |")
    d = []
    if "SQ_WAVES" in c and c["SQ_WAVES"]:
        for k in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR"):
            if k in c:
                d.append(f"- {k} per wave: {c[k] / c['SQ_WAVES']:.1f}")
    if "SQ_WAVE_CYCLES" in c and c["SQ_WAVE_CYCLES"]:
        for k in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS",
                  "SQ_ACTIVE_INST_ANY"):
            if k in c:
                d.append(f"- {k} / SQ_WAVE_CYCLES (share of wave lifetime): {c[k] / c['SQ_WAVE_CYCLES']:.3f}")
    if "SQ_LDS_BANK_CONFLICT" in c and c.get("SQ_LDS_IDX_ACTIVE"):
        d.append(f"- SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE: {c['SQ_LDS_BANK_CONFLICT'] / c['SQ_LDS_IDX_ACTIVE']:.3f}")
    if "VALUBusy" in c:
        d.append(f"- VALUBusy: {c['VALUBusy']:.1f} %")
    return lines + [""] + d


def unet_layers(chans, c_in, batch, side):
    """The forward pass's 3x3 convolutions in launch order: (name, pixels, real input channels,
    output channels, bytes of one BF16 read of the input and one write of the output)."""
    L = len(chans)
    out = []
    for l in range(L):
        px = batch * (side >> l) ** 2
        ci = c_in if l == 0 else chans[l - 1]
        cin_stored = c_in if l == 0 else chans[l - 1]   # the first layer reads only the real channels
        out.append((f"enc{l}a", px, ci, chans[l], 2 * px * (cin_stored + chans[l])))
        pooled = px // 4 * chans[l] if l + 1 < L else 0
        out.append((f"enc{l}b", px, chans[l], chans[l], 2 * (px * 2 * chans[l] + pooled)))
    for l in range(L - 2, -1, -1):
        px = batch * (side >> l) ** 2
        up = px // 4 * chans[l + 1]
        out.append((f"dec{l}a", px, chans[l + 1] + chans[l], chans[l], 2 * (up + px * chans[l] + px * chans[l])))
        out.append((f"dec{l}b", px, chans[l], chans[l], 2 * px * chans[l] * (1 if l == 0 else 2) + (4 * px if l == 0 else 0)))
    return out


def unet_profile(trace_dir, pmc_dirs, chans, c_in, batch, side, peak_tflops=2500.0, peak_gbs=8000.0,
                 after_training=False):
    """Per-layer table of the network's forward convolutions: launch time (kernel trace),
    TFLOP/s, MfmaUtil and HBM traffic (--pmc runs), and each layer's roofline
    min(peak MFMA, arithmetic intensity x peak HBM) on its algorithmic bytes.  Dispatches of
    conv3_first_k and conv3_fwd_k before the first weight-gradient dispatch are the forward
    passes, in layer order
    (with after_training: those after the last weight-gradient dispatch, the inference passes
    that follow the training steps)."""
    layers = unet_layers(chans, c_in, batch, side)
    conv_names = ("conv3_fwd_k", "conv3_first_k", "conv3_pair0_k")

    def fwd_rows(rows, start_key):
        rows = sorted(rows, key=lambda r: int(r[start_key]))
        dws = [i for i, r in enumerate(rows) if "conv3_dw_k" in r["Kernel_Name"]]
        if after_training:
            sel = rows[(dws[-1] + 1 if dws else 0):]
        else:
            sel = rows[:(dws[0] if dws else len(rows))]
        return [r for r in sel if any(c in r["Kernel_Name"] for c in conv_names)]

    trace = fwd_rows(list(csv.DictReader(open(_one(os.path.join(trace_dir, "**", "*kernel_trace.csv"))))),
                     "Start_Timestamp")
    if any("conv3_pair0_k" in r["Kernel_Name"] for r in trace):
        # the first block in one launch: one row for both convolutions, whose algorithmic
        # bytes are the block's input and its outputs (the intermediate stays on chip)
        (na, px, ci, co, ba), (nb, _, cib, cob, bb) = layers[0], layers[1]
        inter = 2 * px * co
        layers = [("enc0a+b", px, ci, co, ba + bb - 2 * inter, 18.0 * px * (ci * co + cib * cob))] + layers[2:]
    n = len(layers)
    groups = len(trace) // n
    if groups < 2:
        raise ValueError(f"{len(trace)} forward convolutions in the trace, not several passes of {n}")
    durs = [[int(trace[g * n + i]["End_Timestamp"]) - int(trace[g * n + i]["Start_Timestamp"])
             for g in range(1, groups)] for i in range(n)]        # the first pass is a warm-up
    ctr = [dict() for _ in range(n)]
    for d in pmc_dirs:
        rows = list(csv.DictReader(open(_one(os.path.join(d, "**", "*counter_collection.csv")))))
        for r in rows:
            r["_id"] = int(r.get("Dispatch_Id") or 0)
        names = sorted({r["Counter_Name"] for r in rows})
        for cname in names:
            cr = fwd_rows([r for r in rows if r["Counter_Name"] == cname], "_id")
            g2 = len(cr) // n
            for i in range(n):
                vals = [float(cr[g * n + i]["Counter_Value"]) for g in range(1, g2)]
                if vals:
                    ctr[i][cname] = statistics.mean(vals)
    table = []
    for i, lay in enumerate(layers):
        name, px, ci, co, abytes = lay[:5]
        ns = statistics.mean(durs[i])
        flop = lay[5] if len(lay) > 5 else 18.0 * px * ci * co
        ai = flop / abytes
        roof = min(peak_tflops, ai * peak_gbs / 1e3)
        tf = flop / (ns * 1e-9) / 1e12
        row = {"layer": name, "pixels": px, "c_in": ci, "c_out": co, "gflop": flop / 1e9, "us": ns / 1e3,
               "tflops": tf, "alg_bytes": abytes, "ai": ai, "roofline_tflops": roof, "frac_of_roofline": tf / roof}
        if "MfmaUtil" in ctr[i]:
            row["mfma_util_pct"] = ctr[i]["MfmaUtil"]
        if "VALUBusy" in ctr[i]:
            row["valu_busy_pct"] = ctr[i]["VALUBusy"]
        if "FETCH_SIZE" in ctr[i] or "WRITE_SIZE" in ctr[i]:
            row["traffic_kib"] = ctr[i].get("FETCH_SIZE", 0.0) + ctr[i].get("WRITE_SIZE", 0.0)
        table.append(row)
    return table


def unet_lines(table):
    """Markdown rows of the per-layer table; a VALUBusy column when a run collected it (the
    vector ALU's share of the cycles: issue-bound layers show it high beside a low MfmaUtil)."""
    valu = any("valu_busy_pct" in r for r in table)
    head = "| layer | pixels | c_in → c_out | GFLOP | µs | TFLOP/s | roofline TFLOP/s (AI flop/B) | of roofline | MfmaUtil %"
    lines = [head + (" | VALUBusy % |" if valu else " |"), "|---|---|---|---|---|---|---|---|---|" + ("---|" if valu else "")]
    for r in table:
        mu = f"{r['mfma_util_pct']:.1f}" if "mfma_util_pct" in r else "—"
        vb = (f" {r['valu_busy_pct']:.1f} |" if "valu_busy_pct" in r else " — |") if valu else ""
        lines.append(f"| {r['layer']} | {r['pixels']} | {r['c_in']} → {r['c_out']} | {r['gflop']:.1f} | {r['us']:.1f} | "
                     f"{r['tflops']:.0f} | {r['roofline_tflops']:.0f} ({r['ai']:.0f}) | {r['frac_of_roofline']:.2f} | {mu} |"
                     + vb)
    tot_f = sum(r["gflop"] for r in table)
    tot_us = sum(r["us"] for r in table)
    lines.append(f"| all 3x3 convolutions | | | {tot_f:.0f} | {tot_us:.0f} | {tot_f / tot_us * 1e3:.0f} | | | |"
                 + (" |" if valu else ""))
    return lines


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", help="FETCH_SIZE run (omit for a kernel-statistics summary only)")
    ap.add_argument("--write", help="WRITE_SIZE run")
    ap.add_argument("--nodes", type=int, default=0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--depth", type=int, default=2, choices=[1, 2], help="time steps per launch of the step kernel")
    ap.add_argument("--lattice", default="d2q9", choices=["d2q9", "d3q15"])
    ap.add_argument("--command", required=True, help="the profiled command lines (for the summary header)")
    ap.add_argument("--out", required=True, help="output prefix, e.g. profiles/step2_fused_spinodal8192_fp32")
    ap.add_argument("--title", default="", help="summary title (stats-only mode)")
    ap.add_argument("--kernel", default="", help="kernel name substring (default: the lattice's step kernel)")
    ap.add_argument("--tiling", default="", help="launch shape of the profiled runs (block_threads,rows), recorded")
    ap.add_argument("--sq", action="append", default=[],
                    help="a --pmc run of shader counters of the step kernel (repeatable), summarised beside the traffic")
    ap.add_argument("--last", type=int, default=0,
                    help="use only the last N dispatches of the kernel (runs that also launch it in other shapes)")
    ap.add_argument("--unet", default="", help="per-layer summary of the network's forward: "
                    "chans,c_in,batch,side (e.g. 32-64-128-256-256,5,16,256); --trace plus --sq runs")
    ap.add_argument("--unet-inference", action="store_true",
                    help="take the forward passes after the training steps (the whole-field inference)")
    args = ap.parse_args()
    if args.unet:
        ch, cin, bsz, side = args.unet.split(",")
        table = unet_profile(args.trace, args.sq, [int(v) for v in ch.split("-")], int(cin), int(bsz), int(side),
                             after_training=args.unet_inference)
        lines = [f"# rocprofv3 summary: {args.title or 'network forward, per layer'}", "", "Commands:", ""]
        lines += ["    " + c for c in args.command.split(";;")]
        lines += ["", "Forward 3x3 convolutions in launch order (pooling, upsampling-concatenation and the head "
                  "are fused into them); roofline = min(2500 TFLOP/s BF16 MFMA, arithmetic intensity x 8000 GB/s) "
                  "on the algorithmic bytes (one BF16 read of the input, one write of the output):", ""]
        lines += unet_lines(table)
        with open(args.out + ".md", "w") as fh:
            fh.write("\n".join(lines) + "\n")
        with open(args.out + ".json", "w") as fh:
            json.dump(table, fh, indent=1)
        print("\n".join(lines))
        return
    d3 = args.lattice == "d3q15"
    if d3:
        args.depth = 1
    STEP_KERNEL = args.kernel or (STEP_KERNEL_3D if d3 else STEP_KERNELS[args.depth])
    q = 15 if d3 else 9
    if not args.fetch:
        stats_only(args)
        return

    esize = 4 if args.precision == "fp32" else 8
    kib = 1024.0
    f_copy = statistics.median(counter_values(args.fetch, "FETCH_SIZE", COPY_KERNEL)) * kib
    w_copy = statistics.median(counter_values(args.write, "WRITE_SIZE", COPY_KERNEL)) * kib
    fetch_scale = COPY_BYTES / f_copy
    write_scale = COPY_BYTES / w_copy
    fv = counter_values(args.fetch, "FETCH_SIZE", STEP_KERNEL)
    wv = counter_values(args.write, "WRITE_SIZE", STEP_KERNEL)
    if args.last:
        fv, wv = fv[-args.last:], wv[-args.last:]
    f_step = statistics.median(fv) * kib * fetch_scale
    w_step = statistics.median(wv) * kib * write_scale
    stats = kernel_stats(args.trace)
    step = dict([s for s in stats if STEP_KERNEL in s["name"]][0])
    if args.last:
        name, durs = last_dispatches(args.trace, STEP_KERNEL, args.last)
        step = {"name": name, "avg_ns": statistics.mean(durs)}
    # algorithmic bytes: q populations read + q written per lattice update
    # (the one-step figure), times the updates of one launch; the launch's
    # own minimum traffic is one read and one write of the state
    alg = 2 * q * esize * args.nodes * args.depth
    min_traffic = 2 * q * esize * args.nodes
    rec = {
        "kernel": step["name"],
        "kernel_sha256_16": kernel_hash(args.lattice),
        "lattice": args.lattice,
        "nodes": args.nodes,
        "precision": args.precision,
        "depth": args.depth,
        "min_bytes_per_launch": min_traffic,
        "avg_duration_ms": step["avg_ns"] / 1e6,
        "dispatches_used": args.last or "all",
        "tiling": [int(v) for v in args.tiling.split(",")] if args.tiling else None,
        "fetch_scale_from_copy": fetch_scale,
        "write_scale_from_copy": write_scale,
        "fetch_bytes_per_launch": f_step,
        "write_bytes_per_launch": w_step,
        "bytes_per_launch": f_step + w_step,
        "algorithmic_bytes_per_launch": alg,
        "traffic_over_algorithmic": (f_step + w_step) / alg,
        "achieved_alg_GBs": alg / (step["avg_ns"] * 1e-9) / 1e9,
        "achieved_traffic_GBs": (f_step + w_step) / (step["avg_ns"] * 1e-9) / 1e9,
    }
    with open(args.out + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    lines = [f"# rocprofv3 summary: {step['name']}", "", "Commands:", ""]
    lines += ["    " + c for c in args.command.split(";;")]
    lines += ["", "Kernel statistics (--kernel-trace --stats):", "",
              "| kernel | calls | avg ms | % time |", "|---|---|---|---|"]
    for s in stats[:8]:
        lines.append(f"| {s['name'][:90]} | {s['calls']} | {s['avg_ns'] / 1e6:.4f} | {s['pct']:.1f} |")
    lines += ["", "HBM traffic of the step kernel (--pmc FETCH_SIZE, then --pmc WRITE_SIZE):", "",
              f"- copy-kernel calibration: FETCH_SIZE x {fetch_scale:.3f}, WRITE_SIZE x {write_scale:.3f} "
              f"(the copy moves {COPY_BYTES} B each way)",
              f"- fetched {f_step / 1e9:.3f} GB, written {w_step / 1e9:.3f} GB per launch of {args.depth} "
              f"time step(s); algorithmic {alg / 1e9:.3f} GB ({2 * q * esize} B per lattice update x "
              f"{args.depth} updates per node); ratio {rec['traffic_over_algorithmic']:.3f}; one read + one write "
              f"of the state = {min_traffic / 1e9:.3f} GB (measured / that = {(f_step + w_step) / min_traffic:.3f})",
              f"- average duration {rec['avg_duration_ms']:.4f} ms"
              f"{f' (last {args.last} dispatches)' if args.last else ''} -> {rec['achieved_alg_GBs']:.0f} GB/s algorithmic, "
              f"{rec['achieved_traffic_GBs']:.0f} GB/s measured traffic (8000 GB/s peak)",
              f"- kernel source sha256[:16] = {rec['kernel_sha256_16']}"]
    if args.sq:
        sq = shader_counters(args.sq, STEP_KERNEL, args.last)
        rec["shader_counters"] = sq
        with open(args.out + ".json", "w") as fh:
            json.dump(rec, fh, indent=1)
        lines += ["", "Shader counters of the step kernel (further --pmc runs of the same command):", ""]
        lines += shader_lines(sq)
    with open(args.out + ".md", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
