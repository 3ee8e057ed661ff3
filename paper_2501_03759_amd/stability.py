"""Stability maps of the collision variants (MRT, SRT, TRT; Section 3), computed on the GPU
with the ensemble.

Each parameter point is one member of a single lbch_batch: a 64 x 64 periodic grid with
the eq 40 droplet (R = 16, interface width D), sigma = 0.01, advanced `steps` time steps.
A point is stable if phi stays finite with max |phi| <= 1.5.  The paper asserts that MRT
is the more stable choice without showing data; these maps are the measurement.  Three
maps, each over two axes with the others at the eq 39 values (M = 0.1, eps_reg = 0.03,
D = 5) and alpha = 0.3:

* mobility x eps_reg (the flux rate s_j against the regularisation strength);
* alpha x eps_reg (the largest stable anisotropy strength);
* interface width D (kappa = 3 sigma D / 8) x mobility.

    python -m paper_2501_03759_amd.stability            # prints the three Markdown tables

The D3Q15 map (``--lattice d3q15``): mobility x eps_reg for the same three rate choices,
applied class by class (even rows, fluxes, other odd rows), each point one simulation of a
ball (R = 10, D = 5) on a 40^3 periodic box for 20 000 steps.
"""
from __future__ import annotations

import argparse
import math

from . import inputs, lbch

MODELS = {"mrt": lbch.COLLISION_MRT, "srt": lbch.COLLISION_SRT, "trt": lbch.COLLISION_TRT}
MOBILITIES = (0.01, 0.02, 0.05, 0.1, 0.2, 0.5, 1.0, 2.0)
EPS_REGS = (0.03, 0.1, 0.2, 0.3, 0.5, 1.0, 2.0, 4.0)
ALPHAS = (0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 5.0)
ALPHA_EPS_REGS = (0.0, 0.03, 0.3, 1.0)
WIDTHS = (1.0, 1.5, 2.0, 3.0, 5.0, 8.0)
WIDTH_MOBILITIES = (0.01, 0.1, 1.0, 2.0, 5.0)
BASE = {"mobility": 0.1, "eps_reg": 0.03, "alpha": 0.3, "width": 5.0}


def flux_rate(mobility: float) -> float:
    """s_j at dx = dt = 1 (the relation stated after eq 38)."""
    return 1.0 / (3.0 * mobility + 0.5)


def scan(points, n=64, steps=30000, magic=0.25, precision=lbch.FP32, bound=1.5):
    """points: dicts with 'model' and any of mobility, eps_reg, alpha, width (the rest from
    BASE).  All run as one ensemble; returns the dicts with 'stable' and 'max_abs_phi'."""
    full = [dict(BASE, **p) for p in points]
    params = []
    for q in full:
        p = lbch.default_params(nx=n, ny=n, precision=precision, sigma_width=(inputs.SIGMA_PAPER, q["width"]),
                                mobility=q["mobility"], alpha=q["alpha"], eps_reg=q["eps_reg"],
                                regularization=lbch.REG_WILLMORE if q["eps_reg"] > 0 else lbch.REG_NONE)
        params.append(lbch.set_collision(p, MODELS[q["model"]], magic))
    with lbch.Batch(params) as b:
        for k, q in enumerate(full):
            b.init(k, inputs.droplet_width(n / 4.0, q["width"], n, n))
        b.step(steps)
        b.synchronize()
        for k, q in enumerate(full):
            try:
                _, _, lo, hi = b.moments(k, want_phi=False)
                amax = max(abs(lo), abs(hi))
                q["stable"] = math.isfinite(amax) and amax <= bound
            except lbch.LbchError:
                amax, q["stable"] = float("nan"), False
            q["max_abs_phi"] = amax
            q["s_j"] = flux_rate(q["mobility"])
    return full


def scan3(points, n=40, radius=10.0, steps=20000, magic=0.25, precision=lbch.FP32, bound=1.5):
    """As `scan` on D3Q15: each point is one simulation of a ball on an n^3 periodic box."""
    full = [dict(BASE, **p) for p in points]
    for q in full:
        p = lbch.default_params(lattice=lbch.D3Q15, nx=n, ny=n, nz=n, precision=precision,
                                sigma_width=(inputs.SIGMA_PAPER, q["width"]), mobility=q["mobility"],
                                alpha=q["alpha"], eps_reg=q["eps_reg"],
                                regularization=lbch.REG_WILLMORE if q["eps_reg"] > 0 else lbch.REG_NONE)
        lbch.set_collision(p, MODELS[q["model"]], magic)
        with lbch.Sim(p) as s:
            s.init(inputs.sphere_width(n, radius, q["width"]))
            s.step(steps)
            try:
                _, _, lo, hi = s.moments(want_phi=False)
                amax = max(abs(lo), abs(hi))
                q["stable"] = math.isfinite(amax) and amax <= bound
            except lbch.LbchError:
                amax, q["stable"] = float("nan"), False
        q["max_abs_phi"] = amax
        q["s_j"] = flux_rate(q["mobility"])
    return full


def stability_map3(models=("mrt", "srt", "trt"), mobilities=MOBILITIES, eps_regs=EPS_REGS, alpha=0.3, **kw):
    """Mobility x eps_reg map on D3Q15 (alpha fixed)."""
    return scan3([{"model": m, "mobility": mob, "eps_reg": e, "alpha": alpha}
                  for m in models for mob in mobilities for e in eps_regs], **kw)


def stability_map(models=("mrt", "srt", "trt"), mobilities=MOBILITIES, eps_regs=EPS_REGS, alpha=0.3, **kw):
    """Mobility x eps_reg map (alpha fixed)."""
    return scan([{"model": m, "mobility": mob, "eps_reg": e, "alpha": alpha}
                 for m in models for mob in mobilities for e in eps_regs], **kw)


def alpha_map(models=("mrt", "srt", "trt"), alphas=ALPHAS, eps_regs=ALPHA_EPS_REGS, **kw):
    """alpha x eps_reg map at M = 0.1 (eps_reg = 0: no regularisation)."""
    return scan([{"model": m, "alpha": a, "eps_reg": e} for m in models for e in eps_regs for a in alphas], **kw)


def width_map(models=("mrt", "srt", "trt"), widths=WIDTHS, mobilities=WIDTH_MOBILITIES, **kw):
    """Interface width D (kappa = 3 sigma D / 8, beta = 3 sigma / (4 D)) x mobility map."""
    return scan([{"model": m, "width": w, "mobility": mob} for m in models for mob in mobilities for w in widths],
                **kw)


def table(results, row="mobility", col="eps_reg") -> str:
    """Markdown: one block per model, `row` down, `col` across; o = stable."""
    cols = sorted({r[col] for r in results})
    names = {"mobility": "M", "eps_reg": "eps", "alpha": "alpha", "width": "D"}
    lines = []
    for model in dict.fromkeys(r["model"] for r in results):
        head = "M (s_j)" if row == "mobility" else names[row]
        lines += [f"{model.upper()}:", "", f"| {head} | " + " | ".join(f"{names[col]} {c:g}" for c in cols) + " |",
                  "|---|" + "---|" * len(cols)]
        for v in sorted({r[row] for r in results}):
            cell = {r[col]: r for r in results if r["model"] == model and r[row] == v}
            label = f"{v:g} ({flux_rate(v):.3f})" if row == "mobility" else f"{v:g}"
            lines.append(f"| {label} | " + " | ".join("o" if cell[c]["stable"] else "x" for c in cols) + " |")
        lines.append("")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=30000)
    ap.add_argument("--magic", type=float, default=0.25)
    ap.add_argument("--lattice", choices=("d2q9", "d3q15"), default="d2q9")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if args.lattice == "d3q15":
        print("## D3Q15: mobility x eps_reg (alpha = 0.3, D = 5, ball R = 10 on 40^3)\n")
        for m in MODELS:
            print(table(stability_map3(models=(m,), steps=args.steps, magic=args.magic), "mobility", "eps_reg"),
                  flush=True)
        return
    kw = dict(steps=args.steps, magic=args.magic)
    print("## mobility x eps_reg (alpha = 0.3, D = 5)\n")
    print(table(stability_map(**kw), "mobility", "eps_reg"), flush=True)
    print("## alpha x eps_reg (M = 0.1, D = 5)\n")
    print(table(alpha_map(**kw), "eps_reg", "alpha"), flush=True)
    print("## interface width D x mobility (alpha = 0.3, eps_reg = 0.03)\n")
    print(table(width_map(**kw), "mobility", "width"), flush=True)


if __name__ == "__main__":
    main()
