"""Stability map of the collision variants (MRT, SRT, TRT; Section 3) over mobility and
regularisation strength, computed on the GPU with the ensemble.

Each parameter point is one member of a single lbch_batch: a 64 x 64 periodic grid with
the eq 40 droplet (R = 16, D = 5), sigma = 0.01, advanced `steps` time steps.  A point is
stable if phi stays finite with max |phi| <= 1.5.  The paper asserts that MRT is the more
stable choice without showing data; this map is the measurement.

    python -m paper_2501_03759_amd.stability            # prints a Markdown table
"""
from __future__ import annotations

import argparse
import itertools
import math

from . import inputs, lbch

MODELS = {"mrt": lbch.COLLISION_MRT, "srt": lbch.COLLISION_SRT, "trt": lbch.COLLISION_TRT}
MOBILITIES = (0.01, 0.02, 0.05, 0.1, 0.2, 0.5, 1.0, 2.0)
EPS_REGS = (0.03, 0.1, 0.2, 0.3, 0.5, 1.0, 2.0, 4.0)


def flux_rate(mobility: float) -> float:
    """s_j at dx = dt = 1 (the relation stated after eq 38)."""
    return 1.0 / (3.0 * mobility + 0.5)


def stability_map(models=("mrt", "srt", "trt"), mobilities=MOBILITIES, eps_regs=EPS_REGS, alpha=0.3, n=64,
                  steps=30000, magic=0.25, precision=lbch.FP32, bound=1.5):
    """Runs every (model, mobility, eps_reg) point as one ensemble member; returns a list of
    dicts {model, mobility, eps_reg, s_j, stable, max_abs_phi}."""
    points = list(itertools.product(models, mobilities, eps_regs))
    params = [lbch.set_collision(lbch.default_params(nx=n, ny=n, precision=precision, mobility=m, alpha=alpha,
                                                     eps_reg=e), MODELS[name], magic)
              for (name, m, e) in points]
    phi0 = inputs.droplet_width(n / 4.0, 5.0, n, n)
    out = []
    with lbch.Batch(params) as b:
        for k in range(len(points)):
            b.init(k, phi0)
        b.step(steps)
        b.synchronize()
        for k, (name, m, e) in enumerate(points):
            try:
                _, _, lo, hi = b.moments(k, want_phi=False)
                amax = max(abs(lo), abs(hi))
                stable = math.isfinite(amax) and amax <= bound
            except lbch.LbchError:
                amax, stable = float("nan"), False
            out.append({"model": name, "mobility": m, "eps_reg": e, "s_j": flux_rate(m), "stable": stable,
                        "max_abs_phi": amax})
    return out


def table(results) -> str:
    """Markdown: one block of rows per model, mobility down, eps_reg across; o = stable."""
    eps = sorted({r["eps_reg"] for r in results})
    lines = []
    for model in dict.fromkeys(r["model"] for r in results):
        lines += [f"{model.upper()}:", "", "| M (s_j) | " + " | ".join(f"eps {e:g}" for e in eps) + " |",
                  "|---|" + "---|" * len(eps)]
        for m in sorted({r["mobility"] for r in results}):
            row = {r["eps_reg"]: r for r in results if r["model"] == model and r["mobility"] == m}
            lines.append(f"| {m:g} ({flux_rate(m):.3f}) | " +
                         " | ".join("o" if row[e]["stable"] else "x" for e in eps) + " |")
        lines.append("")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=30000)
    ap.add_argument("--alpha", type=float, default=0.3)
    ap.add_argument("--magic", type=float, default=0.25)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    res = stability_map(alpha=args.alpha, steps=args.steps, magic=args.magic)
    print(table(res), flush=True)


if __name__ == "__main__":
    main()
