"""Training data from batched lattice Boltzmann runs and training of the surrogate.

Data: an ensemble of periodic spinodal runs (the 1024^2 FP32 workload with
per-run anisotropy alpha ~ U[0, 0.3], fold m in {4, 6}, orientation
theta0 ~ U[0, 2 pi), seeded noise) is advanced in one lbch_batch; at every
snapshot time t the order parameter phi(t) and, `jump` steps later,
phi(t + jump) are cut into random periodic crops (lbsg_gather) that stay
on the device as (input, target) pairs.  Inputs are phi plus constant
conditioning planes alpha, cos(m theta0), sin(m theta0), m / 6.

Everything numeric runs in the library's kernels (lbch_* for the lattice
Boltzmann runs, lbsg_* for crops, forward, backward and Adam); torch only
owns the device buffers.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import inputs, lbch, lbsg

N_COND = 4


def conditioning(alpha: float, m: int, theta0: float) -> np.ndarray:
    return np.array([alpha, math.cos(m * theta0), math.sin(m * theta0), m / 6.0], dtype=np.float32)


@dataclasses.dataclass
class RunSpec:
    alpha: float
    m: int
    theta0: float
    seed: int


def draw_runs(count: int, seed: int) -> list[RunSpec]:
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        out.append(RunSpec(alpha=float(rng.uniform(0.0, 0.3)), m=int(rng.choice([4, 6])),
                           theta0=float(rng.uniform(0.0, 2 * math.pi)), seed=int(seed * 1000 + j + 1)))
    return out


def run_params(spec: RunSpec, side: int, precision=lbch.FP32):
    d = inputs.C2
    return lbch.default_params(nx=side, ny=side, precision=precision,
                               sigma_width=(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"])),
                               mobility=d["mobility"], alpha=spec.alpha, aniso_m=spec.m, aniso_theta0=spec.theta0,
                               eps_reg=d["eps_reg"])


def generate(runs: list[RunSpec], side: int, t_first: int, t_last: int, every: int, jump: int, crop: int,
             crops_per_snapshot: int, seed: int, stream=None, log=print, extrapolate: bool = False,
             amp: float = 0.05, with_rate: bool = False):
    """Returns device tensors X [N, crop, crop, 1 + N_COND], Y [N, crop, crop] (torch float32).

    Y is phi(t + jump); with extrapolate it is phi(t + jump) - jump (phi(t+1) - phi(t)), the residual
    the network adds to the rate-extrapolated jump of the hybrid schedule (one plain step gives the
    rate, as there).  with_rate: a third tensor R [N, crop, crop] holds phi(t + 1) of the same crops
    (for measuring the rate-extrapolated jump beside the network), and the function returns
    (X, Y, R, T) with T [N] the snapshot time of each pair."""
    import torch
    rng = np.random.default_rng(seed)
    times = list(range(t_first, t_last + 1, every))
    n = len(runs) * len(times) * crops_per_snapshot
    X = torch.empty((n, crop, crop, 1 + N_COND), dtype=torch.float32, device="cuda")
    Y = torch.empty((n, crop, crop), dtype=torch.float32, device="cuda")
    field = torch.empty((side, side), dtype=torch.float32, device="cuda")
    per = len(runs) * crops_per_snapshot
    rate = extrapolate or with_rate
    if rate:
        T0 = torch.empty((per, crop, crop), dtype=torch.float32, device="cuda")
        T1 = torch.empty_like(T0)
    if with_rate:
        R = torch.empty((n, crop, crop), dtype=torch.float32, device="cuda")
        tt = np.repeat(np.array(times, dtype=np.int64), per)
    params = [run_params(r, side) for r in runs]
    t0 = time.time()
    with lbch.Batch(params, stream) as b:
        for k, r in enumerate(runs):
            b.init(k, inputs.spinodal(side, side, seed=r.seed, amp=amp))
        t = 0
        row = 0
        for ts in times:
            b.step(ts - t)
            t = ts
            offsets = []
            for k, r in enumerate(runs):
                if crop == side:     # whole periodic fields
                    yx = np.zeros((crops_per_snapshot, 2), dtype=np.int32)
                else:
                    yx = rng.integers(0, side, size=(crops_per_snapshot, 2)).astype(np.int32)
                offsets.append(yx)
                cond = np.tile(conditioning(r.alpha, r.m, r.theta0), (crops_per_snapshot, 1))
                b.phi_device(k, field.data_ptr(), lbch.FP32)
                lbsg.gather(field.data_ptr(), side, side, yx, crop, cond,
                            X[row + k * crops_per_snapshot].data_ptr(),
                            T0[k * crops_per_snapshot].data_ptr() if rate else None, stream)
            steps = jump
            if rate:
                b.step(1)
                steps -= 1
                for k in range(len(runs)):
                    b.phi_device(k, field.data_ptr(), lbch.FP32)
                    lbsg.gather(field.data_ptr(), side, side, offsets[k], crop, None, None,
                                T1[k * crops_per_snapshot].data_ptr(), stream)
                if with_rate:
                    R[row:row + per].copy_(T1)
            b.step(steps)
            t += jump
            for k, r in enumerate(runs):
                b.phi_device(k, field.data_ptr(), lbch.FP32)
                lbsg.gather(field.data_ptr(), side, side, offsets[k], crop, None, None,
                            Y[row + k * crops_per_snapshot].data_ptr(), stream)
            if extrapolate:
                lbch.extrapolate(Y[row].data_ptr(), T0.data_ptr(), T1.data_ptr(), -float(jump), per * crop * crop,
                                 Y[row].data_ptr(), stream)
            row += per
        b.synchronize()
    log(f"generated {n} pairs ({len(runs)} runs x {len(times)} snapshots x {crops_per_snapshot} crops) "
        f"in {time.time() - t0:.1f} s")
    if with_rate:
        return X, Y, R, tt
    return X, Y


def train(net: lbsg.Surrogate, X, Y, epochs: int, batch: int, lr: float, margin: int, seed: int = 0, log=print):
    """Adam with a cosine learning-rate decay; returns the per-epoch mean losses."""
    import torch
    n, crop = X.shape[0], X.shape[1]
    rng = np.random.default_rng(seed)
    xb = torch.empty((batch,) + tuple(X.shape[1:]), dtype=torch.float32, device="cuda")
    yb = torch.empty((batch,) + tuple(Y.shape[1:]), dtype=torch.float32, device="cuda")
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    history = []
    k = 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n)[: steps_per_epoch * batch], device="cuda")
        acc = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(Y, 0, idx, out=yb)
            step_lr = lr * 0.5 * (1.0 + math.cos(math.pi * k / max(1, total)))
            want = s == steps_per_epoch - 1 or s % 50 == 0
            loss = net.train_step(xb.data_ptr(), yb.data_ptr(), batch, crop, crop, margin, step_lr, want_loss=want)
            if want:
                acc = loss
            k += 1
        history.append(acc)
        log(f"epoch {ep}: loss {acc:.3e}")
    return history


def evaluate(net: lbsg.Surrogate, X, Y, margin: int, batch: int = 16):
    """Relative L2 error on the crop interiors: the network vs its input phi(t) as the prediction
    (the identity map phi(t+K) ~ phi(t); for residual targets of generate(extrapolate=True), the
    rate-extrapolated jump without the network)."""
    import torch
    n, crop = X.shape[0], X.shape[1]
    out = torch.empty((batch, crop, crop), dtype=torch.float32, device="cuda")
    s = slice(margin, crop - margin)
    num_net = num_id = den = 0.0
    for i in range(0, n - batch + 1, batch):
        net.forward(X[i:i + batch].data_ptr(), batch, crop, crop, out.data_ptr())
        torch.cuda.synchronize()
        tgt = Y[i:i + batch, s, s].double()
        num_net += float(((out[:, s, s].double() - tgt) ** 2).sum())
        num_id += float(((X[i:i + batch, s, s, 0].double() - tgt) ** 2).sum())
        den += float((tgt ** 2).sum())
    return math.sqrt(num_net / den), math.sqrt(num_id / den)


def evaluate_jumps(net: lbsg.Surrogate, X, Y, R, jump: int, T=None, split: int = 0, batch: int = 8,
                   margin: int = 0):
    """Held-out relative L2 errors of three predictions of phi(t + jump) against the plain
    scheme's: the network, no jump (phi(t)), and the rate-extrapolated jump phi(t) + jump
    (phi(t+1) - phi(t)); each also relative to the size of the true change
    |phi(t + jump) - phi(t)| (1 = no better than not jumping).  With T and split, the same
    for the pairs with t < split and t >= split.  Errors are taken over the crop interiors
    (margin pixels dropped on every side: a crop is not periodic at its edges)."""
    import torch
    n, crop = X.shape[0], X.shape[1]
    out = torch.empty((batch, crop, crop), dtype=torch.float32, device="cuda")
    acc = {}

    def add(key, k, v):
        acc.setdefault(key, np.zeros(5))
        acc[key][k] += v

    for i in range(0, n - batch + 1, batch):
        net.forward(X[i:i + batch].data_ptr(), batch, crop, crop, out.data_ptr())
        torch.cuda.synchronize()
        s = slice(margin, crop - margin)
        tgt = Y[i:i + batch, s, s].double()
        x0 = X[i:i + batch, s, s, 0].double()
        ext = x0 + jump * (R[i:i + batch, s, s].double() - x0)
        terms = [float(((out[:, s, s].double() - tgt) ** 2).sum()), float(((x0 - tgt) ** 2).sum()),
                 float(((ext - tgt) ** 2).sum()), float((tgt ** 2).sum()), float(((tgt - x0) ** 2).sum())]
        keys = ["all"]
        if T is not None and split:
            keys.append("early" if T[i] < split else "late")
        for key in keys:
            for k, v in enumerate(terms):
                add(key, k, v)
    res = {}
    for key, a in acc.items():
        res[key] = {"network": math.sqrt(a[0] / a[3]), "no_jump": math.sqrt(a[1] / a[3]),
                    "rate_extrapolation": math.sqrt(a[2] / a[3]),
                    "network_vs_change": math.sqrt(a[0] / a[4]), "rate_extrapolation_vs_change": math.sqrt(a[2] / a[4])}
    return res
