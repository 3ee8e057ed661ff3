"""Seeded synthetic initial conditions (shared by the tests, the benchmark and the oracle runs).

Only input generation lives here: initial order-parameter fields and the
parameter draws of the workloads.  None of the lattice Boltzmann arithmetic.

Workloads (lattice units, dx = dt = 1, periodic):
* droplet: a centred disc phi = tanh((R - r) / (sqrt(2) * eps_w)), r the
  minimum-image distance to the node (cx, cy); the profile of eq 40 with
  D = 2 sqrt(2) eps_w.
* spinodal: phi = mean + i.i.d. U(-amp, amp) from numpy's PCG64 seeded
  generator (the random initial state of eq 42, at a small amplitude).
* two droplets of eq 41 (sum of two tanh discs plus one).
* three-dimensional ball, spinodal and wavy-layer fields ([nz][ny][nx]).
"""
from __future__ import annotations

import math

import numpy as np


def min_image(d: np.ndarray, n: int) -> np.ndarray:
    return (d + n / 2.0) % n - n / 2.0


def droplet(nx: int, ny: int, radius: float, eps_w: float, cx: float | None = None,
            cy: float | None = None, inside: float = 1.0) -> np.ndarray:
    """Centred tanh disc; default centre is node (nx // 2, ny // 2)."""
    cx = nx // 2 if cx is None else cx
    cy = ny // 2 if cy is None else cy
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    r = np.hypot(min_image(x - cx, nx), min_image(y - cy, ny))
    return inside * np.tanh((radius - r) / (math.sqrt(2.0) * eps_w))


def droplet_width(radius: float, width_D: float, nx: int, ny: int, cx=None, cy=None) -> np.ndarray:
    """Eq 40 form: tanh(2 (R - r) / D)."""
    return droplet(nx, ny, radius, width_D / (2.0 * math.sqrt(2.0)), cx, cy)


def two_droplets(nx: int, ny: int, width_D: float, drops=((28, 35, 40), (9, 70, 70))) -> np.ndarray:
    """Eq 41: sum_i tanh(2 (R_i - r_i) / D) + 1 with (R_i, x_i, y_i)."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    out = np.ones((ny, nx))
    for (R, x0, y0) in drops:
        r = np.hypot(min_image(x - x0, nx), min_image(y - y0, ny))
        out += np.tanh(2.0 * (R - r) / width_D)
    return out


def sphere(nx: int, ny: int, nz: int, radius: float, eps_w: float, centre=None) -> np.ndarray:
    """Three-dimensional tanh ball, [nz][ny][nx]; default centre (nx // 2, ny // 2, nz // 2)."""
    cx, cy, cz = (nx // 2, ny // 2, nz // 2) if centre is None else centre
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    r = np.sqrt(min_image(x - cx, nx) ** 2 + min_image(y - cy, ny) ** 2 + min_image(z - cz, nz) ** 2)
    return np.tanh((radius - r) / (math.sqrt(2.0) * eps_w))


def sphere_width(n: int, radius: float, width_D: float, centre=None) -> np.ndarray:
    """Eq 43 form on an n^3 box: tanh(2 (R - r) / D), default centre (n/2, n/2, n/2)."""
    c = (n // 2,) * 3 if centre is None else centre
    return sphere(n, n, n, radius, width_D / (2.0 * math.sqrt(2.0)), c)


def two_spheres(n: int, width_D: float, balls=((28, 45, 40, 40), (12, 75, 75, 75))) -> np.ndarray:
    """Two-ball form of the paper's second 3D test: sum_i tanh(2 (R_i - r_i) / D) + 1 with
    (R_i, x_i, y_i, z_i), r_i the minimum-image distance."""
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(np.float64)
    out = np.ones((n, n, n))
    for (R, x0, y0, z0) in balls:
        r = np.sqrt(min_image(x - x0, n) ** 2 + min_image(y - y0, n) ** 2 + min_image(z - z0, n) ** 2)
        out += np.tanh(2.0 * (R - r) / width_D)
    return out


def wavy_slab(nx: int, ny: int, nz: int, eps_w: float, z_lo: float, z_hi: float, amp: float = 1.0) -> np.ndarray:
    """A layer phi ~ +1 between two tanh interfaces normal to z, [nz][ny][nx]; the lower
    interface is displaced by amp (sin(2 pi x / nx) + 0.7 cos(2 pi y / ny)), the upper by
    amp / 2 sin(2 pi (x + y) / nx)."""
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    lo = z_lo + amp * (np.sin(2 * np.pi * x / nx) + 0.7 * np.cos(2 * np.pi * y / ny))
    hi = z_hi + 0.5 * amp * np.sin(2 * np.pi * (x + y) / nx)
    w = math.sqrt(2.0) * eps_w
    return np.tanh((z - lo) / w) - np.tanh((z - hi) / w) - 1.0


def spinodal3(nx: int, ny: int, nz: int, seed: int, amp: float = 0.05, mean: float = 0.0) -> np.ndarray:
    """mean + U(-amp, amp), float64, [nz][ny][nx]."""
    rng = np.random.default_rng(seed)
    return mean + rng.uniform(-amp, amp, size=(nz, ny, nx))


def spinodal(nx: int, ny: int, seed: int, amp: float = 0.05, mean: float = 0.0) -> np.ndarray:
    """mean + U(-amp, amp), float64, row-major [ny][nx]."""
    rng = np.random.default_rng(seed)
    return mean + rng.uniform(-amp, amp, size=(ny, nx))


# ---- workload presets --------------------------------------------------------
# Interface-width reading: the workloads give the tanh width eps_w; the paper's
# surface tension sigma = 0.01 (eq 39) and D = 2 sqrt(2) eps_w fix kappa, beta
# through eq 5 on each side of the boundary.
SIGMA_PAPER = 0.01


def width_from_eps(eps_w: float) -> float:
    return 2.0 * math.sqrt(2.0) * eps_w


C1 = dict(name="droplet-64-fp64", n=64, radius=16.0, eps_w=2.0, alpha=0.05, m=4,
          mobility=1.0 / 6.0, eps_reg=0.03, steps=2000)   # tau_phi = 1  <=>  s_j = 1
C1_RATES_DISTINCT = (1.0, 1.1, 1.2, 1.0, 1.3, 1.0, 1.3, 1.4, 1.4)
C2 = dict(name="spinodal-1024-fp32", n=1024, eps_w=1.5, alpha=0.3, m=4, mobility=0.1,
          eps_reg=0.03, seed=0, amp=0.05, steps=50000)
C5 = dict(name="spinodal-8192-fp32", n=8192, eps_w=1.5, alpha=0.2, m=4, mobility=0.1,
          eps_reg=0.03, seed=5, amp=0.05, steps=200000)


def ensemble_members(count: int = 512, seed: int = 3, side_min: int = 64, side_max: int = 512):
    """Ragged ensemble draws: side log-uniform on [side_min, side_max], alpha ~ U[0, 0.3],
    m in {4, 6}, 50/50 spinodal (mean ~ U[-0.3, 0.3] + U(+-0.05)) / droplet of radius side/4.
    Returns a list of dicts with the member's parameters and its own seed."""
    master = np.random.default_rng(seed)
    members = []
    for j in range(count):
        side = int(round(math.exp(master.uniform(math.log(side_min), math.log(side_max)))))
        alpha = float(master.uniform(0.0, 0.3))
        m = int(master.choice([4, 6]))
        kind = "spinodal" if master.uniform() < 0.5 else "droplet"
        mean = float(master.uniform(-0.3, 0.3))
        members.append(dict(side=side, alpha=alpha, m=m, kind=kind, mean=mean,
                            seed=int(master.integers(0, 2**31 - 1))))
    return members


def member_phi0(mem: dict, eps_w: float = 1.5) -> np.ndarray:
    n = mem["side"]
    if mem["kind"] == "spinodal":
        return spinodal(n, n, mem["seed"], 0.05, mem["mean"])
    return droplet(n, n, n / 4.0, eps_w) * 1.0
