"""Test helpers: the same workload handed to the HIP path (through the C-ABI binding)
and to the oracle.  Only configuration is translated here; no method arithmetic."""
from __future__ import annotations

import math

import numpy as np

from oracle import lbm, lbm3
from paper_2501_03759_amd import inputs

REG_NAMES = {0: "none", 1: "linear", 2: "willmore"}
QFORM_NAMES = {0: "derived", 1: "literal"}


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def make_params(nx, ny, precision, sigma=0.01, width=None, eps_w=None, **kw):
    """lbch.Params with kappa, beta from (sigma, D) via the library's eq 5 helper."""
    from paper_2501_03759_amd import lbch
    if width is None:
        width = inputs.width_from_eps(eps_w) if eps_w is not None else 5.0
    return lbch.default_params(nx=nx, ny=ny, precision=precision, sigma_width=(sigma, width), **kw)


def oracle_params(p) -> lbm.Params:
    """The same problem for the oracle.  kappa and beta are the library's values (its eq 5
    helper, which test_sigma_width and the eq 39 golden file pin); every other field is
    copied as it is."""
    return lbm.Params(nx=p.nx, ny=p.ny, kappa=p.kappa, beta=p.beta, mobility=p.mobility, alpha=p.alpha,
                      aniso_m=p.aniso_m, theta0=p.aniso_theta0, reg=REG_NAMES[p.regularization],
                      eps_reg=p.eps_reg, q_form=QFORM_NAMES[p.q_form], grad_floor=p.grad_floor,
                      dx=p.dx, dt=p.dt, s_free=tuple(p.s[i] for i in range(9)))


def oracle_phi(phi0, p, nsteps) -> np.ndarray:
    return lbm.phi_of(lbm.run(phi0, oracle_params(p), nsteps))


def sampled_oracle_phi(phi0: np.ndarray, p, nsteps: int, points) -> np.ndarray:
    """phi after nsteps at the given (y, x) nodes of a large periodic grid, each from an
    oracle run on a periodic window around the node.  A node's value after k steps depends
    on the initial field within Chebyshev radius 4k + 2 (radius-3 stencils of phi plus the
    pull, and the init stencil), so a half-width of 4k + 3 makes the window's own wrap
    irrelevant at its centre."""
    h = 4 * nsteps + 3
    ny, nx = phi0.shape
    out = []
    for (y, x) in points:
        rows = np.arange(y - h, y + h + 1) % ny
        cols = np.arange(x - h, x + h + 1) % nx
        win = phi0[np.ix_(rows, cols)]
        op = oracle_params(p)
        op.nx = op.ny = 2 * h + 1
        out.append(lbm.phi_of(lbm.run(win, op, nsteps))[h, h])
    return np.array(out)


D3Q15_EVEN_ROWS = (1, 2, 9, 10, 11, 12, 13)
D3Q15_ODD_ROWS = (4, 6, 8, 14)


def oracle_params3(p) -> lbm3.Params:
    """The D3Q15 problem for the three-dimensional oracle.  The library takes one rate per
    parity class from the D2Q9 slots: the even rows from s[1] (= s[2] = s[7] = s[8]), the
    odd rows other than the fluxes from s[4] (= s[6])."""
    s = [1.0] * 15
    for r in D3Q15_EVEN_ROWS:
        s[r] = p.s[1]
    for r in D3Q15_ODD_ROWS:
        s[r] = p.s[4]
    return lbm3.Params(nx=p.nx, ny=p.ny, nz=p.nz, kappa=p.kappa, beta=p.beta, mobility=p.mobility, alpha=p.alpha,
                       reg=REG_NAMES[p.regularization], eps_reg=p.eps_reg, q_form=QFORM_NAMES[p.q_form],
                       grad_floor=p.grad_floor, dx=p.dx, dt=p.dt, s_free=tuple(s))


def oracle_phi3(phi0, p, nsteps) -> np.ndarray:
    return lbm3.phi_of(lbm3.run(phi0, oracle_params3(p), nsteps))


def sampled_oracle_phi3(phi0: np.ndarray, p, nsteps: int, points) -> np.ndarray:
    """phi after nsteps at the given (z, y, x) nodes of a large periodic box, each from an
    oracle run on a periodic cube around the node (same dependence radius 4k + 2 as in 2D)."""
    h = 4 * nsteps + 3
    nz, ny, nx = phi0.shape
    out = []
    for (z, y, x) in points:
        idx = (np.arange(z - h, z + h + 1) % nz, np.arange(y - h, y + h + 1) % ny, np.arange(x - h, x + h + 1) % nx)
        win = phi0[np.ix_(*idx)]
        op = oracle_params3(p)
        op.nx = op.ny = op.nz = 2 * h + 1
        out.append(lbm3.phi_of(lbm3.run(win, op, nsteps))[h, h, h])
    return np.array(out)
