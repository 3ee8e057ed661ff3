"""Linearised LB step and continuum dispersion relation (isotropic limit alpha = 0).

TEST INFRASTRUCTURE ONLY.  The symbols below were derived by hand from the
paper's equations; they are written as closed forms (trigonometric symbols of
the eq 26 stencils, moment algebra of eqs 18/19) and do not call the stepping
code in ``lbm``.  Only the constant tables of eq 20 / eq 23 are shared.

About a uniform state phi_bar (alpha = 0, so gamma = 1 and Q = kappa grad phi)
a Fourier mode delta f_i exp(i q.x) evolves under one step of eq 17 as
    delta f_new = A(q) delta f,
    A(q) = diag(exp(-i q.c_i dt)) [I - M^-1 S M (I - a 1^T) + dt M^-1 (I - S/2) M b 1^T],
with a = d f_eq / d phi (eq 18) and b = d F / d phi (eq 19).
"""
from __future__ import annotations

import numpy as np

from . import lbm


def symbol_grad(qx, qy, dx=1.0):
    """Fourier symbol of eq 26a (lattice units scaled by 1/dx): i*(2/3) sin(q_x dx)(1 + cos(q_y dx)/2)/dx."""
    ax, ay = qx * dx, qy * dx
    gx = 1j * (2.0 / 3.0) * np.sin(ax) * (1.0 + 0.5 * np.cos(ay)) / dx
    gy = 1j * (2.0 / 3.0) * np.sin(ay) * (1.0 + 0.5 * np.cos(ax)) / dx
    return gx, gy


def symbol_lap(qx, qy, dx=1.0):
    """Fourier symbol of eq 26b: [4/3 (cos a + cos b - 2) + 2/3 (cos a cos b - 1)] / dx^2."""
    ax, ay = qx * dx, qy * dx
    return ((4.0 / 3.0) * (np.cos(ax) + np.cos(ay) - 2.0)
            + (2.0 / 3.0) * (np.cos(ax) * np.cos(ay) - 1.0)) / (dx * dx)


def _f(phi, p):
    return 4.0 * p.beta * phi * (phi * phi - 1.0)


def _fp(phi, p):
    return 4.0 * p.beta * (3.0 * phi * phi - 1.0)


def _fpp(phi, p):
    return 24.0 * p.beta * phi


def amplification(p: lbm.Params, phi_bar: float, qx: float, qy: float) -> np.ndarray:
    """A(q) for one step linearised about phi_bar (requires alpha = 0)."""
    if p.alpha != 0.0:
        raise ValueError("linearisation is only defined for the isotropic limit")
    gx, gy = symbol_grad(qx, qy, p.dx)
    L = symbol_lap(qx, qy, p.dx)
    fp = _fp(phi_bar, p)
    # d mu_alpha / d phi  (eq 16)
    dmu_a = fp - p.kappa * L
    # d mu / d phi: gamma f - div(kappa grad phi) + regularisation (eqs 12/13)
    dmu = fp - p.kappa * (gx * gx + gy * gy)
    if p.reg == lbm.REG_WILLMORE:
        dmu = dmu + p.eps_reg * ((L - fp) ** 2 + _fpp(phi_bar, p) * _f(phi_bar, p))
    elif p.reg == lbm.REG_LINEAR:
        dmu = dmu + p.eps_reg * L * L
    dmu_b = dmu - dmu_a
    # eq 18 and eq 19, differentiated w.r.t. phi = sum_i f_i
    a = lbm.WEIGHTS * dmu_a
    a = a.astype(np.complex128)
    a[0] = 1.0 + (lbm.WEIGHTS[0] - 1.0) * dmu_a
    b = -lbm.WEIGHTS * p.c * (lbm.E[0] * gx + lbm.E[1] * gy) * dmu_b
    S = np.diag(lbm.relaxation_rates(p))
    I9 = np.eye(9)
    ones = np.ones((1, 9))
    coll = (I9 - lbm.M_INV @ S @ lbm.M_MATRIX @ (I9 - a[:, None] @ ones)
            + p.dt * lbm.M_INV @ (I9 - S / 2.0) @ lbm.M_MATRIX @ (b[:, None] @ ones))
    shift = np.diag(np.exp(-1j * (qx * lbm.E[0] + qy * lbm.E[1]) * p.dx))
    return shift @ coll


def slow_eigenvalue(p: lbm.Params, phi_bar: float, qx: float, qy: float) -> complex:
    """Eigenvalue of A(q) on the conserved (phi) branch: the one closest to 1."""
    lam = np.linalg.eigvals(amplification(p, phi_bar, qx, qy))
    return lam[np.argmin(np.abs(lam - 1.0))]


def continuum_rate(p: lbm.Params, phi_bar: float, q2: float) -> float:
    """omega(q) of d phi/dt = M lap mu linearised about phi_bar (eqs 10, 13, alpha = 0)."""
    fp = _fp(phi_bar, p)
    dmu = fp + p.kappa * q2
    if p.reg == lbm.REG_WILLMORE:
        dmu += p.eps_reg * ((q2 + fp) ** 2 + _fpp(phi_bar, p) * _f(phi_bar, p))
    elif p.reg == lbm.REG_LINEAR:
        dmu += p.eps_reg * q2 * q2
    return -p.mobility * q2 * dmu
