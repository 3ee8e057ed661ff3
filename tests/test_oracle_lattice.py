"""Pins of the oracle's lattice tables and stencils (eqs 20, 23, 26, 27a).

Each check compares the oracle with something other than itself: textbook
definitions of the D2Q9 moments, hand-computed Fourier symbols, exactness on
quadratics.
"""
import json
import os

import numpy as np
import pytest

from oracle import lbm, linear

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_weight_moments_eq27a():
    w, e = lbm.WEIGHTS, lbm.E.astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(e @ w).max() < 1e-15
    second = np.einsum("ai,bi,i->ab", e, e, w)
    assert np.allclose(second, np.eye(2) / 3.0, atol=1e-15, rtol=0)   # c_s^2 = 1/3 at c = 1


def test_moment_matrix_rows_are_lallemand_luo_polynomials():
    # Rows of eq 23 as functions of the velocities (Lallemand & Luo 2000, the source
    # the paper cites for the transform): 1, 3|c|^2-4, (9|c|^4-21|c|^2+8)/2, cx,
    # (3|c|^2-5)cx, cy, (3|c|^2-5)cy, cx^2-cy^2, cx cy.
    cx, cy = lbm.E.astype(float)
    c2 = cx * cx + cy * cy
    rows = [np.ones(9), 3 * c2 - 4, (9 * c2 * c2 - 21 * c2 + 8) / 2, cx, (3 * c2 - 5) * cx,
            cy, (3 * c2 - 5) * cy, cx * cx - cy * cy, cx * cy]
    assert np.array_equal(np.array(rows), lbm.M_MATRIX)


def test_moment_matrix_orthogonal_and_inverse():
    gram = lbm.M_MATRIX @ lbm.M_MATRIX.T
    norms = np.array([9, 36, 36, 6, 12, 6, 12, 4, 4], dtype=float)
    assert np.array_equal(gram, np.diag(norms))
    assert np.allclose(lbm.M_INV, lbm.M_MATRIX.T / norms[None, :], atol=1e-15, rtol=0)


def test_eq39_parameters_golden():
    g = json.load(open(os.path.join(GOLDEN, "eq39_parameters.json")))
    kappa, beta = lbm.kappa_beta_from_sigma_width(g["sigma"], g["width_D"])
    assert abs(kappa - g["kappa"]) < 1e-15 and abs(beta - g["beta"]) < 1e-15
    p = lbm.Params(nx=8, ny=8, kappa=kappa, beta=beta, mobility=g["mobility"])
    s = lbm.relaxation_rates(p)
    assert abs(s[3] - g["s_j"]) < 1e-14 and abs(s[5] - g["s_j"]) < 1e-14
    # eq 5 forward
    assert abs(4 * np.sqrt(2 * kappa * beta) / 3 - g["sigma"]) < 1e-15
    assert abs(np.sqrt(2 * kappa / beta) - g["width_D"]) < 1e-13


def _params(n=16, dx=1.0):
    return lbm.Params(nx=n, ny=n, kappa=0.02, beta=0.0015, dx=dx, dt=dx * dx)


@pytest.mark.parametrize("mode,lap_val,gx_val", [
    ((4, 0), -2.0, 1.0),              # q = (pi/2, 0): hand values of eq 26b / eq 26a symbols
    ((4, 4), -10.0 / 3.0, 2.0 / 3.0),  # q = (pi/2, pi/2)
])
def test_stencils_hand_symbols(mode, lap_val, gx_val):
    n = 16
    p = _params(n)
    y, x = np.mgrid[0:n, 0:n].astype(float)
    qx, qy = 2 * np.pi * mode[0] / n, 2 * np.pi * mode[1] / n
    arg = qx * x + qy * y
    lap = lbm.laplacian(np.cos(arg), p)
    assert np.abs(lap - lap_val * np.cos(arg)).max() < 1e-14
    g = lbm.grad(np.sin(arg), p)
    assert np.abs(g[0] - gx_val * np.cos(arg)).max() < 1e-14


def test_stencils_fourier_symbols_all_modes():
    nx, ny = 12, 10
    p = lbm.Params(nx=nx, ny=ny, kappa=0.02, beta=0.0015)
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    for kx in range(nx):
        for ky in range(ny):
            qx, qy = 2 * np.pi * kx / nx, 2 * np.pi * ky / ny
            mode = np.exp(1j * (qx * x + qy * y))
            gxs, gys = linear.symbol_grad(qx, qy)
            lap = lbm.laplacian(mode.real, p) + 1j * lbm.laplacian(mode.imag, p)
            gr = lbm.grad(mode.real, p) + 1j * lbm.grad(mode.imag, p)
            assert np.abs(lap - linear.symbol_lap(qx, qy) * mode).max() < 1e-13
            assert np.abs(gr[0] - gxs * mode).max() < 1e-13
            assert np.abs(gr[1] - gys * mode).max() < 1e-13


@pytest.mark.parametrize("dx", [1.0, 0.5])
def test_stencils_exact_on_quadratics(dx):
    # Second-order isotropic stencils are exact on quadratics (checked away from the periodic seam).
    n = 24
    p = _params(n, dx)
    y, x = np.mgrid[0:n, 0:n].astype(float) * dx
    a, b, c, d, e = 0.3, -0.7, 1.1, 0.2, -0.4
    phi = a * x * x + b * x * y + c * y * y + d * x + e * y
    g = lbm.grad(phi, p)
    lap = lbm.laplacian(phi, p)
    s = (slice(2, n - 2), slice(2, n - 2))
    assert np.abs(g[0][s] - (2 * a * x + b * y + d)[s]).max() < 1e-11
    assert np.abs(g[1][s] - (b * x + 2 * c * y + e)[s]).max() < 1e-11
    assert np.abs(lap[s] - (2 * a + 2 * c)).max() < 1e-11
