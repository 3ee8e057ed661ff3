"""Pins of two oracle functions that the whole-step pins do not fix on their own:

* the initial populations (reading R4: the equilibrium of eq 18 at phi0, with mu_alpha of
  eq 16 evaluated on phi0), on D2Q9 and D3Q15.  Their zeroth, first and second moments are
  fixed by eq 27b, and the second moment carries mu_alpha, whose Fourier amplitude on a
  cosine field is fixed by the hand-derived symbol of the eq 26b Laplacian;
* the m-fold anisotropy with orientation theta0 (reading R6, gamma = 1 + alpha cos(m (theta -
  theta0))), checked against Chebyshev closed forms of cos m theta and sin m theta written as
  polynomials in the normal's components, and against rotation covariance.

Each group also plants a mistake in the oracle (on the CPU) and checks that the pin sees it.
"""
import math

import numpy as np
import pytest

from oracle import lbm, lbm3, linear

RNG = np.random.default_rng(4321)
K39, B39 = lbm.kappa_beta_from_sigma_width(0.01, 5.0)


# ------------------------------------------------------------ initial populations --
def _cos_field_2d(nx, ny, kx, ky, phi_bar, eps):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    qx, qy = 2 * math.pi * kx / nx, 2 * math.pi * ky / ny
    c = np.cos(qx * x + qy * y)
    return phi_bar + eps * c, c, qx, qy


def _lap_symbol_d3q15(qx, qy, qz):
    # eq 26b on D3Q15 (weights 2/9, 1/9 x 6, 1/72 x 8; c_s^2 = 1/3), derived by hand:
    # 6 [ (2/9)(sum cos - 3) + (1/9)(8 prod cos - 8) ]
    cx, cy, cz = math.cos(qx), math.cos(qy), math.cos(qz)
    return (4.0 / 3.0) * (cx + cy + cz - 3.0) + (2.0 / 3.0) * (cx * cy * cz - 1.0)


def _mu_alpha_amplitude(phi_bar, eps, beta, kappa, lap_sym):
    # mu_alpha = f(phi) - kappa lap(phi) on phi = phi_bar + eps cos(q.x).  f is the cubic
    # 4 beta phi (phi^2 - 1): its Taylor series about phi_bar projects onto cos(q.x) as
    # f'(phi_bar) eps + (f'''/6)(3/4) eps^3 = f'(phi_bar) eps + 3 beta eps^3 (the eps^2 term
    # lives on the 0 and 2q modes), and lap(cos) = lap_sym cos exactly.
    return linear._fp(phi_bar, lbm.Params(nx=1, ny=1, kappa=kappa, beta=beta)) * eps + 3.0 * beta * eps ** 3 \
        - kappa * lap_sym * eps


def _check_init_2d(init):
    """Max relative deviations of the three moment pins for the given init function."""
    nx, ny = 16, 12
    worst = 0.0
    for (kx, ky, phi_bar, eps) in [(1, 0, 1.0, 1e-3), (2, 1, 0.0, 0.2), (3, 2, 0.3, 0.05), (5, 5, -0.6, 0.1)]:
        p = lbm.Params(nx=nx, ny=ny, kappa=K39, beta=B39)
        phi0, c, qx, qy = _cos_field_2d(nx, ny, kx, ky, phi_bar, eps)
        f = init(phi0, p)
        e = lbm.E.astype(float)
        zeroth = f.sum(0)
        first = np.einsum("ai,iyx->ayx", e, f)
        second = np.einsum("ai,bi,iyx->abyx", e, e, f)
        assert np.abs(zeroth - phi0).max() < 4e-15 * max(1.0, np.abs(phi0).max())
        assert np.abs(first).max() < 1e-15
        assert np.abs(second[0, 1]).max() < 1e-15
        assert np.abs(second[0, 0] - second[1, 1]).max() < 1e-15
        # second moment = c_s^2 mu_alpha; its cos(q.x) amplitude against the closed form
        mu = second[0, 0] / p.cs2
        amp = float((mu * c).sum() / (c * c).sum())
        want = _mu_alpha_amplitude(phi_bar, eps, p.beta, p.kappa, linear.symbol_lap(qx, qy))
        worst = max(worst, abs(amp - want) / abs(want))
    return worst


def test_initial_populations_moments_and_mu_alpha_2d():
    assert _check_init_2d(lbm.initial_populations) < 1e-12


def _check_init_3d(init):
    nx, ny, nz = 8, 6, 5
    worst = 0.0
    for (k, phi_bar, eps) in [((1, 0, 0), 1.0, 1e-3), ((2, 1, 1), 0.0, 0.2), ((1, 3, 2), -0.4, 0.1)]:
        p = lbm3.Params(nx=nx, ny=ny, nz=nz, kappa=K39, beta=B39)
        z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
        qx, qy, qz = 2 * math.pi * k[0] / nx, 2 * math.pi * k[1] / ny, 2 * math.pi * k[2] / nz
        c = np.cos(qx * x + qy * y + qz * z)
        phi0 = phi_bar + eps * c
        f = init(phi0, p)
        e = lbm3.E.astype(float)
        assert np.abs(f.sum(0) - phi0).max() < 4e-15 * max(1.0, np.abs(phi0).max())
        assert np.abs(np.einsum("ai,izyx->azyx", e, f)).max() < 1e-15
        second = np.einsum("ai,bi,izyx->abzyx", e, e, f)
        for a in range(3):
            for b in range(3):
                if a != b:
                    assert np.abs(second[a, b]).max() < 1e-15
            assert np.abs(second[a, a] - second[0, 0]).max() < 1e-15
        mu = second[0, 0] / p.cs2
        amp = float((mu * c).sum() / (c * c).sum())
        want = _mu_alpha_amplitude(phi_bar, eps, p.beta, p.kappa, _lap_symbol_d3q15(qx, qy, qz))
        worst = max(worst, abs(amp - want) / abs(want))
    return worst


def test_initial_populations_moments_and_mu_alpha_3d():
    assert _check_init_3d(lbm3.initial_populations) < 1e-12


@pytest.mark.parametrize("mod,check", [(lbm, _check_init_2d), (lbm3, _check_init_3d)])
@pytest.mark.parametrize("planted", ["laplacian_sign", "bulk_sign"])
def test_initial_population_pins_catch_planted_mistakes(mod, check, planted, monkeypatch):
    # a sign slip in kappa lap(phi0) or in f(phi0) inside mu_alpha of the initial state
    if planted == "laplacian_sign":
        orig = mod.laplacian
        monkeypatch.setattr(mod, "laplacian", lambda chi, p: -orig(chi, p))
    else:
        orig = mod.bulk_f
        monkeypatch.setattr(mod, "bulk_f", lambda phi, p: -orig(phi, p))
    assert check(mod.initial_populations) > 1e-2


# --------------------------------------------------------------------- anisotropy --
def _cheb_T(m, x):
    """cos(m theta) as a polynomial in x = cos(theta) (Chebyshev T_4, T_6)."""
    return {4: 8 * x ** 4 - 8 * x ** 2 + 1, 6: 32 * x ** 6 - 48 * x ** 4 + 18 * x ** 2 - 1}[m]


def _cheb_U(m, x):
    """sin(m theta) / sin(theta) as a polynomial in x = cos(theta) (Chebyshev U_3, U_5)."""
    return {4: 8 * x ** 3 - 4 * x, 6: 32 * x ** 5 - 32 * x ** 3 + 6 * x}[m]


def _closed_form(pg, alpha, m, shift):
    """gamma and |p| P grad_n gamma for gamma = 1 + alpha cos(m theta - shift), shift in
    {0, pi/2, pi}, from polynomials of the unit normal n = p / |p| (no trigonometry of theta)."""
    mag = np.hypot(pg[0], pg[1])
    nx, ny = pg[0] / mag, pg[1] / mag
    cos_m = _cheb_T(m, nx)
    sin_m = ny * _cheb_U(m, nx)
    if shift == 0.0:
        g, dg = cos_m, -m * sin_m            # d/dtheta cos(m theta) = -m sin(m theta)
    elif shift == "half":                    # cos(m theta - pi/2) = sin(m theta)
        g, dg = sin_m, m * cos_m
    else:                                    # cos(m theta - pi) = -cos(m theta)
        g, dg = -cos_m, m * sin_m
    gamma = 1.0 + alpha * g
    proj = alpha * dg * np.stack([-ny, nx]) * mag
    return gamma, proj


CASES = [  # (m, theta0, shift of m*theta0)
    (6, 0.0, 0.0),
    (4, math.pi / 8, "half"),
    (6, math.pi / 12, "half"),
    (4, math.pi / 4, "pi"),
    (6, math.pi / 6, "pi"),
]


def _aniso_error(fn, m, theta0, shift):
    alpha = 0.27
    pg = RNG.normal(size=(2, 400)) * 0.7
    pg = pg[:, np.hypot(pg[0], pg[1]) > 1e-3]
    p = lbm.Params(nx=8, ny=8, kappa=K39, beta=B39, alpha=alpha, aniso_m=m, theta0=theta0)
    gamma, proj = fn(pg, p)
    g_want, p_want = _closed_form(pg, alpha, m, shift)
    return max(np.abs(gamma - g_want).max(), np.abs(proj - p_want).max() / np.abs(p_want).max())


@pytest.mark.parametrize("m,theta0,shift", CASES)
def test_anisotropy_matches_chebyshev_closed_forms(m, theta0, shift):
    assert _aniso_error(lbm.anisotropy, m, theta0, shift) < 1e-13


def test_anisotropy_quarter_turn_orientation_flips_eq6_polynomial():
    # m = 4, theta0 = pi/4: gamma = 1 - alpha cos 4 theta = 1 - alpha (4 sum n^4 - 3), and the
    # tangential term is the negative of the eq 6 form's (I - n n^T) 16 alpha n^3 |p|
    pg = RNG.normal(size=(2, 300))
    p0 = lbm.Params(nx=8, ny=8, kappa=K39, beta=B39, alpha=0.2)
    p1 = lbm.Params(nx=8, ny=8, kappa=K39, beta=B39, alpha=0.2, theta0=math.pi / 4)
    g0, j0 = lbm.anisotropy(pg, p0)
    g1, j1 = lbm.anisotropy(pg, p1)
    assert np.abs((g1 - 1.0) + (g0 - 1.0)).max() < 1e-14
    assert np.abs(j1 + j0).max() < 1e-13 * np.abs(j0).max()


@pytest.mark.parametrize("m", [4, 6])
def test_anisotropy_rotation_covariance(m):
    # rotating the gradient by psi and the orientation by psi rotates the tangential term by
    # psi and leaves gamma unchanged
    pg = RNG.normal(size=(2, 300))
    for psi, theta0 in [(0.37, 0.0), (math.pi / 2, 0.21), (2.1, -0.8)]:
        R = np.array([[math.cos(psi), -math.sin(psi)], [math.sin(psi), math.cos(psi)]])
        pa = lbm.Params(nx=8, ny=8, kappa=K39, beta=B39, alpha=0.3, aniso_m=m, theta0=theta0)
        pb = lbm.Params(nx=8, ny=8, kappa=K39, beta=B39, alpha=0.3, aniso_m=m, theta0=theta0 + psi)
        ga, ja = lbm.anisotropy(pg, pa)
        gb, jb = lbm.anisotropy(R @ pg, pb)
        assert np.abs(ga - gb).max() < 1e-13
        assert np.abs(R @ ja - jb).max() < 1e-13 * np.abs(ja).max()


# cos(m (theta + theta0)) equals cos(m (theta - theta0)) when m theta0 is a multiple of pi, so
# the orientation slip is planted only where m theta0 = pi/2
PLANTS = [(c, "theta_plus_theta0") for c in CASES if c[2] == "half"] + [(c, "tangent_sign") for c in CASES]


@pytest.mark.parametrize("case,planted", PLANTS)
def test_anisotropy_pins_catch_planted_mistakes(case, planted, monkeypatch):
    m, theta0, shift = case
    orig = lbm.anisotropy
    if planted == "theta_plus_theta0":
        # cos(m (theta + theta0)) is the correct function called with -theta0
        def wrong(pg, p):
            import dataclasses
            return orig(pg, dataclasses.replace(p, theta0=-p.theta0))
    else:
        def wrong(pg, p):
            g, proj = orig(pg, p)
            return g, -proj
    monkeypatch.setattr(lbm, "anisotropy", wrong)
    assert _aniso_error(lbm.anisotropy, m, theta0, shift) > 1e-2
