"""Pins of the oracle's pointwise pieces: anisotropy (eqs 2, 6, 14, 15), equilibrium and
source moments (eqs 18, 19, 27b, 27c) and the collision (eq 17) special cases."""
import numpy as np
import pytest

from oracle import lbm

RNG = np.random.default_rng(1234)


def _p(**kw):
    base = dict(nx=8, ny=8, kappa=0.0212, beta=0.00133, mobility=0.1)
    base.update(kw)
    return lbm.Params(**base)


def test_eq6_polynomial_equals_cos4theta():
    p = _p(alpha=0.27)
    pg = RNG.normal(size=(2, 500))
    gamma, _ = lbm.anisotropy(pg, p)
    theta = np.arctan2(pg[1], pg[0])
    assert np.abs(gamma - (1 + 0.27 * np.cos(4 * theta))).max() < 1e-14


def _energy_density_fd(pg, p, F0):
    """Q of eq 14 is d/d(grad phi) of gamma(n)(kappa/2 |grad phi|^2 + F); central differences
    with F frozen at F0 (the eq 15 approximation sets F0 = kappa |grad phi|^2 / 2)."""
    h = 1e-6
    out = np.zeros_like(pg)
    for a in range(2):
        d = np.zeros_like(pg)
        d[a] = h
        vals = []
        for sgn in (1, -1):
            q = pg + sgn * d
            g, _ = lbm.anisotropy(q, p)
            vals.append(g * (0.5 * p.kappa * (q[0] ** 2 + q[1] ** 2) + F0))
        out[a] = (vals[0] - vals[1]) / (2 * h)
    return out


@pytest.mark.parametrize("m,theta0", [(4, 0.0), (6, 0.0), (4, 0.4), (6, 1.3)])
def test_Q_is_gradient_of_energy_density(m, theta0):
    p = _p(alpha=0.3, aniso_m=m, theta0=theta0)
    pg = RNG.normal(size=(2, 200)) * 0.3
    pg = pg[:, np.hypot(pg[0], pg[1]) > 0.05]
    F0 = 0.5 * p.kappa * (pg[0] ** 2 + pg[1] ** 2)
    Q = lbm.vector_Q(pg, p)
    fd = _energy_density_fd(pg, p, F0)
    assert np.abs(Q - fd).max() < 1e-8 * np.abs(fd).max()


def test_Q_literal_form_drops_kappa_on_tangential_term():
    p = _p(alpha=0.2)
    pg = RNG.normal(size=(2, 50))
    qd = lbm.vector_Q(pg, p)
    pl = _p(alpha=0.2, q_form="literal")
    ql = lbm.vector_Q(pg, pl)
    gamma, proj = lbm.anisotropy(pg, p)
    assert np.allclose(qd - gamma * p.kappa * pg, p.kappa * (ql - gamma * p.kappa * pg), rtol=1e-13, atol=1e-16)


def test_floor_reading_zero_gradient():
    p = _p(alpha=0.3)
    pg = np.zeros((2, 3))
    gamma, proj = lbm.anisotropy(pg, p)
    assert np.all(gamma == 1.0) and np.all(proj == 0.0)
    assert np.all(lbm.vector_Q(pg, p) == 0.0)


def test_isotropic_limit_Q():
    p = _p(alpha=0.0)
    pg = RNG.normal(size=(2, 40))
    assert np.allclose(lbm.vector_Q(pg, p), p.kappa * pg, rtol=1e-15, atol=0)


def test_equilibrium_moments_eq27b():
    phi = RNG.normal(size=(5, 6))
    mu_a = RNG.normal(size=(5, 6))
    feq = lbm.equilibrium(phi, mu_a)
    e = lbm.E.astype(float)
    assert np.abs(feq.sum(0) - phi).max() < 1e-14
    assert np.abs(np.einsum("ai,iyx->ayx", e, feq)).max() < 1e-14
    second = np.einsum("ai,bi,iyx->abyx", e, e, feq)
    cs2 = 1.0 / 3.0
    for a in range(2):
        for b in range(2):
            want = cs2 * mu_a if a == b else 0 * mu_a
            assert np.abs(second[a, b] - want).max() < 1e-14


def test_source_moments_eq27c():
    p = _p()
    g = RNG.normal(size=(2, 4, 7))
    F = lbm.source(g, p)
    e = lbm.E.astype(float)
    assert np.abs(F.sum(0)).max() < 1e-15
    first = np.einsum("ai,iyx->ayx", e, F)
    assert np.abs(first + g / 3.0).max() < 1e-15


def test_moment_space_closed_forms():
    # Hand-derived: M f_eq = (phi, -4phi + 2mu_a, 4phi - 3mu_a, 0, ...); M F = (0,0,0,-gx/3, gx/3, -gy/3, gy/3, 0, 0).
    p = _p()
    phi, mu_a = RNG.normal(size=20), RNG.normal(size=20)
    g = RNG.normal(size=(2, 20))
    meq = lbm.M_MATRIX @ lbm.equilibrium(phi, mu_a)
    want = np.zeros((9, 20))
    want[0], want[1], want[2] = phi, -4 * phi + 2 * mu_a, 4 * phi - 3 * mu_a
    assert np.abs(meq - want).max() < 1e-14
    mF = lbm.M_MATRIX @ lbm.source(g, p)
    want = np.zeros((9, 20))
    want[3], want[4], want[5], want[6] = -g[0] / 3, g[0] / 3, -g[1] / 3, g[1] / 3
    assert np.abs(mF - want).max() < 1e-15


def test_collision_conserves_phi():
    p = _p(s_free=(1.0, 1.1, 1.2, 1.0, 1.3, 1.0, 1.3, 1.4, 1.4))
    f = RNG.normal(size=(9, 4, 5))
    feq = lbm.equilibrium(f.sum(0), RNG.normal(size=(4, 5)))
    F = lbm.source(RNG.normal(size=(2, 4, 5)), p)
    post = lbm.collide(f, feq, F, p)
    assert np.abs(post.sum(0) - f.sum(0)).max() < 1e-13


def test_collision_equal_rates_is_textbook_bgk():
    s = 1.25
    p = _p(mobility=(1.0 / s - 0.5) / 3.0, s_free=(s,) * 9, alpha=0.2, nx=12, ny=10)
    rng = np.random.default_rng(5)
    phi0 = 0.3 * rng.normal(size=(10, 12))
    f = lbm.initial_populations(phi0, p)
    f = lbm.step(f, p)       # leave equilibrium
    a = lbm.step(f, p)
    b = lbm.srt_step(f, p, s)
    assert np.abs(a - b).max() < 1e-14


def test_collision_unit_rates_gives_feq_plus_half_source():
    p = _p(mobility=1.0 / 6.0)
    f = RNG.normal(size=(9, 3, 3))
    feq = lbm.equilibrium(f.sum(0), RNG.normal(size=(3, 3)))
    F = lbm.source(RNG.normal(size=(2, 3, 3)), p)
    assert np.abs(lbm.collide(f, feq, F, p) - (feq + 0.5 * F)).max() < 1e-14
