"""Pins of the three-dimensional (D3Q15) oracle: lattice moments (eq 21, 27), the
Gram-Schmidt moment basis, exact stencil symbols (eq 26), the cubic anisotropy of
eq 6 with d = 3, collision special cases, and whole-step invariants and dispersion."""
import math

import numpy as np
import pytest

from oracle import lbm, lbm3, linear

RNG = np.random.default_rng(77)
K39, B39 = lbm.kappa_beta_from_sigma_width(0.01, 5.0)


def _p(**kw):
    base = dict(nx=6, ny=5, nz=4, kappa=K39, beta=B39, mobility=0.1)
    base.update(kw)
    return lbm3.Params(**base)


def test_weight_moments_eq27a_and_fourth_order_isotropy():
    w, c = lbm3.WEIGHTS, lbm3.E.astype(float)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(c @ w).max() < 1e-15
    assert np.abs((c * w) @ c.T - np.eye(3) / 3.0).max() < 1e-15
    # fourth moments of an isotropic lattice: c_s^4 (d_ab d_cd + d_ac d_bd + d_ad d_bc)
    for a in range(3):
        assert abs((w * c[a] ** 4).sum() - 1.0 / 3.0) < 1e-15
        for b in range(3):
            if a != b:
                assert abs((w * c[a] ** 2 * c[b] ** 2).sum() - 1.0 / 9.0) < 1e-15


def test_moment_basis_is_orthogonal_with_flux_rows():
    M = lbm3.M_MATRIX
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() < 1e-12
    assert np.linalg.matrix_rank(M) == 15
    assert np.array_equal(M[0], np.ones(15))
    for r, a in zip(lbm3.J_ROWS, range(3)):
        assert np.array_equal(M[r], lbm3.E[a].astype(float))


def test_equilibrium_and_source_moments_eq27bc():
    phi, mua = RNG.normal(size=7), RNG.normal(size=7)
    feq = lbm3.equilibrium(phi, mua)
    c = lbm3.E.astype(float)
    assert np.allclose(feq.sum(0), phi, atol=1e-14)
    assert np.allclose(c @ feq, 0.0, atol=1e-14)
    second = np.einsum("ai,bi,in->abn", c, c, feq)
    assert np.allclose(second, np.einsum("ab,n->abn", np.eye(3), mua / 3.0), atol=1e-14)
    g = RNG.normal(size=(3, 7))
    F = lbm3.source(g, _p())
    assert np.allclose(F.sum(0), 0.0, atol=1e-15)
    assert np.allclose(c @ F, -g / 3.0, atol=1e-15)


def test_stencil_symbols_every_mode():
    # eq 26 on D3Q15 in Fourier space (derived by hand from the weights):
    #   grad_x: i (2/3) sin kx (1 + cos ky cos kz / 2)
    #   lap   : (4/3)(cos kx + cos ky + cos kz - 3) + (2/3)(cos kx cos ky cos kz - 1)
    p = _p(nx=6, ny=5, nz=4)
    chi = RNG.normal(size=(4, 5, 6))
    kz, ky, kx = np.meshgrid(2 * np.pi * np.fft.fftfreq(4), 2 * np.pi * np.fft.fftfreq(5),
                             2 * np.pi * np.fft.fftfreq(6), indexing="ij")
    X = np.fft.fftn(chi)
    gx = 1j * (2 / 3) * np.sin(kx) * (1 + 0.5 * np.cos(ky) * np.cos(kz))
    gy = 1j * (2 / 3) * np.sin(ky) * (1 + 0.5 * np.cos(kx) * np.cos(kz))
    gz = 1j * (2 / 3) * np.sin(kz) * (1 + 0.5 * np.cos(kx) * np.cos(ky))
    L = (4 / 3) * (np.cos(kx) + np.cos(ky) + np.cos(kz) - 3) + (2 / 3) * (np.cos(kx) * np.cos(ky) * np.cos(kz) - 1)
    g = lbm3.grad(chi, p)
    for a, sym in enumerate((gx, gy, gz)):
        assert np.abs(g[a] - np.fft.ifftn(sym * X).real).max() < 1e-13
    assert np.abs(lbm3.laplacian(chi, p) - np.fft.ifftn(L * X).real).max() < 1e-13


def test_stencils_exact_on_quadratics():
    p = _p(nx=12, ny=12, nz=12)
    z, y, x = np.meshgrid(*(np.arange(12.0),) * 3, indexing="ij")
    lin = 0.3 * x - 0.7 * y + 0.2 * z
    g = lbm3.grad(lin, p)[:, 2:-2, 2:-2, 2:-2]           # away from the periodic seam
    assert np.allclose(g[0], 0.3) and np.allclose(g[1], -0.7) and np.allclose(g[2], 0.2)
    quad = x * x + 2 * y * y - z * z + x * y
    assert np.allclose(lbm3.laplacian(quad, p)[2:-2, 2:-2, 2:-2], 2 + 4 - 2)


def test_anisotropy_in_plane_reduces_to_eq6_and_2d_projection():
    p3, p2 = _p(alpha=0.23), lbm.Params(nx=4, ny=4, kappa=K39, beta=B39, alpha=0.23)
    pg2 = RNG.normal(size=(2, 300))
    pg3 = np.vstack([pg2, np.zeros((1, 300))])
    g3, pr3 = lbm3.anisotropy(pg3, p3)
    g2, pr2 = lbm.anisotropy(pg2, p2)
    theta = np.arctan2(pg2[1], pg2[0])
    assert np.abs(g3 - (1 + 0.23 * np.cos(4 * theta))).max() < 1e-14
    assert np.abs(pr3[:2] - pr2).max() < 1e-14 and np.abs(pr3[2]).max() < 1e-15


def test_Q_is_gradient_of_energy_density_3d():
    p = _p(alpha=0.3)
    pg = RNG.normal(size=(3, 200)) * 0.3
    F0 = 0.5 * p.kappa * (pg ** 2).sum(0)
    Q = lbm3.vector_Q(pg, p)
    h = 1e-6
    fd = np.zeros_like(pg)
    for a in range(3):
        d = np.zeros_like(pg)
        d[a] = h
        vals = []
        for sgn in (1, -1):
            q = pg + sgn * d
            g, _ = lbm3.anisotropy(q, p)
            vals.append(g * (0.5 * p.kappa * (q ** 2).sum(0) + F0))
        fd[a] = (vals[0] - vals[1]) / (2 * h)
    assert np.abs(Q - fd).max() < 1e-8 * np.abs(fd).max()
    # projection is tangential
    _, proj = lbm3.anisotropy(pg, p)
    assert np.abs((proj * pg).sum(0)).max() < 1e-13


def _rand_state(n=20):
    f = RNG.normal(size=(15, n)) * 0.1 + 0.05
    feq = lbm3.equilibrium(f.sum(0), RNG.normal(size=n) * 0.01)     # the equilibrium of the node's own phi
    F = lbm3.source(RNG.normal(size=(3, n)) * 0.01, _p())
    return f, feq, F


def test_collision_unit_free_rates_closed_form_and_basis_independence():
    # with every free rate 1 the post-collision state is f_eq + F/2 plus the relaxed flux,
    # (1 - s_j) / |flux row|^2 sum_a c_ia (j_a + F_m,a / 2), |flux row|^2 = 10 on D3Q15
    p = _p()
    f, feq, F = _rand_state()
    post = lbm3.collide(f, feq, F, p)
    s_j = lbm3.relaxation_rates(p)[3]
    c = lbm3.E.astype(float)
    j = c @ f
    Fm = c @ F
    closed = feq + 0.5 * F + (1.0 - s_j) / 10.0 * (c.T @ (j + 0.5 * Fm))
    assert np.abs(post - closed).max() < 1e-14
    # any orthogonal basis with the same conserved and flux rows gives the same result
    Q, _ = np.linalg.qr(RNG.normal(size=(11, 11)))
    others = [r for r in range(15) if r not in (0,) + lbm3.J_ROWS]
    M2 = lbm3.M_MATRIX.copy()
    norm = np.sqrt((M2[others] ** 2).sum(1, keepdims=True))
    M2[others] = Q @ (M2[others] / norm)
    assert np.abs(lbm3.collide(f, feq, F, p, M2) - post).max() < 1e-13
    # ... which stops being true once a free rate is not 1 (the basis then matters)
    pd = _p(s_free=(1.0,) * 9 + (1.4,) + (1.0,) * 5)
    assert np.abs(lbm3.collide(f, feq, F, pd, M2) - lbm3.collide(f, feq, F, pd)).max() > 1e-6


def test_collision_conserves_phi_and_equal_rates_is_bgk():
    f, feq, F = _rand_state()
    p = _p(s_free=(0.7,) * 15, mobility=1.0 / 3.0 * (1 / 0.7 - 0.5))
    assert abs(lbm3.relaxation_rates(p)[3] - 0.7) < 1e-14
    post = lbm3.collide(f, feq, F, p)
    assert np.allclose(post.sum(0), f.sum(0), atol=1e-14)
    assert np.abs(post - (f - 0.7 * (f - feq) + (1 - 0.35) * F)).max() < 1e-14


EVEN_ROWS = (1, 2, 9, 10, 11, 12, 13)     # even in c: e, eps and the five second-order rows
ODD_ROWS = (4, 6, 8, 14)                   # odd, not fluxes: |c|^2 c_a and c_x c_y c_z


def _class_rates(s_e, s_q):
    s = [1.0] * 15
    for r in EVEN_ROWS:
        s[r] = s_e
    for r in ODD_ROWS:
        s[r] = s_q
    return tuple(s)


def test_basis_rows_split_by_parity():
    # the even rows span the vectors symmetric under c -> -c, the odd rows the antisymmetric
    M = lbm3.M_MATRIX
    opp = [int(np.flatnonzero((lbm3.E == -lbm3.E[:, [i]]).all(0))[0]) for i in range(15)]
    for r in (0,) + EVEN_ROWS:
        assert np.array_equal(M[r], M[r][opp])
    for r in lbm3.J_ROWS + ODD_ROWS:
        assert np.array_equal(M[r], -M[r][opp])


def test_collision_trt_is_the_textbook_two_rate_update():
    # even rows at s_+, odd rows at s_j: the symmetric / antisymmetric update with each part
    # of the source scaled by its own (1 - s / 2)
    p0 = _p(mobility=0.05)
    s_j = lbm3.relaxation_rates(p0)[3]
    s_p = 1.37
    p = _p(mobility=0.05, s_free=_class_rates(s_p, s_j))
    f, feq, F = _rand_state()
    opp = [int(np.flatnonzero((lbm3.E == -lbm3.E[:, [i]]).all(0))[0]) for i in range(15)]
    sym = lambda a: 0.5 * (a + a[opp])
    asym = lambda a: 0.5 * (a - a[opp])
    ref = (f - s_p * (sym(f) - sym(feq)) - s_j * (asym(f) - asym(feq))
           + (1 - s_p / 2) * sym(F) + (1 - s_j / 2) * asym(F))
    assert np.abs(lbm3.collide(f, feq, F, p) - ref).max() < 1e-14


def test_collision_three_class_rates_closed_form():
    # even rows at s_e, fluxes at s_j, other odd rows at s_q: with f_eq even and the source
    # odd, f* = f_eq + (1 - s_e)(f+ - f_eq) + (1 - s_q) f- + (1 - s_q / 2) F
    #           + (s_q - s_j) / 10 e_i.(j + F_m / 2)
    p = _p(mobility=0.2, s_free=_class_rates(1.3, 0.8))
    s_j = lbm3.relaxation_rates(p)[3]
    f, feq, F = _rand_state()
    opp = [int(np.flatnonzero((lbm3.E == -lbm3.E[:, [i]]).all(0))[0]) for i in range(15)]
    assert np.abs(feq - feq[opp]).max() == 0 and np.abs(F + F[opp]).max() < 1e-18
    c = lbm3.E.astype(float)
    j, Fm = c @ f, c @ F
    closed = (feq + (1 - 1.3) * (0.5 * (f + f[opp]) - feq) + (1 - 0.8) * 0.5 * (f - f[opp])
              + (1 - 0.8 / 2) * F + (0.8 - s_j) / 10.0 * (c.T @ (j + 0.5 * Fm)))
    assert np.abs(lbm3.collide(f, feq, F, p) - closed).max() < 1e-14
    # and a change of any one odd non-flux rate alone changes the result
    for r in ODD_ROWS:
        s = list(_class_rates(1.3, 0.8))
        s[r] = 0.9
        assert np.abs(lbm3.collide(f, feq, F, _p(mobility=0.2, s_free=tuple(s))) - closed).max() > 1e-6


@pytest.fixture(scope="module")
def droplet_run():
    n = 14
    p = lbm3.Params(nx=n, ny=n, nz=n, kappa=K39, beta=B39, mobility=0.1, alpha=0.2)
    z, y, x = np.meshgrid(*(np.arange(n, dtype=float),) * 3, indexing="ij")
    r = np.sqrt((x - n // 2) ** 2 + (y - n // 2) ** 2 + (z - n // 2) ** 2)
    phi0 = np.tanh(2 * (4.5 - r) / 5.0)
    f = lbm3.initial_populations(phi0, p)
    E, M = [lbm3.free_energy(f, p)], [lbm3.mass(f, p)]
    for _ in range(60):
        f = lbm3.step(f, p)
        E.append(lbm3.free_energy(f, p))
        M.append(lbm3.mass(f, p))
    return f, np.array(E), np.array(M)


def test_mass_conserved_3d(droplet_run):
    f, _, M = droplet_run
    assert np.abs(M - M[0]).max() / np.abs(lbm3.phi_of(f)).sum() < 1e-12


def test_energy_non_increasing_3d(droplet_run):
    _, E, _ = droplet_run
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))


def test_cubic_symmetry_about_centre_node(droplet_run):
    phi = lbm3.phi_of(droplet_run[0])
    c = phi.shape[0] // 2
    assert np.abs(phi - phi.transpose(0, 2, 1)).max() < 1e-13
    assert np.abs(phi - phi.transpose(2, 1, 0)).max() < 1e-13
    mirrored = np.roll(phi[:, :, ::-1], 2 * c + 1 - phi.shape[2], axis=2)
    assert np.abs(phi - mirrored).max() < 1e-13


def _measured_rate(p, mode, n0=100, n1=1600):
    x = np.arange(p.nx, dtype=float)
    phi0 = 1.0 + 1e-7 * np.broadcast_to(np.cos(2 * np.pi * mode * x / p.nx), (p.nz, p.ny, p.nx)).copy()
    f = lbm3.initial_populations(phi0, p)
    amp = {}
    for n in range(n1 + 1):
        if n in (n0, n1):
            amp[n] = np.abs(np.fft.fft(lbm3.phi_of(f)[0, 0] - 1.0)[mode])
        f = lbm3.step(f, p)
    return math.log(amp[n1] / amp[n0]) / (n1 - n0)


@pytest.mark.parametrize("planted", ["none", "flipped_source"])
def test_dispersion_3d_catches_planted_mistakes(planted, monkeypatch):
    # a Fourier mode along x about phi = 1 decays at the rate of the recovered PDE
    # (isotropic limit; eps_reg = 0.3 makes the source term a leading part of the rate)
    good = lbm3.source
    if planted == "flipped_source":
        monkeypatch.setattr(lbm3, "source", lambda g, p: -good(g, p))
    p = lbm3.Params(nx=128, ny=2, nz=2, kappa=K39, beta=B39, mobility=0.1, eps_reg=0.3)
    q = 2 * np.pi * 2 / 128
    p2 = lbm.Params(nx=128, ny=2, kappa=K39, beta=B39, mobility=0.1, eps_reg=0.3)
    rel = abs(_measured_rate(p, 2) / linear.continuum_rate(p2, 1.0, q * q) - 1.0)
    if planted == "none":
        assert rel < 3e-4
    else:
        assert not rel < 1e-3
