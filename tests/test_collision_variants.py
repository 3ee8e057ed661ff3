"""Collision variants on D2Q9 (Section 3: the paper prefers MRT for stability): the oracle's
SRT and TRT rate choices pinned to the textbook single- and two-relaxation-time updates, and
the library's presets (host-only C calls) against the oracle's."""
import numpy as np
import pytest

from oracle import lbm
from tests import common

RNG = np.random.default_rng(17)


def _state(p):
    phi = 0.3 * RNG.standard_normal((6, 7))
    cp = lbm.chemical_potentials(phi, p)
    feq = lbm.equilibrium(phi, cp["mu_alpha"])
    f = feq + 0.01 * RNG.standard_normal(feq.shape)
    f += (phi - lbm.phi_of(f))[None] / 9.0                     # phi of f equals phi
    F = lbm.source(lbm.grad(cp["mu_beta"], p), p)
    return f, feq, F


def _opposite():
    E = lbm.E
    return [int(np.flatnonzero((E[0] == -E[0, i]) & (E[1] == -E[1, i]))[0]) for i in range(9)]


def _params(**kw):
    kappa, beta = lbm.kappa_beta_from_sigma_width(0.01, 5.0)
    args = dict(nx=7, ny=6, kappa=kappa, beta=beta, alpha=0.3)
    args.update(kw)
    return lbm.Params(**args)


@pytest.mark.parametrize("magic", [1.0 / 4.0, 1.0 / 12.0, 3.0 / 16.0])
@pytest.mark.parametrize("mobility", [0.02, 0.1, 1.0])
def test_trt_rates_give_the_textbook_two_relaxation_time_update(magic, mobility):
    # f_i = f+_i + f-_i with f+-_i = (f_i +- f_opp(i)) / 2; the even part relaxes at s+, the odd
    # part at s-, each with its (1 - s/2) forcing weight
    p = _params(mobility=mobility)
    p.s_free = lbm.collision_free_rates("trt", p, magic)
    s_minus = lbm.relaxation_rates(p)[3]
    s_plus = p.s_free[1]
    assert abs((1.0 / s_plus - 0.5) * (1.0 / s_minus - 0.5) - magic) <= 1e-14
    f, feq, F = _state(p)
    opp = _opposite()
    even = lambda a: 0.5 * (a + a[opp])
    odd = lambda a: 0.5 * (a - a[opp])
    want = (f - s_plus * (even(f) - even(feq)) - s_minus * (odd(f) - odd(feq))
            + p.dt * ((1.0 - s_plus / 2.0) * even(F) + (1.0 - s_minus / 2.0) * odd(F)))
    got = lbm.collide(f, feq, F, p)
    assert np.abs(got - want).max() <= 1e-14


@pytest.mark.parametrize("mobility", [0.02, 0.1, 1.0])
def test_srt_rates_give_bgk(mobility):
    p = _params(mobility=mobility)
    p.s_free = lbm.collision_free_rates("srt", p)
    s = lbm.relaxation_rates(p)[3]
    f, feq, F = _state(p)
    want = f - s * (f - feq) + (1.0 - s / 2.0) * p.dt * F
    assert np.abs(lbm.collide(f, feq, F, p) - want).max() <= 1e-14


def test_trt_with_equal_rates_is_srt():
    p = _params(mobility=0.1)
    s_j = lbm.relaxation_rates(p)[3]
    trt = lbm.collision_free_rates("trt", p, (1.0 / s_j - 0.5) ** 2)
    assert np.allclose(trt, lbm.collision_free_rates("srt", p), rtol=0, atol=1e-15)


def lb():
    from paper_2501_03759_amd import lbch
    return lbch


@pytest.mark.parametrize("units", [(1.0, 1.0), (0.5, 0.25), (2.0, 3.0)])
@pytest.mark.parametrize("mobility", [0.02, 0.1, 1.0])
@pytest.mark.parametrize("model,name,magic", [(0, "mrt", 0.25), (1, "srt", 0.25), (2, "trt", 0.25),
                                              (2, "trt", 1.0 / 12.0)])
def test_library_presets_match_oracle(units, mobility, model, name, magic):
    L = lb()
    dx, dt = units
    p = L.set_collision(L.default_params(mobility=mobility, dx=dx, dt=dt, s=(0.7,) * 9), model, magic)
    op = common.oracle_params(p)
    want = lbm.collision_free_rates(name, op, magic)
    assert np.abs(np.array(p.s[:]) - np.array(want)).max() <= 1e-15
    assert L.validate(p) == L.OK


def test_library_preset_errors():
    L = lb()
    p = L.default_params(s=(0.7,) * 9)
    for model, magic in [(3, 0.25), (-1, 0.25), (2, 0.0), (2, -1.0), (2, float("nan")), (2, float("inf"))]:
        with pytest.raises(L.LbchError) as ei:
            L.set_collision(p, model, magic)
        assert ei.value.status == L.E_INVALID
        assert p.s[1] == 0.7                                     # unchanged on error
    q = L.set_collision(L.default_params(lattice=L.D3Q15, nz=8), L.COLLISION_SRT)
    assert L.validate(q) == L.OK                                 # one rate per parity class
    q.s[7] = 0.9
    assert L.validate(q) == L.E_UNSUPPORTED                      # even rows at two rates
