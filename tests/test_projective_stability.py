"""Stability of the projective correction steps of the hybrid schedule, on the exact
linearised lattice Boltzmann step (the 9x9 amplification matrix of the oracle).

After n plain steps (run two per launch), the populations are advanced by
f <- f + (J/2)(f_n - f_{n-2}).  Per eigenmode (eigenvalue lam of one step) that is
lam^(n-2) (lam^2 + (J/2)(lam^2 - 1)): every mode except the slow one must shrink,
and the slow one must follow lam^(n+J) to first order.  The schedule's default
(n, J) = (4, 16) is stable; shorter plain phases are not (the flux mode, eigenvalue
1 - s_j = -0.25, is amplified)."""
import numpy as np
import pytest

from oracle import lbm, linear
from paper_2501_03759_amd import inputs


@pytest.fixture(scope="module")
def spectra():
    d = inputs.C5
    kappa, beta = lbm.kappa_beta_from_sigma_width(inputs.SIGMA_PAPER, inputs.width_from_eps(d["eps_w"]))
    p = lbm.Params(nx=64, ny=64, kappa=kappa, beta=beta, mobility=d["mobility"], alpha=0.0, eps_reg=d["eps_reg"])
    qs = np.linspace(0.0, np.pi, 25)
    out = []
    for phib in (1.0, 0.6):
        for qx in qs:
            for qy in qs[qs <= qx + 1e-12]:
                out.append(np.linalg.eigvals(linear.amplification(p, phib, qx, qy)))
    return out


def worst_gain(spectra, n, jump):
    worst = 0.0
    for lam in spectra:
        g = lam ** (n - 2) * (lam ** 2 + 0.5 * jump * (lam ** 2 - 1.0))
        slow = np.argmin(np.abs(lam - 1.0))
        for j in range(lam.size):
            if j == slow and abs(lam[j]) > 1.0 - 1e-3:
                continue            # the conserved / slow mode itself
            worst = max(worst, abs(g[j]))
    return worst


def test_default_inner_step_is_stable(spectra):
    assert worst_gain(spectra, 4, 16) < 1.0
    assert worst_gain(spectra, 4, 12) < 1.0


def test_short_plain_phase_is_unstable(spectra):
    assert worst_gain(spectra, 2, 8) > 1.5


def test_longest_stable_jump_after_four_plain_steps(spectra):
    # 4 + 20 is the last stable inner cycle after four plain steps; 4 + 24 amplifies
    assert worst_gain(spectra, 4, 20) < 1.0
    assert worst_gain(spectra, 4, 24) > 1.1


def test_slow_mode_first_order(spectra):
    # slow modes (|1 - lam| < 1e-3): the projective step reproduces lam^(n+J) to O(((n+J)(1-lam))^2)
    for lam in spectra:
        l = lam[np.argmin(np.abs(lam - 1.0))]
        eps = abs(1.0 - l)
        if eps < 1e-3:
            g = l ** 2 * (l ** 2 + 8.0 * (l ** 2 - 1.0))
            assert abs(g - l ** 20) <= 2.0 * (20 * eps) ** 2 + 1e-12
