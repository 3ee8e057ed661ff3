"""Pseudo-spectral evaluation of the recovered macroscopic equation.

TEST INFRASTRUCTURE ONLY.  Independent of ``lbm``: derivatives are exact
Fourier multipliers, the anisotropy is evaluated through the angle
theta = atan2(phi_y, phi_x) (gamma = 1 + alpha cos(m(theta - theta0)),
gamma' = d gamma / d theta), and time is integrated with integrating-factor RK4.

Equations: CH equation eq 10 with the chemical potential of eq 11, the
regularisations of eqs 12/13 and the vector field Q under the eq 15
approximation (with the factor kappa implied by eq 14; q_form='literal'
keeps the printed eq 15).  Near-zero gradients follow the same floor reading
as the LB oracle (gamma = 1, no tangential term).
"""
from __future__ import annotations

import numpy as np


class SpectralCH:
    def __init__(self, n: int, length: float, kappa: float, beta: float, mobility: float,
                 alpha: float = 0.0, m: int = 4, theta0: float = 0.0,
                 reg: str = "willmore", eps_reg: float = 0.03, q_form: str = "derived",
                 grad_floor: float = 1e-10):
        self.n, self.length = n, length
        k = 2.0 * np.pi * np.fft.fftfreq(n, d=length / n)
        self.kx = k[None, :]
        self.ky = k[:, None]
        self.k2 = self.kx ** 2 + self.ky ** 2
        self.kappa, self.beta, self.mobility = kappa, beta, mobility
        self.alpha, self.m, self.theta0 = alpha, m, theta0
        self.reg, self.eps_reg, self.q_form, self.floor = reg, eps_reg, q_form, grad_floor

    # exact spectral derivatives of periodic real fields
    def dx(self, u):
        return np.real(np.fft.ifft2(1j * self.kx * np.fft.fft2(u)))

    def dy(self, u):
        return np.real(np.fft.ifft2(1j * self.ky * np.fft.fft2(u)))

    def lap(self, u):
        return np.real(np.fft.ifft2(-self.k2 * np.fft.fft2(u)))

    def f(self, phi):
        return 4.0 * self.beta * phi * (phi * phi - 1.0)

    def fp(self, phi):
        return 4.0 * self.beta * (3.0 * phi * phi - 1.0)

    def mu(self, phi):
        """Chemical potential (eq 11 with eq 13 / eq 12 and Q of eq 15)."""
        px, py = self.dx(phi), self.dy(phi)
        mag = np.hypot(px, py)
        live = mag > self.floor
        theta = np.arctan2(py, px)
        arg = self.m * (theta - self.theta0)
        gamma = np.where(live, 1.0 + self.alpha * np.cos(arg), 1.0)
        gprime = np.where(live, -self.alpha * self.m * np.sin(arg), 0.0)
        # |grad phi| P grad_n gamma = gamma'(theta) * (-phi_y, phi_x)
        tx, ty = -gprime * py, gprime * px
        if self.q_form == "derived":
            qx, qy = self.kappa * (gamma * px + tx), self.kappa * (gamma * py + ty)
        else:
            qx, qy = self.kappa * gamma * px + tx, self.kappa * gamma * py + ty
        f = self.f(phi)
        out = gamma * f - (self.dx(qx) + self.dy(qy))
        if self.reg == "willmore":
            w = self.lap(phi) - f
            out = out + self.eps_reg * (self.lap(w) - self.fp(phi) * w)
        elif self.reg == "linear":
            out = out + self.eps_reg * self.lap(self.lap(phi))
        return out

    def rhs(self, phi):
        """d phi / dt = div(M grad mu) (eq 10, constant mobility)."""
        return self.mobility * self.lap(self.mu(phi))

    def integrate(self, phi0, t_end: float, dt: float):
        """Integrating-factor (Lawson) RK4.

        The stiff linear part eps * Delta^2 phi of eqs 12/13 contributes
        -M eps k^6 to the Fourier symbol of the right-hand side; it is
        integrated exactly, the rest of mu explicitly with classical RK4.
        """
        nsteps = int(round(t_end / dt))
        assert abs(nsteps * dt - t_end) < 1e-9 * max(1.0, t_end)
        eps_lin = self.eps_reg if self.reg in ("willmore", "linear") else 0.0
        lam = -self.mobility * eps_lin * self.k2 ** 3
        e_half = np.exp(lam * dt / 2.0)
        e_full = e_half * e_half

        def nonlin_hat(phi_hat):
            phi = np.real(np.fft.ifft2(phi_hat))
            mu_rest = self.mu(phi) - eps_lin * self.lap(self.lap(phi))
            return -self.mobility * self.k2 * np.fft.fft2(mu_rest)

        u = np.fft.fft2(np.array(phi0, dtype=np.float64))
        for _ in range(nsteps):
            k1 = nonlin_hat(u)
            k2 = nonlin_hat(e_half * (u + 0.5 * dt * k1))
            k3 = nonlin_hat(e_half * u + 0.5 * dt * k2)
            k4 = nonlin_hat(e_full * u + dt * e_half * k3)
            u = e_full * u + dt / 6.0 * (e_full * k1 + 2.0 * e_half * (k2 + k3) + k4)
        return np.real(np.fft.ifft2(u))
