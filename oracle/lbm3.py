"""FP64 oracle of the scheme on the three-dimensional D3Q15 lattice.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The same method as
``lbm`` (Sections 2-3 of arXiv 2501.03759): phi = sum f_i (eq 22), the eq 26
stencils, the anisotropic chemical potential (eqs 13, 16), the modified
equilibrium (eq 18), the source (eq 19) and the MRT collision (eq 17), on the
D3Q15 velocities and weights of eq 21.  Plain and literal: dense 15 x 15
matrices, ``np.roll`` for every periodic shift.

Array conventions: a scalar field is ``chi[z, y, x]``; the populations are
``f[i, z, y, x]`` with i the D3Q15 direction of eq 21a; the state carried
between steps is the pre-collision population f_i(x, t).

Readings beyond those of ``lbm``:

* Moment matrix: eq 24 prints a 15 x 15 matrix (captioned for D3Q19) whose
  flux rows do not match the velocity order of eq 21a for the last two
  velocities.  The matrix is rebuilt as the paper says it is built: unweighted
  Gram-Schmidt orthogonalisation, over the fifteen velocities, of the
  polynomial basis 1, |c|^2, |c|^4, c_x, |c|^2 c_x, c_y, |c|^2 c_y, c_z,
  |c|^2 c_z, 3 c_x^2 - |c|^2, c_y^2 - c_z^2, c_x c_y, c_y c_z, c_x c_z,
  c_x c_y c_z.  Rows 3, 5, 7 are the fluxes c_x, c_y, c_z and relax at s_j
  from the mobility; the other rates are inputs (default 1).
* Anisotropy: eq 6 with d = 3, gamma = 1 + alpha (4 sum n_i^4 - 3), and
  grad_n gamma = 16 alpha n^3; only this cubic form is defined in 3D.
* Discrete free energy: eq 7 summed over nodes with the eq 26 stencils,
  times dx^3.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .lbm import REG_LINEAR, REG_NONE, REG_WILLMORE, bulk_F, bulk_f, bulk_fprime, kappa_beta_from_sigma_width  # noqa: F401

# eq 21a: D3Q15 directions (in units of c), columns i = 0..14.
E = np.array([[0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1],
              [0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1],
              [0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1]], dtype=np.int64)
# eq 21b: weights.
WEIGHTS = np.array([2 / 9] + [1 / 9] * 6 + [1 / 72] * 8, dtype=np.float64)
Q15 = 15
J_ROWS = (3, 5, 7)


def _moment_matrix() -> np.ndarray:
    cx, cy, cz = (E[a].astype(np.float64) for a in range(3))
    c2 = cx * cx + cy * cy + cz * cz
    basis = [np.ones(Q15), c2, c2 * c2, cx, c2 * cx, cy, c2 * cy, cz, c2 * cz,
             3 * cx * cx - c2, cy * cy - cz * cz, cx * cy, cy * cz, cx * cz, cx * cy * cz]
    rows = []
    for v in basis:
        w = v.copy()
        for r in rows:
            w = w - (w @ r) / (r @ r) * r
        rows.append(w)
    return np.array(rows)


M_MATRIX = _moment_matrix()
M_INV = np.linalg.inv(M_MATRIX)


@dataclasses.dataclass
class Params:
    nx: int
    ny: int
    nz: int
    kappa: float
    beta: float
    mobility: float = 0.1
    alpha: float = 0.0
    reg: str = REG_WILLMORE
    eps_reg: float = 0.03
    q_form: str = "derived"
    grad_floor: float = 1e-10
    dx: float = 1.0
    dt: float = 1.0
    s_free: tuple = (1.0,) * 15      # rates of the moments other than the fluxes (entries 3, 5, 7 ignored)

    @property
    def c(self) -> float:
        return self.dx / self.dt

    @property
    def cs2(self) -> float:
        return self.c * self.c / 3.0


def relaxation_rates(p: Params) -> np.ndarray:
    """Diagonal of S; the flux rates from M = c_s^2 (1/s - 1/2) dt (after eq 38)."""
    s = np.array(p.s_free, dtype=np.float64).copy()
    s_j = 1.0 / (p.mobility / (p.cs2 * p.dt) + 0.5)
    for r in J_ROWS:
        s[r] = s_j
    return s


# --------------------------------------------------------------- stencils --
def neighbour(chi: np.ndarray, i: int) -> np.ndarray:
    """chi(x + c_i dt), periodic."""
    return np.roll(chi, shift=(-int(E[2, i]), -int(E[1, i]), -int(E[0, i])), axis=(0, 1, 2))


def grad(chi: np.ndarray, p: Params) -> np.ndarray:
    """Eq 26a on D3Q15.  Returns [3, nz, ny, nx]."""
    out = np.zeros((3,) + chi.shape)
    for i in range(Q15):
        nb = neighbour(chi, i)
        for a in range(3):
            if E[a, i]:
                out[a] += WEIGHTS[i] * (E[a, i] * p.c) * nb
    return out / (p.cs2 * p.dt)


def laplacian(chi: np.ndarray, p: Params) -> np.ndarray:
    """Eq 26b on D3Q15."""
    out = np.zeros_like(chi)
    for i in range(Q15):
        out += 2.0 * WEIGHTS[i] * (neighbour(chi, i) - chi)
    return out / (p.cs2 * p.dt * p.dt)


def divergence(vec: np.ndarray, p: Params) -> np.ndarray:
    return grad(vec[0], p)[0] + grad(vec[1], p)[1] + grad(vec[2], p)[2]


# ------------------------------------------------------------- anisotropy --
def anisotropy(pg: np.ndarray, p: Params):
    """gamma(n) of eq 6 (d = 3) and |grad phi| P grad_n gamma (eq 14), n = grad phi / |grad phi| (eq 3)."""
    mag = np.sqrt(pg[0] ** 2 + pg[1] ** 2 + pg[2] ** 2)
    live = mag > p.grad_floor
    safe = np.where(live, mag, 1.0)
    n = pg / safe
    gamma = 1.0 + p.alpha * (4.0 * (n[0] ** 4 + n[1] ** 4 + n[2] ** 4) - 3.0)
    dg = 16.0 * p.alpha * n ** 3
    ndg = n[0] * dg[0] + n[1] * dg[1] + n[2] * dg[2]
    proj_unit = dg - n * ndg                        # P = I - n n^T
    gamma = np.where(live, gamma, 1.0)
    proj = np.where(live, proj_unit * mag, 0.0)
    return gamma, proj


def vector_Q(pg: np.ndarray, p: Params) -> np.ndarray:
    gamma, proj = anisotropy(pg, p)
    if p.q_form == "derived":
        return p.kappa * (gamma * pg + proj)
    if p.q_form == "literal":
        return gamma * p.kappa * pg + proj
    raise ValueError(p.q_form)


def chemical_potentials(phi: np.ndarray, p: Params) -> dict:
    pg = grad(phi, p)
    lap = laplacian(phi, p)
    f = bulk_f(phi, p)
    gamma, _ = anisotropy(pg, p)
    Q = vector_Q(pg, p)
    mu = gamma * f - divergence(Q, p)
    if p.reg == REG_WILLMORE:
        w = lap - f
        mu = mu + p.eps_reg * (laplacian(w, p) - bulk_fprime(phi, p) * w)
    elif p.reg == REG_LINEAR:
        mu = mu + p.eps_reg * laplacian(lap, p)
    elif p.reg != REG_NONE:
        raise ValueError(p.reg)
    mu_alpha = f - p.kappa * lap
    return {"grad_phi": pg, "lap_phi": lap, "gamma": gamma, "Q": Q, "mu": mu, "mu_alpha": mu_alpha,
            "mu_beta": mu - mu_alpha}


# ------------------------------------------------------------- LB pieces --
def equilibrium(phi: np.ndarray, mu_alpha: np.ndarray) -> np.ndarray:
    """Eq 18."""
    feq = WEIGHTS.reshape((Q15,) + (1,) * np.ndim(mu_alpha)) * mu_alpha[None]
    feq[0] = phi + (WEIGHTS[0] - 1.0) * mu_alpha
    return feq


def source(grad_mu_beta: np.ndarray, p: Params) -> np.ndarray:
    """Eq 19: F_i = -w_i c_i . grad(mu_beta)."""
    F = np.empty((Q15,) + grad_mu_beta.shape[1:])
    for i in range(Q15):
        F[i] = -WEIGHTS[i] * p.c * (E[0, i] * grad_mu_beta[0] + E[1, i] * grad_mu_beta[1] + E[2, i] * grad_mu_beta[2])
    return F


def collide(f: np.ndarray, feq: np.ndarray, F: np.ndarray, p: Params, M: np.ndarray | None = None) -> np.ndarray:
    """Right-hand side of eq 17 with literal matrices (M defaults to the Gram-Schmidt basis)."""
    M = M_MATRIX if M is None else M
    Minv = np.linalg.inv(M)
    S = np.diag(relaxation_rates(p))
    shape = f.shape
    flat = lambda a: a.reshape(Q15, -1)
    post = flat(f) - (Minv @ S @ M) @ (flat(f) - flat(feq)) + p.dt * ((Minv @ (np.eye(Q15) - S / 2.0) @ M) @ flat(F))
    return post.reshape(shape)


def stream(fpost: np.ndarray) -> np.ndarray:
    out = np.empty_like(fpost)
    for i in range(Q15):
        out[i] = np.roll(fpost[i], shift=(int(E[2, i]), int(E[1, i]), int(E[0, i])), axis=(0, 1, 2))
    return out


def initial_populations(phi0: np.ndarray, p: Params) -> np.ndarray:
    mu_alpha = bulk_f(phi0, p) - p.kappa * laplacian(phi0, p)
    return equilibrium(phi0, mu_alpha)


def phi_of(f: np.ndarray) -> np.ndarray:
    return f.sum(axis=0)


def step(f: np.ndarray, p: Params, M: np.ndarray | None = None) -> np.ndarray:
    phi = phi_of(f)
    cp = chemical_potentials(phi, p)
    g = grad(cp["mu_beta"], p)
    return stream(collide(f, equilibrium(phi, cp["mu_alpha"]), source(g, p), p, M))


def run(phi0: np.ndarray, p: Params, nsteps: int) -> np.ndarray:
    f = initial_populations(np.asarray(phi0, dtype=np.float64), p)
    for _ in range(nsteps):
        f = step(f, p)
    return f


def mass(f: np.ndarray, p: Params) -> float:
    return float(phi_of(f).sum() * p.dx ** 3)


def free_energy_terms(phi: np.ndarray, p: Params) -> dict:
    pg = grad(phi, p)
    gamma, _ = anisotropy(pg, p)
    vol = p.dx ** 3
    grad_term = float((gamma * 0.5 * p.kappa * (pg[0] ** 2 + pg[1] ** 2 + pg[2] ** 2)).sum() * vol)
    bulk_term = float((gamma * bulk_F(phi, p)).sum() * vol)
    if p.reg == REG_WILLMORE:
        G = (laplacian(phi, p) - bulk_f(phi, p)) ** 2
    elif p.reg == REG_LINEAR:
        G = laplacian(phi, p) ** 2
    else:
        G = np.zeros_like(phi)
    reg_term = float((0.5 * p.eps_reg * G).sum() * vol)
    return {"grad": grad_term, "bulk": bulk_term, "reg": reg_term, "total": grad_term + bulk_term + reg_term}


def free_energy(f: np.ndarray, p: Params) -> float:
    return free_energy_terms(phi_of(f), p)["total"]
