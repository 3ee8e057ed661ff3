"""FP64 oracle of the MRT lattice Boltzmann scheme for the anisotropic CH equation.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain, slow and literal:
dense 9x9 matrices, ``np.roll`` for every periodic shift, no fusion or
reordering beyond what the paper's equations state.

Paper: Liu, Wang & Liu, "Modelling anisotropic Cahn-Hilliard equation with the
lattice Boltzmann method" (arXiv 2501.03759).

Array conventions: a scalar field is ``chi[y, x]`` (ny rows of nx columns); the
populations are ``f[i, y, x]`` with i the D2Q9 direction of eq 20.  The state
carried between steps is the pre-collision (post-streaming) population
f_i(x, t) of eq 17, so that phi(t) = sum_i f_i(x, t) (eq 22).

Readings of passages the paper leaves silent or prints inconsistently (each is
a field of ``Params`` so the HIP path can be given the same reading):

* q_form='derived' (default): Q = kappa*(gamma*grad(phi) + |grad(phi)| P grad_n gamma).
  Eq 15 as printed drops the factor kappa that eq 14 together with the
  approximation F ~ kappa |grad phi|^2 / 2 implies; q_form='literal' keeps
  the printed eq 15.
* Free relaxation rates s_k (k not 3, 5) are not given: they are inputs,
  default 1.  s_3 = s_5 follow from the mobility (the relation after eq 38).
* Initial populations: equilibrium of eq 18 at phi0, no source term.
* |grad phi| <= grad_floor: gamma = 1 and the projected anisotropy term is 0
  (the normal of eq 2 is undefined there).
* Willmore term uses Delta(phi) - f(phi) exactly as eq 9/13 print it.
* m-fold anisotropy with orientation theta0 generalises eq 6:
  gamma = 1 + alpha cos(m (theta - theta0)); for m = 4, theta0 = 0 the
  oracle evaluates the literal eq 6 polynomial form instead.
* Discrete free energy: eq 7 summed over nodes with the eq 26 stencils for
  grad and Laplacian, the exact double well F (eq 4), gamma as above.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------- lattice --
# eq 20a: D2Q9 directions (in units of c), columns i = 0..8.
E = np.array([[0, 1, 0, -1, 0, 1, -1, -1, 1],
              [0, 0, 1, 0, -1, 1, 1, -1, -1]], dtype=np.int64)
# eq 20b: weights.
WEIGHTS = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)
Q9 = 9

# eq 23: the D2Q9 moment transform, rows (rho, e, eps, jx, qx, jy, qy, pxx, pxy).
M_MATRIX = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1],
], dtype=np.float64)
M_INV = np.linalg.inv(M_MATRIX)

REG_NONE, REG_LINEAR, REG_WILLMORE = "none", "linear", "willmore"


@dataclasses.dataclass
class Params:
    """Problem statement of Sections 2-3 (grid, rates, mobility, interface, anisotropy, regularisation)."""
    nx: int
    ny: int
    kappa: float
    beta: float
    mobility: float = 0.1            # eq 39
    alpha: float = 0.0               # eq 6 strength
    aniso_m: int = 4                 # eq 6 uses 4-fold
    theta0: float = 0.0
    reg: str = REG_WILLMORE          # Section 4 uses Willmore
    eps_reg: float = 0.03            # eq 39
    q_form: str = "derived"
    grad_floor: float = 1e-10
    dx: float = 1.0
    dt: float = 1.0
    s_free: tuple = (1.0,) * 9       # rates of moments other than j_x, j_y (entries 3, 5 ignored)

    @property
    def c(self) -> float:            # c = dx / dt (below eq 21)
        return self.dx / self.dt

    @property
    def cs2(self) -> float:          # c_s = c / sqrt(3)
        return self.c * self.c / 3.0


def kappa_beta_from_sigma_width(sigma: float, width: float) -> tuple[float, float]:
    """Invert eq 5: sigma = 4 sqrt(2 kappa beta) / 3, D = sqrt(2 kappa / beta)."""
    # From eq 5: sigma * D = 4/3 * sqrt(2 kappa beta) * sqrt(2 kappa / beta) = 8 kappa / 3,
    # and sigma / D = 4/3 * sqrt(2 kappa beta) / sqrt(2 kappa / beta) = 4 beta / 3.
    kappa = 3.0 * sigma * width / 8.0
    beta = 3.0 * sigma / (4.0 * width)
    return kappa, beta


def relaxation_rates(p: Params) -> np.ndarray:
    """Diagonal of S (eq 25); s_3 = s_5 from M = c_s^2 (1/s - 1/2) dt (after eq 38)."""
    s = np.array(p.s_free, dtype=np.float64).copy()
    s_j = 1.0 / (p.mobility / (p.cs2 * p.dt) + 0.5)
    s[3] = s_j
    s[5] = s_j
    return s


def collision_free_rates(model: str, p: Params, magic: float = 0.25) -> tuple:
    """Free rates of the collision variants, for the given mobility and lattice units.

    The paper picks MRT for stability (Section 3) without showing the alternatives:
    * 'mrt': every rate other than the fluxes' is 1 (the default reading of the free rates).
    * 'srt': one rate for every moment, the flux rate s_j (BGK).
    * 'trt': rates by parity under c -> -c: the moments even in c (rows 1, 2, 7, 8 of eq 23:
      e, eps, p_xx, p_xy) relax at s_plus, the odd ones (rows 3-6: j and q) at s_j, with
      the magic number (1/s_plus - 1/2)(1/s_j - 1/2) = magic.
    Entry 0 (phi, conserved) is set like the others and has no effect."""
    s_j = relaxation_rates(p)[3]
    if model == "mrt":
        return (1.0,) * 9
    if model == "srt":
        return (s_j,) * 9
    if model == "trt":
        s_plus = 1.0 / (0.5 + magic / (1.0 / s_j - 0.5))
        return (s_plus, s_plus, s_plus, s_j, s_j, s_j, s_j, s_plus, s_plus)
    raise ValueError(model)


# --------------------------------------------------------------- stencils --
def neighbour(chi: np.ndarray, i: int) -> np.ndarray:
    """chi(x + c_i dt) on the periodic grid (Section 4 uses periodic boundaries)."""
    return np.roll(chi, shift=(-int(E[1, i]), -int(E[0, i])), axis=(0, 1))


def grad(chi: np.ndarray, p: Params) -> np.ndarray:
    """Isotropic gradient eq 26a: sum_i w_i c_i chi(x + c_i dt) / (c_s^2 dt).  Returns [2, ny, nx]."""
    out = np.zeros((2,) + chi.shape)
    for i in range(Q9):
        nb = neighbour(chi, i)
        out[0] += WEIGHTS[i] * (E[0, i] * p.c) * nb
        out[1] += WEIGHTS[i] * (E[1, i] * p.c) * nb
    return out / (p.cs2 * p.dt)


def laplacian(chi: np.ndarray, p: Params) -> np.ndarray:
    """Isotropic Laplacian eq 26b: sum_i 2 w_i (chi(x + c_i dt) - chi(x)) / (c_s^2 dt^2)."""
    out = np.zeros_like(chi)
    for i in range(Q9):
        out += 2.0 * WEIGHTS[i] * (neighbour(chi, i) - chi)
    return out / (p.cs2 * p.dt * p.dt)


def divergence(vec: np.ndarray, p: Params) -> np.ndarray:
    """div of a vector field, eq 26a applied per component."""
    return grad(vec[0], p)[0] + grad(vec[1], p)[1]


# ------------------------------------------------------------ free energy --
def bulk_F(phi, p: Params):
    """Double-well potential eq 4."""
    return p.beta * (phi - 1.0) ** 2 * (phi + 1.0) ** 2


def bulk_f(phi, p: Params):
    """f = F'(phi) = 4 beta phi (phi + 1)(phi - 1) (below eq 9)."""
    return 4.0 * p.beta * phi * (phi + 1.0) * (phi - 1.0)


def bulk_fprime(phi, p: Params):
    """f'(phi) = 4 beta (3 phi^2 - 1) (below eq 13)."""
    return 4.0 * p.beta * (3.0 * phi * phi - 1.0)


def anisotropy(pg: np.ndarray, p: Params):
    """gamma(n) and |grad phi| * P grad_n gamma for n = grad phi / |grad phi| (eqs 2, 6, 14).

    Returns (gamma, proj) with proj of shape [2, ...].  For m = 4, theta0 = 0 the
    literal eq 6 polynomial is used: gamma = 1 + alpha (4 sum n_i^4 - 3),
    grad_n gamma = 16 alpha n^3 (componentwise), P = I - n n^T.  Other (m, theta0)
    use gamma = 1 + alpha cos(m (theta - theta0)); P grad_n gamma is then the
    tangential derivative d gamma / d theta along t = (-n_y, n_x).
    """
    mag = np.sqrt(pg[0] ** 2 + pg[1] ** 2)
    live = mag > p.grad_floor
    safe = np.where(live, mag, 1.0)
    n = pg / safe
    if p.aniso_m == 4 and p.theta0 == 0.0:
        gamma = 1.0 + p.alpha * (4.0 * (n[0] ** 4 + n[1] ** 4) - 3.0)
        dg = 16.0 * p.alpha * n ** 3
        ndg = n[0] * dg[0] + n[1] * dg[1]
        proj_unit = dg - n * ndg
    else:
        theta = np.arctan2(n[1], n[0])
        arg = p.aniso_m * (theta - p.theta0)
        gamma = 1.0 + p.alpha * np.cos(arg)
        dgamma = -p.alpha * p.aniso_m * np.sin(arg)
        proj_unit = dgamma * np.stack([-n[1], n[0]])
    gamma = np.where(live, gamma, 1.0)
    proj = np.where(live, proj_unit * mag, 0.0)
    return gamma, proj


def vector_Q(pg: np.ndarray, p: Params) -> np.ndarray:
    """Vector field Q under the eq 15 approximation (reading chosen by p.q_form)."""
    gamma, proj = anisotropy(pg, p)
    if p.q_form == "derived":
        return p.kappa * (gamma * pg + proj)
    if p.q_form == "literal":
        return gamma * p.kappa * pg + proj
    raise ValueError(p.q_form)


def chemical_potentials(phi: np.ndarray, p: Params) -> dict:
    """mu of eqs 11-13 and the split mu = mu_alpha + mu_beta of eq 16."""
    pg = grad(phi, p)
    lap = laplacian(phi, p)
    f = bulk_f(phi, p)
    gamma, _ = anisotropy(pg, p)
    Q = vector_Q(pg, p)
    mu = gamma * f - divergence(Q, p)
    if p.reg == REG_WILLMORE:                       # eq 13
        w = lap - f
        mu = mu + p.eps_reg * (laplacian(w, p) - bulk_fprime(phi, p) * w)
    elif p.reg == REG_LINEAR:                       # eq 12
        mu = mu + p.eps_reg * laplacian(lap, p)
    elif p.reg != REG_NONE:
        raise ValueError(p.reg)
    mu_alpha = f - p.kappa * lap                    # eq 16
    mu_beta = mu - mu_alpha
    return {"grad_phi": pg, "lap_phi": lap, "gamma": gamma, "Q": Q,
            "mu": mu, "mu_alpha": mu_alpha, "mu_beta": mu_beta}


# ------------------------------------------------------------- LB pieces --
def equilibrium(phi: np.ndarray, mu_alpha: np.ndarray) -> np.ndarray:
    """Modified equilibrium eq 18."""
    feq = WEIGHTS.reshape((Q9,) + (1,) * np.ndim(mu_alpha)) * mu_alpha[None]
    feq[0] = phi + (WEIGHTS[0] - 1.0) * mu_alpha
    return feq


def source(grad_mu_beta: np.ndarray, p: Params) -> np.ndarray:
    """Source distribution eq 19: F_i = -w_i c_i . grad(mu_beta)."""
    F = np.empty((Q9,) + grad_mu_beta.shape[1:])
    for i in range(Q9):
        F[i] = -WEIGHTS[i] * p.c * (E[0, i] * grad_mu_beta[0] + E[1, i] * grad_mu_beta[1])
    return F


def collide(f: np.ndarray, feq: np.ndarray, F: np.ndarray, p: Params) -> np.ndarray:
    """Right-hand side of eq 17 with the literal matrices (eq 23, eq 25)."""
    S = np.diag(relaxation_rates(p))
    shape = f.shape
    flat = lambda a: a.reshape(Q9, -1)
    relax = M_INV @ S @ M_MATRIX
    forcing = M_INV @ (np.eye(Q9) - S / 2.0) @ M_MATRIX
    post = flat(f) - relax @ (flat(f) - flat(feq)) + p.dt * (forcing @ flat(F))
    return post.reshape(shape)


def stream(fpost: np.ndarray) -> np.ndarray:
    """Left-hand side of eq 17: f_i(x + c_i dt) <- f*_i(x), periodic."""
    out = np.empty_like(fpost)
    for i in range(Q9):
        out[i] = np.roll(fpost[i], shift=(int(E[1, i]), int(E[0, i])), axis=(0, 1))
    return out


def initial_populations(phi0: np.ndarray, p: Params) -> np.ndarray:
    """Populations at t = 0: equilibrium (eq 18) of phi0 with mu_alpha(phi0) of eq 16."""
    mu_alpha = bulk_f(phi0, p) - p.kappa * laplacian(phi0, p)
    return equilibrium(phi0, mu_alpha)


def phi_of(f: np.ndarray) -> np.ndarray:
    """Zeroth moment eq 22."""
    return f.sum(axis=0)


def step(f: np.ndarray, p: Params, want_fields: bool = False):
    """One time step of eq 17 from the pre-collision populations f(x, t)."""
    phi = phi_of(f)
    cp = chemical_potentials(phi, p)
    g = grad(cp["mu_beta"], p)
    feq = equilibrium(phi, cp["mu_alpha"])
    F = source(g, p)
    fnew = stream(collide(f, feq, F, p))
    if want_fields:
        cp = dict(cp, phi=phi, grad_mu_beta=g, feq=feq, F=F)
        return fnew, cp
    return fnew


def run(phi0: np.ndarray, p: Params, nsteps: int) -> np.ndarray:
    """Initialise at equilibrium and advance nsteps; returns the populations."""
    f = initial_populations(np.asarray(phi0, dtype=np.float64), p)
    for _ in range(nsteps):
        f = step(f, p)
    return f


# ------------------------------------------------------------- reductions --
def mass(f: np.ndarray, p: Params) -> float:
    """Total order parameter sum phi dx^2 (conserved, eq 34)."""
    return float(phi_of(f).sum() * p.dx * p.dx)


def free_energy_terms(phi: np.ndarray, p: Params) -> dict:
    """Discrete eq 7: sum over nodes of gamma (kappa/2 |grad phi|^2 + F) + eps/2 G, times dx^2."""
    pg = grad(phi, p)
    gamma, _ = anisotropy(pg, p)
    area = p.dx * p.dx
    grad_term = float((gamma * 0.5 * p.kappa * (pg[0] ** 2 + pg[1] ** 2)).sum() * area)
    bulk_term = float((gamma * bulk_F(phi, p)).sum() * area)
    if p.reg == REG_WILLMORE:                       # eq 9
        G = (laplacian(phi, p) - bulk_f(phi, p)) ** 2
    elif p.reg == REG_LINEAR:                       # eq 8
        G = laplacian(phi, p) ** 2
    else:
        G = np.zeros_like(phi)
    reg_term = float((0.5 * p.eps_reg * G).sum() * area)
    return {"grad": grad_term, "bulk": bulk_term, "reg": reg_term,
            "total": grad_term + bulk_term + reg_term}


def free_energy(f: np.ndarray, p: Params) -> float:
    return free_energy_terms(phi_of(f), p)["total"]


def srt_step(f: np.ndarray, p: Params, s: float) -> np.ndarray:
    """Textbook single-relaxation (BGK) step with forcing, used only as a special-case check."""
    phi = phi_of(f)
    cp = chemical_potentials(phi, p)
    feq = equilibrium(phi, cp["mu_alpha"])
    F = source(grad(cp["mu_beta"], p), p)
    return stream(f - s * (f - feq) + (1.0 - s / 2.0) * p.dt * F)
