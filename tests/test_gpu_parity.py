"""Parity of the HIP path (through the C-ABI) with the FP64 oracle, on seeded inputs.

Tolerances: FP64 mode max|d phi| <= 1e-11; FP32 mode <= 1e-4 after 1000 steps.
"""
import numpy as np
import pytest

from paper_2501_03759_amd import inputs
from tests import common

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
FP32_TOL = 1e-4


def lb():
    from paper_2501_03759_amd import lbch
    return lbch


def c1_params(precision=0, **kw):
    d = inputs.C1
    args = dict(eps_w=d["eps_w"], mobility=d["mobility"], alpha=d["alpha"], aniso_m=4, eps_reg=d["eps_reg"])
    args.update(kw)
    return common.make_params(64, 64, precision, **args)


def run_gpu(p, phi0, nsteps, tiling=None, loader=0, depth=None):
    L = lb()
    with L.Sim(p) as s:
        s.set_row_loader(loader)
        if depth:
            s.set_time_blocking(depth)
        if tiling:
            s.set_tiling(*tiling)
        s.init(phi0)
        s.step(nsteps)
        return s.phi()


@pytest.mark.parametrize("rates", ["unit", "distinct"])
def test_c1_droplet_fp64_2000_steps(rates):
    kw = {} if rates == "unit" else {"s": inputs.C1_RATES_DISTINCT}
    p = c1_params(0, **kw)
    phi0 = inputs.droplet(64, 64, 16.0, 2.0)
    want = common.oracle_phi(phi0, p, 2000)
    for depth in (1, 2):
        print(f"case c1 rates={rates} depth={depth}", flush=True)
        got = run_gpu(p, phi0, 2000, depth=depth)
        assert np.abs(got - want).max() <= FP64_TOL, depth


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("rates", ["unit", "distinct"])
@pytest.mark.parametrize("shape", [(300, 130), (203, 77), (40, 24)])
def test_time_blocking_is_bitwise(precision, rates, shape):
    # two steps per launch (and the single-step tail of an odd count) against
    # one step per launch; staged and per-lane row loaders, several tilings
    nx, ny = shape
    kw = {} if rates == "unit" else {"s": inputs.C1_RATES_DISTINCT}
    p = common.make_params(nx, ny, precision, width=4.0, alpha=0.3, **kw)
    phi0 = inputs.spinodal(nx, ny, seed=5, amp=0.3)
    print(f"case time-blocking {shape} precision={precision} rates={rates}", flush=True)
    ref = {k: run_gpu(p, phi0, k, depth=1) for k in (60, 61)}
    tilings = [None, (128, 1), (128, 37), (256, 130), (256, 1000)] + ([(512, 64)] if precision == 1 else [])
    for loader in (0, 1):
        for tiling in tilings:
            for nsteps in (61, 60):
                got = run_gpu(p, phi0, nsteps, tiling, loader, depth=2)
                assert np.array_equal(got, ref[nsteps]), (tiling, loader, nsteps)


@pytest.mark.parametrize("alpha", [0.1, 0.3])
def test_paper_parameter_droplet_eq39(alpha):
    # the paper's own parameters (Section 4, eq 39: M = 0.1, Willmore eps = 0.03, D = 5,
    # sigma = 0.01) on its droplet test: R = 25 on 100 x 100, phi0 = tanh(2 (R - r) / D)
    L = lb()
    p = L.default_params(precision=L.FP64, alpha=alpha)
    phi0 = inputs.droplet_width(25.0, 5.0, 100, 100)
    want = common.oracle_phi(phi0, p, 501)
    for depth in (1, 2):
        got = run_gpu(p, phi0, 501, depth=depth)
        assert np.abs(got - want).max() <= FP64_TOL, depth


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (9, 1), (3, 2), (13, 5)])
def test_degenerate_grids_against_oracle(shape):
    # grids smaller than one strip or one stencil radius: every lane and every pipeline row
    # wraps onto the same few nodes; both depths, odd step count, FP64
    nx, ny = shape
    p = common.make_params(nx, ny, 0, width=4.0, alpha=0.3, s=inputs.C1_RATES_DISTINCT)
    phi0 = inputs.spinodal(nx, ny, seed=31, amp=0.4)
    want = common.oracle_phi(phi0, p, 21)
    for depth in (1, 2):
        got = run_gpu(p, phi0, 21, depth=depth)
        assert np.abs(got - want).max() <= FP64_TOL, depth


def test_isotropic_limit_without_regularisation_against_oracle():
    # alpha = 0 (gamma = 1 everywhere) and no regularisation: the pure Cahn-Hilliard limit
    p = common.make_params(72, 40, 0, width=4.0, alpha=0.0, regularization=0)
    phi0 = inputs.spinodal(72, 40, seed=2, amp=0.3)
    want = common.oracle_phi(phi0, p, 150)
    assert np.abs(run_gpu(p, phi0, 150) - want).max() <= FP64_TOL


@pytest.mark.parametrize("precision", [0, 1])
def test_uniform_field_is_steady(precision):
    # grad phi = 0 everywhere: the floor reading (gamma = 1, gamma' = 0) on every node, and a
    # uniform field is an exact steady state of the scheme
    p = common.make_params(64, 48, precision, width=4.0, alpha=0.3)
    phi0 = np.full((48, 64), 0.37)
    got = run_gpu(p, phi0, 40)
    assert np.abs(got - 0.37).max() <= (1e-14 if precision == 0 else 1e-6)
    want = common.oracle_phi(phi0, p, 40)
    assert np.abs(got - want).max() <= (FP64_TOL if precision == 0 else 1e-6)


def test_zero_steps_is_a_no_op():
    L = lb()
    p = common.make_params(40, 24, 0, width=4.0)
    phi0 = inputs.spinodal(40, 24, seed=3, amp=0.3)
    with L.Sim(p) as s:
        s.init(phi0)
        before = s.phi()
        s.step(0)
        assert s.nstep == 0 and np.array_equal(s.phi(), before)


def test_time_blocking_errors():
    L = lb()
    with L.Sim(common.make_params(1024, 257, 0, width=4.0)) as big:
        assert big.time_blocking() == 2                 # more than 512^2 nodes
    with L.Sim(common.make_params(96, 64, 0, width=4.0)) as s:
        assert s.time_blocking() == 1                   # small grids: one step per launch
        with pytest.raises(L.LbchError):
            s.set_time_blocking(3)
        s.set_time_blocking(1)
        assert s.time_blocking() == 1
        s.set_time_blocking(2)
        with pytest.raises(L.LbchError):
            s.set_tiling(512, 16)          # float64 rings of 512 lanes do not fit in LDS
        with pytest.raises(L.LbchError):
            s.set_tiling(64, 16)
        s.set_tiling(256, 16)
        assert s.tiling() == (256, 16)
        s.set_time_blocking(1)
        s.set_tiling(64, 16)


def test_c2_parameters_at_128_fp64():
    d = inputs.C2
    p = common.make_params(128, 128, 0, eps_w=d["eps_w"], mobility=d["mobility"], alpha=d["alpha"],
                           eps_reg=d["eps_reg"])
    phi0 = inputs.spinodal(128, 128, seed=11, amp=0.05)
    got = run_gpu(p, phi0, 400)
    want = common.oracle_phi(phi0, p, 400)
    assert np.abs(got - want).max() <= FP64_TOL


VARIANTS = [
    dict(nx=67, ny=45, regularization=1, alpha=0.2),                      # linear reg, ragged
    dict(nx=67, ny=45, regularization=0, alpha=0.05),                     # no reg
    dict(nx=70, ny=33, q_form=1, alpha=0.1),                              # literal eq 15
    dict(nx=61, ny=64, aniso_m=6, alpha=0.1),                             # 6-fold
    dict(nx=64, ny=50, aniso_m=4, aniso_theta0=0.35, alpha=0.25),          # rotated
    dict(nx=40, ny=40, dx=0.5, dt=0.25, alpha=0.3),                       # non-unit lattice units
    dict(nx=5, ny=7, alpha=0.3),                                          # tiny grid
    dict(nx=1, ny=9, alpha=0.3),
    dict(nx=130, ny=3, alpha=0.3, s=inputs.C1_RATES_DISTINCT),
    dict(nx=300, ny=20, alpha=0.3),                                       # several strips
]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("var", VARIANTS, ids=[str(i) for i in range(len(VARIANTS))])
def test_variants_against_oracle(var, precision):
    var = dict(var)
    nx, ny = var.pop("nx"), var.pop("ny")
    p = common.make_params(nx, ny, precision, width=4.0, **var)
    phi0 = inputs.spinodal(nx, ny, seed=nx * 31 + ny, amp=0.3, mean=0.1)
    nsteps = 150
    print(f"case variant {nx}x{ny} {var} precision={precision}", flush=True)
    got = run_gpu(p, phi0, nsteps)
    want = common.oracle_phi(phi0, p, nsteps)
    tol = FP64_TOL if precision == 0 else 2e-5
    assert np.abs(got - want).max() <= tol


def test_fp32_c2_parameters_1000_steps_at_128():
    d = inputs.C2
    p = common.make_params(128, 128, 1, eps_w=d["eps_w"], mobility=d["mobility"], alpha=d["alpha"],
                           eps_reg=d["eps_reg"])
    phi0 = inputs.spinodal(128, 128, seed=3, amp=0.05)
    got = run_gpu(p, phi0, 1000)
    want = common.oracle_phi(phi0, p, 1000)
    assert np.abs(got - want).max() <= FP32_TOL


@pytest.mark.parametrize("precision", [0, 1])
def test_tiling_is_bitwise_invariant(precision):
    p = common.make_params(300, 130, precision, width=4.0, alpha=0.3, s=inputs.C1_RATES_DISTINCT)
    phi0 = inputs.spinodal(300, 130, seed=5, amp=0.3)
    ref = None
    shapes = {1: [(64, 1), (64, 7), (128, 16), (256, 5), (256, 130), (512, 33), (128, 1000)],
              2: [(128, 3), (256, 29), (128, 130)] + ([(512, 40)] if precision == 1 else [])}
    for loader in (0, 1):
        for depth, tilings in shapes.items():
            for tiling in tilings:
                got = run_gpu(p, phi0, 60, tiling, loader, depth=depth)
                if ref is None:
                    ref = got
                assert np.array_equal(got, ref), (depth, tiling, loader)


def test_reductions_against_oracle():
    from oracle import lbm
    p = c1_params(0, alpha=0.2)
    phi0 = inputs.droplet(64, 64, 16.0, 2.0)
    L = lb()
    with L.Sim(p) as s:
        s.init(phi0)
        s.step(100)
        phi, mass, lo, hi = s.moments()
        E, terms = s.free_energy()
    op = common.oracle_params(p)
    f = lbm.run(phi0, op, 100)
    ph = lbm.phi_of(f)
    t = lbm.free_energy_terms(ph, op)
    assert abs(mass - lbm.mass(f, op)) <= 1e-10
    assert abs(lo - ph.min()) <= FP64_TOL and abs(hi - ph.max()) <= FP64_TOL
    for got, key in zip(terms, ["grad", "bulk", "reg", "total"]):
        assert abs(got - t[key]) <= 1e-11 * max(1.0, abs(t[key])), key
    assert abs(E - t["total"]) <= 1e-11 * abs(t["total"])


@pytest.mark.parametrize("precision", [0, 1])
def test_checkpoint_resume_is_bitwise(precision):
    p = common.make_params(96, 80, precision, width=4.0, alpha=0.3)
    phi0 = inputs.spinodal(96, 80, seed=9, amp=0.2)
    L = lb()
    with L.Sim(p) as a:
        a.init(phi0)
        a.step(50)
        blob = a.save_state()
        a.step(50)
        want = a.phi()
        assert a.nstep == 100
    with L.Sim(p) as b:
        b.load_state(blob)
        assert b.nstep == 50
        b.step(50)
        got = b.phi()
    assert np.array_equal(got, want)


def test_saved_state_is_oracle_populations():
    from oracle import lbm
    p = c1_params(0, alpha=0.3)
    phi0 = inputs.droplet(64, 64, 16.0, 2.0)
    L = lb()
    with L.Sim(p) as s:
        s.init(phi0)
        s.step(20)
        blob = s.save_state()
    body = np.frombuffer(blob[len(blob) - 9 * 64 * 64 * 8:], dtype=np.float64).reshape(9, 64, 64)
    want = lbm.run(phi0, common.oracle_params(p), 20)
    assert np.abs(body - want).max() <= FP64_TOL


def test_state_errors():
    L = lb()
    p = c1_params(0)
    with L.Sim(p) as s:
        with pytest.raises(L.LbchError) as ei:
            s.step(1)
        assert ei.value.status == L.E_STATE
        bad = inputs.droplet(64, 64, 16.0, 2.0)
        bad[3, 4] = np.nan
        with pytest.raises(L.LbchError) as ei:
            s.init(bad)
        assert ei.value.status == L.E_INVALID
        with pytest.raises(L.LbchError) as ei:
            s.init(np.zeros(10))
        assert ei.value.status == L.E_INVALID
        s.init(inputs.droplet(64, 64, 16.0, 2.0))
        with pytest.raises(L.LbchError):
            s.step(-1)
    q = c1_params(0)
    q.nx = 32
    with L.Sim(q) as other, L.Sim(p) as s:
        s.init(inputs.droplet(64, 64, 16.0, 2.0))
        blob = s.save_state()
        with pytest.raises(L.LbchError) as ei:
            other.load_state(blob)
        assert ei.value.status == L.E_INVALID


def test_literal_reading_reports_nonfinite():
    L = lb()
    p = c1_params(0)
    p.kappa, p.beta = 4.0, 0.25
    with L.Sim(p) as s:
        s.init(inputs.droplet(64, 64, 16.0, 2.0))
        s.step(60)
        _, _, _, _ = s.moments(want_phi=False, check=False)
        with pytest.raises(L.LbchError) as ei:
            s.moments(want_phi=False)
        assert ei.value.status == L.E_NONFINITE


@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_init_device_and_phi_device(dtype):
    import torch
    L = lb()
    p = c1_params(0, alpha=0.3)
    phi0 = inputs.spinodal(64, 64, seed=2, amp=0.4)
    if dtype == "float32":
        phi0 = phi0.astype(np.float32).astype(np.float64)
    t = torch.tensor(phi0, dtype=getattr(torch, dtype), device="cuda")
    with L.Sim(p) as a, L.Sim(p) as b:
        a.init(phi0)
        torch.cuda.synchronize()
        b.init_device(t.data_ptr(), L.FP64 if dtype == "float64" else L.FP32, t.numel())
        a.step(10)
        b.step(10)
        pa, pb = a.phi(), b.phi()
        assert np.array_equal(pa, pb)
        out = torch.empty((64, 64), dtype=torch.float64, device="cuda")
        b.phi_device(out.data_ptr(), L.FP64)
        b.synchronize()
        assert np.array_equal(out.cpu().numpy(), pb)


def test_init_device_nonfinite_surfaces_at_moments():
    import torch
    L = lb()
    p = c1_params(0)
    t = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
    t[5, 5] = float("inf")
    with L.Sim(p) as s:
        s.init_device(t.data_ptr(), L.FP64, t.numel())
        with pytest.raises(L.LbchError) as ei:
            s.moments(want_phi=False)
        assert ei.value.status == L.E_NONFINITE


def test_fp32_vs_fp64_c2_full_size_1000_steps():
    # C2 size (1024^2): FP32 production mode against the FP64 mode after 1000 steps.
    d = inputs.C2
    phi0 = inputs.spinodal(1024, 1024, seed=d["seed"], amp=d["amp"])
    out = {}
    for prec in (0, 1):
        p = common.make_params(1024, 1024, prec, eps_w=d["eps_w"], mobility=d["mobility"], alpha=d["alpha"],
                               eps_reg=d["eps_reg"])
        out[prec] = run_gpu(p, phi0, 1000)
    assert np.abs(out[1] - out[0]).max() <= FP32_TOL


@pytest.mark.parametrize("n,precision,seed,depth", [(1024, 0, 0, 1), (1024, 1, 0, 1), (8192, 1, 5, 1),
                                                     (1024, 0, 0, 2), (8192, 1, 5, 2)])
def test_full_size_sampled_against_oracle(n, precision, seed, depth):
    # Full-size grids in the default launch shape of each depth (3 steps: at
    # depth 2 one two-step and one single-step launch): sampled nodes against
    # oracle windows.
    d = inputs.C5 if n == 8192 else inputs.C2
    p = common.make_params(n, n, precision, eps_w=d["eps_w"], mobility=d["mobility"], alpha=d["alpha"],
                           eps_reg=d["eps_reg"])
    phi0 = inputs.spinodal(n, n, seed=seed, amp=d["amp"])
    k = 3
    print(f"case full-size n={n} precision={precision} depth={depth}", flush=True)
    got = run_gpu(p, phi0, k, depth=depth)
    rng = np.random.default_rng(77)
    pts = [(int(y), int(x)) for y, x in rng.integers(0, n, size=(24, 2))]
    pts += [(0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0), (n // 2, 249), (n // 2, 250), (131, 500)]
    want = common.sampled_oracle_phi(phi0, p, k, pts)
    gv = np.array([got[y, x] for (y, x) in pts])
    tol = FP64_TOL if precision == 0 else 2e-6
    assert np.abs(gv - want).max() <= tol


def test_full_size_mass_conservation_fp32():
    d = inputs.C5
    n = 8192
    p = common.make_params(n, n, 1, eps_w=d["eps_w"], mobility=d["mobility"], alpha=d["alpha"],
                           eps_reg=d["eps_reg"])
    phi0 = inputs.spinodal(n, n, seed=d["seed"], amp=d["amp"])
    L = lb()
    with L.Sim(p) as s:
        s.init(phi0)
        _, m0, _, _ = s.moments(want_phi=False)
        s.step(100)
        _, m1, lo, hi = s.moments(want_phi=False)
    scale = np.abs(phi0).sum()
    assert abs(m1 - m0) / scale <= 1e-6
    assert -1.5 < lo < hi < 1.5


def test_autotune_keeps_state_and_results():
    L = lb()
    p = common.make_params(200, 120, 1, width=4.0, alpha=0.3)
    phi0 = inputs.spinodal(200, 120, seed=21, amp=0.3)
    want = run_gpu(p, phi0, 40)
    with L.Sim(p) as s:
        s.init(phi0)
        s.step(10)
        before = s.phi()
        nt, hc, ms = s.autotune(2)
        assert nt in (64, 128, 256, 512) and hc >= 1 and ms > 0 and s.time_blocking() in (1, 2)
        assert s.nstep == 10 and np.array_equal(s.phi(), before)
        s.step(30)
        assert np.array_equal(s.phi(), want)


@pytest.mark.parametrize("model,magic", [(1, 0.25), (2, 0.25), (2, 1.0 / 12.0)])
def test_collision_variants_against_oracle(model, magic):
    # SRT and TRT rate presets (host-side lbch_params_set_collision) on the eq 40 droplet at
    # the eq 39 parameters with alpha = 0.3: the general-rate collision path, both depths
    L = lb()
    p = L.set_collision(L.default_params(nx=64, ny=48, precision=L.FP64, alpha=0.3), model, magic)
    phi0 = inputs.droplet_width(16.0, 5.0, 64, 48)
    want = common.oracle_phi(phi0, p, 301)
    for depth in (1, 2):
        got = run_gpu(p, phi0, 301, depth=depth)
        assert np.abs(got - want).max() <= FP64_TOL, depth
