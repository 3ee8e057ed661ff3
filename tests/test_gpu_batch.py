"""The batched ensemble: every member equals a standalone simulation bitwise, and the
oracle within the parity tolerances; the ensemble workload (ragged sides, m-fold
anisotropy, spinodal / droplet mix) runs in one persistent launch per step."""
import numpy as np
import pytest

from paper_2501_03759_amd import inputs
from tests import common

pytestmark = pytest.mark.gpu


def lb():
    from paper_2501_03759_amd import lbch
    return lbch


def member_params(mem, precision):
    return common.make_params(mem["side"], mem["side"], precision, eps_w=1.5, mobility=0.1, alpha=mem["alpha"],
                              aniso_m=mem["m"], eps_reg=0.03)


def standalone(p, phi0, nsteps):
    L = lb()
    with L.Sim(p) as s:
        s.init(phi0)
        s.step(nsteps)
        return s.phi()


@pytest.mark.parametrize("depth", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_ragged_batch_matches_standalone_bitwise(precision, depth):
    import torch
    L = lb()
    rng = np.random.default_rng(4)
    shapes = [(37, 53), (64, 64), (5, 9), (130, 71), (1, 12), (250, 250), (17, 300)]
    params, fields = [], []
    for k, (ny, nx) in enumerate(shapes):
        kw = dict(alpha=float(rng.uniform(0, 0.3)), aniso_m=int(rng.choice([4, 6])),
                  aniso_theta0=float(rng.uniform(0, 1)))
        if k % 3 == 1:
            kw["s"] = inputs.C1_RATES_DISTINCT
        if k == 2:
            kw["regularization"] = 1
        params.append(common.make_params(nx, ny, precision, width=4.0, **kw))
        fields.append(inputs.spinodal(nx, ny, seed=100 + k, amp=0.3, mean=0.05))
    stream = torch.cuda.Stream()
    with L.Batch(params, stream) as b:
        b.set_time_blocking(depth)
        assert b.time_blocking() == depth
        for k, f in enumerate(fields):
            b.init(k, f)
        # depth 1: 2 graph replays of 16 launches + 13 launches; depth 2: 1 replay of 16 two-step
        # launches + 6 two-step launches + 1 single-step launch
        b.step(45)
        got = [b.phi(k) for k in range(len(shapes))]
        assert b.nstep == 45
    for k in range(len(shapes)):
        want = standalone(params[k], fields[k], 45)
        assert np.array_equal(got[k], want), shapes[k]


def test_batch_members_against_oracle_fp64():
    L = lb()
    shapes = [(24, 40), (33, 33)]
    params = [common.make_params(nx, ny, 0, width=4.0, alpha=0.25, aniso_m=m) for (ny, nx), m in zip(shapes, (4, 6))]
    fields = [inputs.spinodal(nx, ny, seed=7 + k, amp=0.3) for k, (ny, nx) in enumerate(shapes)]
    with L.Batch(params) as b:
        for k, f in enumerate(fields):
            b.init(k, f)
        b.step(120)
        for k in range(len(shapes)):
            want = common.oracle_phi(fields[k], params[k], 120)
            assert np.abs(b.phi(k) - want).max() <= 1e-11


def test_batch_tiling_and_autotune_bitwise():
    L = lb()
    shapes = [(90, 61), (128, 128), (33, 200)]
    params = [common.make_params(nx, ny, 1, width=4.0, alpha=0.2) for (ny, nx) in shapes]
    fields = [inputs.spinodal(nx, ny, seed=70 + k, amp=0.3) for k, (ny, nx) in enumerate(shapes)]
    ref = None
    with L.Batch(params) as b:
        for depth, cfg in [(1, (128, 0, 0)), (1, (64, 7, 3)), (1, (256, 50, 1)), (1, (512, 16, 0)),
                           (2, (128, 0, 0)), (2, (256, 33, 1)), (2, (512, 70, 0)), (2, (128, 5, 0))]:
            b.set_time_blocking(depth)
            for k, f in enumerate(fields):
                b.init(k, f)
            b.set_tiling(*cfg)
            b.step(20 if cfg[1] != 5 else 19)
            if cfg[1] == 5:
                b.step(1)
            got = [b.phi(k) for k in range(3)]
            if ref is None:
                ref = got
            for g, r in zip(got, ref):
                assert np.array_equal(g, r), cfg
        for k, f in enumerate(fields):
            b.init(k, f)
        b.step(5)
        before = [b.phi(k) for k in range(3)]
        nt, hc, ms = b.autotune(2)
        assert ms > 0 and nt in (64, 128, 256) and b.time_blocking() in (1, 2)
        after = [b.phi(k) for k in range(3)]
        for x, y in zip(before, after):
            assert np.array_equal(x, y)
        b.step(15)
        for g, r in zip([b.phi(k) for k in range(3)], ref):
            assert np.array_equal(g, r)


def test_batch_errors():
    L = lb()
    p0 = common.make_params(16, 16, 0, width=4.0)
    p1 = common.make_params(16, 16, 1, width=4.0)
    with pytest.raises(L.LbchError):
        L.Batch([p0, p1])
    with L.Batch([p0, p0]) as b:
        with pytest.raises(L.LbchError) as ei:
            b.step(1)
        assert ei.value.status == L.E_STATE
        b.init(0, np.zeros((16, 16)))
        with pytest.raises(L.LbchError) as ei:
            b.step(1)
        assert ei.value.status == L.E_STATE
        with pytest.raises(L.LbchError) as ei:
            b.set_time_blocking(3)
        assert ei.value.status == L.E_INVALID
        b.set_time_blocking(2)
        with pytest.raises(L.LbchError):
            b.set_tiling(512, 0, 0)        # float64 rings of 512 lanes do not fit in LDS
        with pytest.raises(L.LbchError):
            b.set_tiling(64, 0, 0)
        with pytest.raises(L.LbchError) as ei:
            b.init(2, np.zeros((16, 16)))
        assert ei.value.status == L.E_INVALID


def test_ensemble_workload_sampled_members():
    # The 512-member ensemble (sides log-uniform in [64, 512], alpha ~ U[0, 0.3], m in {4, 6},
    # spinodal / droplet 50/50), FP32, one persistent launch per two steps; sampled members
    # are checked bitwise against standalone runs and mass is conserved for all.
    import torch
    L = lb()
    mems = inputs.ensemble_members(512, seed=3)
    params = [member_params(m, 1) for m in mems]
    stream = torch.cuda.Stream()
    nsteps = 40
    with L.Batch(params, stream) as b:
        fields = {}
        for k, m in enumerate(mems):
            f = inputs.member_phi0(m)
            if k % 97 == 0:
                fields[k] = f
            b.init(k, f)
        m0 = [b.moments(k, want_phi=False)[1] for k in range(len(mems))]
        b.step(nsteps)
        for k in fields:
            assert np.array_equal(b.phi(k), standalone(params[k], fields[k], nsteps)), k
        for k in range(0, len(mems), 7):
            _, m1, lo, hi = b.moments(k, want_phi=False)
            side = mems[k]["side"]
            assert abs(m1 - m0[k]) <= 1e-6 * side * side
            assert -1.5 < lo <= hi < 1.5
