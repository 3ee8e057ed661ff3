"""Pins of the NumPy reference U-Net: its 3x3 periodic convolution against scipy's
correlation with wrap-around, and every gradient against central finite differences."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import unet

RNG = np.random.default_rng(11)


def test_conv3_matches_scipy_wrap_correlation():
    x = RNG.normal(size=(2, 7, 9, 3))
    W = RNG.normal(size=(4, 3, 3, 3))
    b = RNG.normal(size=4)
    out = unet.conv3(x, W, b)
    for n in range(2):
        for co in range(4):
            want = b[co] + sum(ndimage.correlate(x[n, :, :, ci], W[co, ci], mode="wrap") for ci in range(3))
            assert np.abs(out[n, :, :, co] - want).max() < 1e-12


def test_pool_and_upsample_are_adjoint_up_to_scale():
    x = RNG.normal(size=(1, 8, 6, 2))
    y = RNG.normal(size=(1, 4, 3, 2))
    assert abs((unet.avgpool2(x) * y).sum() - (x * unet.avgpool2_backward(y)).sum()) < 1e-12
    assert abs((unet.up2(y) * x).sum() - (y * unet.up2_backward(x)).sum()) < 1e-12


@pytest.mark.parametrize("levels,chans,scale", [(2, (4, 6), 1.0), (3, (3, 4, 5), 0.3)])
def test_gradients_match_finite_differences(levels, chans, scale):
    c_in = 3
    params = unet.init_params(levels, chans, c_in, seed=3)
    x = RNG.normal(size=(2, 8, 8, c_in))
    target = RNG.normal(size=(2, 8, 8))

    def loss_of(p, xx):
        pred, _ = unet.forward(p, xx, levels, chans, scale)
        return unet.masked_mse(pred, target, 1)[0]

    pred, cache = unet.forward(params, x, levels, chans, scale)
    _, g = unet.masked_mse(pred, target, 1)
    grads, dx = unet.backward(params, cache, g, levels, chans)
    h = 1e-6
    for name, P in params.items():
        flat = P.reshape(-1)
        for idx in RNG.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = loss_of(params, x)
            flat[idx] = old - h
            lm = loss_of(params, x)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = grads[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, idx, fd, an)
    xf = x.reshape(-1)
    for idx in RNG.choice(xf.size, size=6, replace=False):
        old = xf[idx]
        xf[idx] = old + h
        lp = loss_of(params, x)
        xf[idx] = old - h
        lm = loss_of(params, x)
        xf[idx] = old
        assert abs((lp - lm) / (2 * h) - dx.reshape(-1)[idx]) <= 1e-6 * max(1.0, abs(lp)) + 1e-9


def test_residual_output_identity_when_head_is_zero():
    params = unet.init_params(2, (4, 6), 2, seed=1)
    params["head.W"][:] = 0
    params["head.b"][:] = 0
    x = RNG.normal(size=(1, 4, 4, 2))
    pred, _ = unet.forward(params, x, 2, (4, 6))
    assert np.array_equal(pred, x[..., 0])
