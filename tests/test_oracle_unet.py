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
    # the plain float64 network (storage rounding off, passed explicitly)
    c_in = 3
    params = unet.init_params(levels, chans, c_in, seed=3)
    x = RNG.normal(size=(2, 8, 8, c_in))
    target = RNG.normal(size=(2, 8, 8))

    def loss_of(p, xx):
        pred, _ = unet.forward(p, xx, levels, chans, scale, bf16=False)
        return unet.masked_mse(pred, target, 1)[0]

    pred, cache = unet.forward(params, x, levels, chans, scale, bf16=False)
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


def test_bf16_rounding_matches_the_library_conversion():
    # torch's float32 -> bfloat16 conversion rounds to nearest, ties to even; on float32
    # inputs (exact ties included) the oracle's float64 rounding must give the same values
    import torch
    rng = np.random.default_rng(5)
    a = (rng.normal(size=4000) * np.exp(rng.uniform(-20, 20, size=4000))).astype(np.float32)
    bits = a.view(np.uint32).copy()
    ties = bits[:1000] & np.uint32(0xFFFF0000) | np.uint32(0x8000)     # exactly halfway
    near = bits[1000:2000] & np.uint32(0xFFFF0000) | np.uint32(0x7FFF)  # just below halfway
    bits[:1000], bits[1000:2000] = ties, near
    a = bits.view(np.float32)
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    got = unet.bf16(a.astype(np.float64))
    assert np.array_equal(got, want)
    assert np.array_equal(unet.bf16(np.array([0.0, -0.0, 1.0, -3.5])), [0.0, -0.0, 1.0, -3.5])


def test_bf16_option_rounds_the_stored_tensors_and_stays_close_to_float64():
    levels, chans, c_in = 3, (4, 6, 8), 3
    params = unet.init_params(levels, chans, c_in, seed=7)
    x = RNG.normal(size=(2, 16, 16, c_in))
    dphi = RNG.normal(size=(2, 16, 16))
    p64, c64 = unet.forward(params, x, levels, chans, 0.5)
    p16, c16 = unet.forward(params, x, levels, chans, 0.5, bf16=True)
    for tag in [f"enc{l}" for l in range(levels)] + [f"dec{l}" for l in range(levels - 1)]:
        z, a_pre, a, b_pre, Wa, Wb = c16[tag]
        for t in (z, a, Wa, Wb):
            assert np.array_equal(unet.bf16(t), t), tag
    for e in c16["enc"]:
        assert np.array_equal(unet.bf16(e), e)
    # storage at 8 significant bits moves the output residual by O(2^-8) per layer.  The
    # parameter gradients are sums over pixels of terms of both signs, which magnifies the
    # per-element rounding (here up to ~0.4 relative on 512 pixels), so they are only
    # checked to stay of the float64 network's size and direction
    def rel(u, v):
        return np.linalg.norm(u - v) / np.linalg.norm(v)
    assert 1e-5 < rel(p16 - x[..., 0], p64 - x[..., 0]) < 3e-2
    g64, _ = unet.backward(params, c64, dphi, levels, chans)
    g16, _ = unet.backward(params, c16, dphi, levels, chans)
    for k in g64:
        if k != "head.b":
            assert 0 < rel(g16[k], g64[k]) < 0.6, k
    assert g16["head.b"] == g64["head.b"]
