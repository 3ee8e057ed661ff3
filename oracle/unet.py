"""Float64 NumPy reference of the convolutional surrogate (a periodic U-Net).

TEST INFRASTRUCTURE ONLY.  Written from the surrogate's definition, independent
of the HIP kernels.  Layout: activations [B, H, W, C] (channels last).

Definition (levels L, channels C_0..C_{L-1}, input channels c_in):
  encoder   e_0 = block(x);  e_l = block(avgpool2(e_{l-1}))          l = 1..L-1
  decoder   d_{L-1} = e_{L-1};  d_l = block(concat(up2(d_{l+1}), e_l))  l = L-2..0
  block(z)  = relu(conv3(relu(conv3(z) + b) ) + b)  (two 3x3 convolutions)
  head      y = conv1(d_0) + b                      (one output channel)
  output    phi_pred = x[..., 0] + s * y             (residual on the phi channel, fixed scale s)
conv3 pads periodically (circular), stride 1; avgpool2 is the 2x2 mean; up2
repeats each pixel 2x2; concat puts the upsampled tensor first.
Weights of a 3x3 conv: W[co, ci, ky, kx] with tap (ky, kx) reading pixel
(y + ky - 1, x + kx - 1).

Storage precision (``bf16=True``): the surrogate's configuration stores weights and
activations in BF16 and accumulates in FP32.  With the option on, every tensor the
definition above names is rounded to BF16 where it is formed, and nothing else:
the input planes fed to the first convolution, the 3x3 weights, each convolution's
post-ReLU output, each pooled tensor; in the backward pass the gradient with respect
to each of those tensors (the head's, each data gradient, the upsampling adjoint's
block sums, the skip gradient after the pooling adjoint has been added to it).
Biases, the 1x1 head, the residual base and every sum stay in float64.  With the
option off the network is the plain float64 definition.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest BF16 value (8 significant bits, ties to even), from float64.

    x = m 2^e with 0.5 <= |m| < 1 (frexp); m 2^8 rounded half-to-even (rint) keeps 8 bits.
    Normal range only (the network's values are far from BF16's limits)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.rint(m * 256.0), e - 8)


def _ident(x):
    return x


def _pix(a):
    """[B, H, W, C] as a [B*H*W, C] matrix: each tap is one library matrix product (on
    contiguous operands, which the library multiplies blockwise; a strided weight view
    falls back to a slow elementwise loop)."""
    return a.reshape(-1, a.shape[-1])


def conv3(x, W, b):
    """3x3 periodic convolution: out[n,y,x,co] = b[co] + sum W[co,ci,ky,kx] x[n,y+ky-1,x+kx-1,ci]."""
    out = np.zeros(x.shape[:3] + (W.shape[0],))
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(1 - ky, 1 - kx), axis=(1, 2))
            out += (_pix(xs) @ np.ascontiguousarray(W[:, :, ky, kx].T)).reshape(out.shape)
    return out + b


def conv3_backward(x, W, dout):
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(1 - ky, 1 - kx), axis=(1, 2))
            dW[:, :, ky, kx] = _pix(dout).T @ _pix(xs)
            dx += np.roll((_pix(dout) @ np.ascontiguousarray(W[:, :, ky, kx])).reshape(x.shape),
                          shift=(ky - 1, kx - 1), axis=(1, 2))
    return dx, dW, dout.sum(axis=(0, 1, 2))


def avgpool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def avgpool2_backward(dout):
    return np.repeat(np.repeat(dout, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(dout):
    n, h, w, c = dout.shape
    return dout.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def relu(x):
    return np.maximum(x, 0.0)


def layer_shapes(levels, chans, c_in):
    """Ordered conv layers: (name, c_in, c_out, k) with k = 3 or 1."""
    shapes = []
    prev = c_in
    for l in range(levels):
        shapes.append((f"enc{l}a", prev, chans[l], 3))
        shapes.append((f"enc{l}b", chans[l], chans[l], 3))
        prev = chans[l]
    for l in range(levels - 2, -1, -1):
        shapes.append((f"dec{l}a", chans[l + 1] + chans[l], chans[l], 3))
        shapes.append((f"dec{l}b", chans[l], chans[l], 3))
    shapes.append(("head", chans[0], 1, 1))
    return shapes


def init_params(levels, chans, c_in, seed=0):
    rng = np.random.default_rng(seed)
    params = {}
    for name, ci, co, k in layer_shapes(levels, chans, c_in):
        fan_in = ci * k * k
        params[name + ".W"] = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(co, ci, k, k))
        params[name + ".b"] = rng.normal(0.0, 0.01, size=(co,))
    return params


def forward(params, x, levels, chans, scale=1.0, bf16=False):
    """Returns (phi_pred [B,H,W], cache).  bf16: storage rounding (module docstring)."""
    r = globals()["bf16"] if bf16 else _ident
    cache = {"round": r}

    def block(z, tag):
        Wa, Wb = r(params[tag + "a.W"]), r(params[tag + "b.W"])
        a_pre = conv3(z, Wa, params[tag + "a.b"])
        a = r(relu(a_pre))
        b_pre = conv3(a, Wb, params[tag + "b.b"])
        out = r(relu(b_pre))
        cache[tag] = (z, a_pre, a, b_pre, Wa, Wb)
        return out

    enc = []
    z = r(x)
    for l in range(levels):
        if l > 0:
            z = r(avgpool2(enc[-1]))
        enc.append(block(z, f"enc{l}"))
    d = enc[-1]
    for l in range(levels - 2, -1, -1):
        z = np.concatenate([up2(d), enc[l]], axis=3)
        d = block(z, f"dec{l}")
    W = params["head.W"][:, :, 0, 0]
    y = d @ W.T + params["head.b"]
    cache["head"] = d
    cache["enc"] = enc
    cache["scale"] = scale
    return x[..., 0] + scale * y[..., 0], cache


def backward(params, cache, dphi, levels, chans):
    """Gradients of sum(dphi * phi_pred) w.r.t. every parameter (and the input)."""
    r = cache["round"]
    grads = {}
    d = cache["head"]
    W = params["head.W"][:, :, 0, 0]
    dy = cache["scale"] * dphi[..., None]
    grads["head.W"] = np.einsum("nyxo,nyxi->oi", dy, d)[:, :, None, None]
    grads["head.b"] = dy.sum(axis=(0, 1, 2))
    dd = r(dy @ W)

    def block_back(tag, dout):
        z, a_pre, a, b_pre, Wa, Wb = cache[tag]
        g = dout * (b_pre > 0)
        da, grads[tag + "b.W"], grads[tag + "b.b"] = conv3_backward(a, Wb, g)
        g = r(da) * (a_pre > 0)
        dz, grads[tag + "a.W"], grads[tag + "a.b"] = conv3_backward(z, Wa, g)
        return r(dz)

    enc = cache["enc"]
    denc = [np.zeros_like(e) for e in enc]
    for l in range(0, levels - 1):
        dz = block_back(f"dec{l}", dd)
        cu = chans[l + 1]
        denc[l] += dz[..., cu:]
        dd = r(up2_backward(dz[..., :cu]))
    denc[levels - 1] += dd
    dx = None
    for l in range(levels - 1, -1, -1):
        dz = block_back(f"enc{l}", denc[l])
        if l > 0:
            denc[l - 1] = r(denc[l - 1] + avgpool2_backward(dz))
        else:
            dx = dz
    dx = dx.copy()
    dx[..., 0] += dphi
    return grads, dx


def masked_mse(pred, target, margin):
    """Mean squared error over the interior (margin pixels dropped on every side)."""
    s = (slice(None), slice(margin, pred.shape[1] - margin), slice(margin, pred.shape[2] - margin))
    diff = pred[s] - target[s]
    loss = float((diff ** 2).mean())
    g = np.zeros_like(pred)
    g[s] = 2.0 * diff / diff.size
    return loss, g
