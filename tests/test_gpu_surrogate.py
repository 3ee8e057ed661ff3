"""The BF16-MFMA surrogate against the float64 NumPy reference network: forward,
parameter gradients (same weights, same inputs), and that training lowers the loss."""
import numpy as np
import pytest

from oracle import unet

pytestmark = pytest.mark.gpu


def flat_to_dict(flat, levels, chans, c_in):
    d, off = {}, 0
    for name, ci, co, k in unet.layer_shapes(levels, chans, c_in):
        n = co * ci * k * k
        d[name + ".W"] = flat[off:off + n].reshape(co, ci, k, k).astype(np.float64)
        off += n
        d[name + ".b"] = flat[off:off + co].astype(np.float64)
        off += co
    assert off == flat.size
    return d


def dict_to_flat(d, levels, chans, c_in):
    parts = []
    for name, ci, co, k in unet.layer_shapes(levels, chans, c_in):
        parts += [d[name + ".W"].reshape(-1), d[name + ".b"].reshape(-1)]
    return np.concatenate(parts).astype(np.float32)


def bf16_round(a):
    import torch
    return torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def calibrate_biases(params, x, levels, chans, k=5.0):
    """Biases that put every channel's pre-activation k standard deviations away from the
    ReLU kink, on alternating sides (even channels mostly active, odd ones mostly zero), set
    layer by layer on the BF16-storage reference's own forward pass.  Near the kink, a
    pre-activation that FP32 and float64 accumulation round to different BF16 values flips
    its ReLU decision, and such flips cascade through the later layers; away from it the
    comparison measures the network's composition."""
    names = [n for n, *_ in unet.layer_shapes(levels, chans, x.shape[-1]) if n != "head"]
    for n in names:
        params[n + ".b"] = np.zeros_like(params[n + ".b"])
    for n in names:
        _, cache = unet.forward(params, x, levels, chans, bf16=True)
        z, a_pre, a, b_pre, Wa, Wb = cache[n[:-1]]
        pre = a_pre if n.endswith("a") else b_pre
        mu, sd = pre.mean(axis=(0, 1, 2)), pre.std(axis=(0, 1, 2))
        side = np.where(np.arange(pre.shape[-1]) % 2 == 0, 1.0, -1.0)
        params[n + ".b"] = bf16_round(side * k * sd - mu)


def run_both(levels, chans, hw, bias_shift, seed, B=2, bf16=True, conditioned=False):
    """The HIP network and the float64 reference on the same BF16 parameters and inputs;
    bf16: the reference rounds its stored tensors to BF16 where the definition forms them
    (its storage-precision option), else it is the plain float64 network.

    conditioned: a case whose sums do not cancel, so that relative differences measure the
    composition rather than amplified rounding noise: the input is shaped as the surrogate's
    (phi, then four constant conditioning planes), biases from calibrate_biases, positive
    head weights, and an output gradient of mostly one sign (1 + 0.5 N(0, 1), as for a
    prediction biased high).  Otherwise: normal inputs and output gradient, the
    initialisation's biases (plus bias_shift)."""
    import torch
    from paper_2501_03759_amd import lbsg
    c_in = 5
    rng = np.random.default_rng(seed)
    net = lbsg.Surrogate(chans, c_in, B, hw, hw, train=True, seed=1)
    params = unet.init_params(levels, chans, c_in, seed=seed)
    params["head.W"] *= 0.5
    if conditioned:
        params["head.W"] = np.abs(params["head.W"])
    for k in params:
        if k.endswith(".b") and not k.startswith("head"):
            params[k] = params[k] + bias_shift
        params[k] = bf16_round(params[k])
    if conditioned:
        x = np.empty((B, hw, hw, c_in))
        x[..., 0] = rng.normal(size=(B, hw, hw)) * 0.5
        x[..., 1:] = [0.2, 0.7, -0.7, 2.0 / 3.0]
        x = bf16_round(x)
        calibrate_biases(params, x, levels, chans)
    else:
        x = bf16_round(rng.normal(size=(B, hw, hw, c_in)) * 0.5)
    net.set_params(dict_to_flat(params, levels, chans, c_in))
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    out = torch.empty((B, hw, hw), dtype=torch.float32, device="cuda")
    net.forward(xt.data_ptr(), B, hw, hw, out.data_ptr())
    torch.cuda.synchronize()
    pred_ref, cache = unet.forward(params, x, levels, chans, bf16=bf16)
    got = out.cpu().numpy().astype(np.float64)
    dphi = rng.normal(size=(B, hw, hw))
    if conditioned:
        dphi = 1.0 + 0.5 * dphi
    dphi = dphi.astype(np.float32).astype(np.float64)
    dt = torch.tensor(dphi, dtype=torch.float32, device="cuda")
    grads = torch.empty(net.nparam, dtype=torch.float32, device="cuda")
    net.backward(dt.data_ptr(), grads.data_ptr())
    torch.cuda.synchronize()
    g_gpu = flat_to_dict(grads.cpu().numpy(), levels, chans, c_in)
    g_ref, _ = unet.backward(params, cache, dphi, levels, chans)
    return got - x[..., 0], pred_ref - x[..., 0], g_gpu, g_ref


OPS = [(2, 32, 48, 32, 64), (1, 16, 16, 96, 32), (3, 48, 32, 64, 128)]
# at >= 512 (16 x 16 tile, 64-channel block) pairs the forward takes 64-channel workgroups
OPS_FWD = OPS + [(2, 256, 256, 32, 64), (1, 256, 512, 64, 128), (4, 256, 256, 32, 32), (2, 256, 512, 64, 32)]


def diag():
    from paper_2501_03759_amd import lbch
    L = lbch.lib()
    import ctypes
    for name, nargs in (("lbsg_diag_conv3", 10), ("lbsg_diag_conv3_dgrad", 8), ("lbsg_diag_conv3_wgrad", 8),
                        ("lbsg_diag_conv3_bgrad", 8)):
        fn = getattr(L, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_void_p] * (4 if name == "lbsg_diag_conv3" else 3) + [ctypes.c_int32] * (
            nargs - (4 if name == "lbsg_diag_conv3" else 3))
    return L


@pytest.mark.parametrize("n,h,w,ci,co", OPS_FWD)
def test_mfma_conv_forward_exact_on_bf16_inputs(n, h, w, ci, co):
    import torch
    L = diag()
    rng = np.random.default_rng(ci + co)
    x = bf16_round(rng.normal(size=(n, h, w, ci)))
    W = bf16_round(rng.normal(size=(co, ci, 3, 3)) * 0.1)
    b = rng.normal(size=co)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    wt = torch.tensor(W, dtype=torch.float32, device="cuda")
    bt = torch.tensor(b, dtype=torch.float32, device="cuda")
    yt = torch.empty((n, h, w, co), dtype=torch.float32, device="cuda")
    for relu in (0, 1):
        assert L.lbsg_diag_conv3(xt.data_ptr(), wt.data_ptr(), bt.data_ptr(), yt.data_ptr(), n, h, w, ci, co, relu) == 0
        ref = unet.conv3(x, W, b.astype(np.float32).astype(np.float64))
        if relu:
            ref = np.maximum(ref, 0)
        got = yt.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 32, 48, 5, 32), (1, 64, 64, 1, 64), (4, 256, 256, 5, 32),
                                         (1, 48, 32, 8, 32)])
def test_first_layer_with_packed_k_exact_and_phi_form_bitwise(n, h, w, ci, co):
    # the first convolution with its <= 8 input channels packed into K (12 taps x 8): exact on
    # BF16 inputs; fed phi and constant conditioning values directly, it gives the bits it gives
    # on the packed input holding them
    import ctypes
    import torch
    L = diag()
    fn = L.lbsg_diag_conv3_first
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_int32] * 5
    rng = np.random.default_rng(ci * 31 + co)
    x = bf16_round(rng.normal(size=(n, h, w, ci)))
    W = bf16_round(rng.normal(size=(co, ci, 3, 3)) * 0.3)
    b = rng.normal(size=co) * 0.1
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    xt, wt, bt = dev(x), dev(W), dev(b)
    y = torch.empty((n, h, w, co), dtype=torch.float32, device="cuda")
    print(f"case first layer {(n, h, w, ci, co)}", flush=True)
    assert fn(xt.data_ptr(), None, None, wt.data_ptr(), bt.data_ptr(), y.data_ptr(), n, h, w, ci, co) == 0
    ref = np.maximum(unet.conv3(x, W, b.astype(np.float32).astype(np.float64)), 0)
    got = y.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())
    # constant planes 1..ci-1: the packed form against the phi form
    cond = (np.arange(1, ci) * 0.37 - 0.9).astype(np.float32)
    xc = x.copy()
    xc[..., 1:] = bf16_round(cond.astype(np.float64))
    yc = torch.empty_like(y)
    yp = torch.empty_like(y)
    assert fn(dev(xc).data_ptr(), None, None, wt.data_ptr(), bt.data_ptr(), yc.data_ptr(), n, h, w, ci, co) == 0
    pt = dev(x[..., 0])
    cp = cond.ctypes.data_as(ctypes.c_void_p) if ci > 1 else None
    assert fn(None, pt.data_ptr(), cp, wt.data_ptr(), bt.data_ptr(), yp.data_ptr(), n, h, w, ci, co) == 0
    assert torch.equal(yc.cpu(), yp.cpu())


# (n, h, w, cu, cs, co): 32- and 64-channel workgroups, one and several chunks per source
OPS_UPCAT = [(2, 32, 48, 64, 32, 32), (3, 16, 32, 32, 64, 64), (2, 256, 256, 64, 32, 64), (1, 256, 256, 32, 64, 128),
             (1, 128, 256, 256, 128, 128), (4, 256, 256, 64, 32, 32)]


@pytest.mark.parametrize("n,h,w,cu,cs,co", OPS_UPCAT)
def test_mfma_conv_of_upsampled_concat_exact_on_bf16_inputs(n, h, w, cu, cs, co):
    import ctypes
    import torch
    L = diag()
    fn = L.lbsg_diag_conv3_upcat
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int32] * 7
    rng = np.random.default_rng(cu + cs + co)
    u = bf16_round(rng.normal(size=(n, h // 2, w // 2, cu)))
    sk = bf16_round(rng.normal(size=(n, h, w, cs)))
    W = bf16_round(rng.normal(size=(co, cu + cs, 3, 3)) * 0.1)
    b = rng.normal(size=co)
    dev = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    ut, st, wt, bt = dev(u), dev(sk), dev(W), dev(b)
    yt = torch.empty((n, h, w, co), dtype=torch.float32, device="cuda")
    z = np.concatenate([unet.up2(u), sk], axis=3)
    ref0 = unet.conv3(z, W, b.astype(np.float32).astype(np.float64))
    for relu in (0, 1):
        print(f"case upcat {(n, h, w, cu, cs, co)} relu={relu}", flush=True)
        assert fn(ut.data_ptr(), st.data_ptr(), wt.data_ptr(), bt.data_ptr(), yt.data_ptr(), n, h, w, cu, cs, co,
                  relu) == 0
        ref = np.maximum(ref0, 0) if relu else ref0
        got = yt.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 32, 48, 64, 32), (1, 48, 32, 96, 64), (2, 256, 256, 32, 64),
                                         (1, 64, 64, 128, 256), (4, 256, 256, 32, 32)])
def test_mfma_conv_with_fused_pooling_is_bitwise(n, h, w, ci, co):
    # y equals the plain ReLU kernel's output and yp the 2x2 average of it with the pooling
    # kernel's arithmetic: bf16(0.25 ((a + b) + (c + d))) in FP32, bit for bit
    import ctypes
    import torch
    L = diag()
    fn = L.lbsg_diag_conv3_pool
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int32] * 5
    rng = np.random.default_rng(ci + 7 * co)
    x = bf16_round(rng.normal(size=(n, h, w, ci)))
    W = bf16_round(rng.normal(size=(co, ci, 3, 3)) * 0.1)
    b = rng.normal(size=co)
    dev = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    xt, wt, bt = dev(x), dev(W), dev(b)
    y = torch.empty((n, h, w, co), dtype=torch.float32, device="cuda")
    yp = torch.empty((n, h // 2, w // 2, co), dtype=torch.float32, device="cuda")
    y0 = torch.empty_like(y)
    assert fn(xt.data_ptr(), wt.data_ptr(), bt.data_ptr(), y.data_ptr(), yp.data_ptr(), n, h, w, ci, co) == 0
    assert L.lbsg_diag_conv3(xt.data_ptr(), wt.data_ptr(), bt.data_ptr(), y0.data_ptr(), n, h, w, ci, co, 1) == 0
    yc = y.cpu()
    assert torch.equal(yc, y0.cpu())
    a, bb, c, d = yc[:, 0::2, 0::2], yc[:, 0::2, 1::2], yc[:, 1::2, 0::2], yc[:, 1::2, 1::2]
    want = (0.25 * ((a + bb) + (c + d))).to(torch.bfloat16).to(torch.float32)
    assert torch.equal(yp.cpu(), want)


@pytest.mark.parametrize("n,h,w,cu,cs,co,masked", [(2, 32, 48, 64, 32, 32, True), (1, 64, 64, 128, 64, 64, True),
                                                     (2, 256, 256, 64, 64, 32, True), (1, 32, 32, 96, 32, 64, True),
                                                     (1, 32, 64, 64, 32, 32, False),
                                                     (4, 256, 256, 32, 32, 32, True)])
def test_data_gradient_through_upsampling_adjoint_is_bitwise(n, h, w, cu, cs, co, masked):
    # the decoder's first convolution: its data gradient's up channels summed over 2x2
    # blocks in the kernel's order ((a + b) + c) + d, its skip channels stored, both masked,
    # equal the plain data-gradient kernel followed by those steps, bit for bit
    import ctypes
    import torch
    L = diag()
    fn = L.lbsg_diag_conv3_dgrad_upadj
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_int32] * 6
    dg = L.lbsg_diag_conv3_dgrad
    dg.restype = ctypes.c_int
    dg.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int32] * 5
    rng = np.random.default_rng(cu + 3 * cs + 11 * co)
    ci = cu + cs
    dy = bf16_round(rng.normal(size=(n, h, w, co)))
    W = bf16_round(rng.normal(size=(co, ci, 3, 3)) * 0.1)
    mu = rng.normal(size=(n, h // 2, w // 2, cu))
    ms = rng.normal(size=(n, h, w, cs))
    dev = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    dyt, wt, mut, mst = dev(dy), dev(W), dev(mu), dev(ms)
    du = torch.empty((n, h // 2, w // 2, cu), dtype=torch.float32, device="cuda")
    ds = torch.empty((n, h, w, cs), dtype=torch.float32, device="cuda")
    dx = torch.empty((n, h, w, ci), dtype=torch.float32, device="cuda")
    print(f"case upadj n={n} h={h} w={w} cu={cu} cs={cs} co={co} masked={masked}", flush=True)
    assert fn(dyt.data_ptr(), wt.data_ptr(), mut.data_ptr() if masked else None,
              mst.data_ptr() if masked else None, du.data_ptr(), ds.data_ptr(), n, h, w, cu, cs, co) == 0
    assert dg(dyt.data_ptr(), wt.data_ptr(), dx.data_ptr(), n, h, w, ci, co) == 0
    x = dx.cpu()
    up = x[..., :cu]
    a, b, c, d = up[:, 0::2, 0::2], up[:, 0::2, 1::2], up[:, 1::2, 0::2], up[:, 1::2, 1::2]
    want_u = (((a + b) + c) + d).to(torch.bfloat16).to(torch.float32)
    want_s = x[..., cu:].clone()
    if masked:
        want_u = torch.where(torch.tensor(mu) > 0, want_u, torch.zeros_like(want_u))
        want_s = torch.where(torch.tensor(ms) > 0, want_s, torch.zeros_like(want_s))
    assert torch.equal(du.cpu(), want_u)
    assert torch.equal(ds.cpu(), want_s)


# (4, 128, 128, 128, 64): 256 tiles x 2 blocks of 64 output channels reach the 64-channel workgroups
@pytest.mark.parametrize("n,h,w,ci,co,masked", [(2, 32, 48, 32, 64, True), (1, 64, 64, 64, 128, True),
                                                 (4, 128, 128, 64, 64, True), (1, 16, 32, 96, 32, False),
                                                 (4, 128, 128, 128, 64, True), (4, 256, 256, 32, 32, True)])
def test_data_gradient_through_pooling_adjoint_is_bitwise(n, h, w, ci, co, masked):
    # an encoder level's first convolution: its data gradient, spread over the 2x2 children
    # and accumulated into the finer level's gradient as bf16(0.25 dx + old), then masked,
    # equals the plain data-gradient kernel followed by those steps, bit for bit
    import ctypes
    import torch
    L = diag()
    fn = L.lbsg_diag_conv3_dgrad_pooladj
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32] * 5
    dg = L.lbsg_diag_conv3_dgrad
    dg.restype = ctypes.c_int
    dg.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int32] * 5
    rng = np.random.default_rng(ci + 5 * co + h)
    dy = bf16_round(rng.normal(size=(n, h, w, co)))
    W = bf16_round(rng.normal(size=(co, ci, 3, 3)) * 0.1)
    base = bf16_round(rng.normal(size=(n, 2 * h, 2 * w, ci)))
    mask = rng.normal(size=(n, 2 * h, 2 * w, ci))
    dev = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    dyt, wt, mt = dev(dy), dev(W), dev(mask)
    dx2 = dev(base)
    dx = torch.empty((n, h, w, ci), dtype=torch.float32, device="cuda")
    print(f"case pooladj n={n} h={h} w={w} ci={ci} co={co} masked={masked}", flush=True)
    assert fn(dyt.data_ptr(), wt.data_ptr(), mt.data_ptr() if masked else None, dx2.data_ptr(), n, h, w, ci, co) == 0
    assert dg(dyt.data_ptr(), wt.data_ptr(), dx.data_ptr(), n, h, w, ci, co) == 0
    up = dx.cpu().repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)
    want = (0.25 * up + torch.tensor(base, dtype=torch.float32)).to(torch.bfloat16).to(torch.float32)
    if masked:
        want = torch.where(torch.tensor(mask) > 0, want, torch.zeros_like(want))
    assert torch.equal(dx2.cpu(), want)


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 32, 48, 64, 32), (1, 48, 32, 96, 64), (2, 256, 256, 32, 32),
                                         (4, 256, 256, 32, 32)])
def test_mfma_conv_with_fused_head(n, h, w, ci, co):
    # the BF16 activations are those of the plain kernel; only the FP32 order of the
    # head's channel sum differs from a sequential dot product
    import ctypes
    import torch
    L = diag()
    fn = L.lbsg_diag_conv3_head
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] * 6 + [ctypes.c_int32, ctypes.c_float, ctypes.c_void_p] + [ctypes.c_int32] * 5
    rng = np.random.default_rng(ci * co)
    cin = 3
    x = bf16_round(rng.normal(size=(n, h, w, ci)))
    W = bf16_round(rng.normal(size=(co, ci, 3, 3)) * 0.1)
    b = rng.normal(size=co).astype(np.float32)
    hw = rng.normal(size=co).astype(np.float32)
    hb = np.float32(rng.normal())
    xin = rng.normal(size=(n, h, w, cin)).astype(np.float32)
    scale = 0.37
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")
    xt, wt, bt, hwt, hbt, xint = dev(x), dev(W), dev(b), dev(hw), dev(np.array([hb])), dev(xin)
    out = torch.empty((n, h, w), dtype=torch.float32, device="cuda")
    assert fn(xt.data_ptr(), wt.data_ptr(), bt.data_ptr(), hwt.data_ptr(), hbt.data_ptr(), xint.data_ptr(), cin,
              scale, out.data_ptr(), n, h, w, ci, co) == 0
    # activations from the plain kernel, then the head in float64
    yt = torch.empty((n, h, w, co), dtype=torch.float32, device="cuda")
    assert L.lbsg_diag_conv3(xt.data_ptr(), wt.data_ptr(), bt.data_ptr(), yt.data_ptr(), n, h, w, ci, co, 1) == 0
    y = yt.cpu().numpy().astype(np.float64)
    ref = xin[..., 0].astype(np.float64) + scale * (float(hb) + y @ hw.astype(np.float64))
    got = out.cpu().numpy().astype(np.float64)
    bound = 5e-6 * (np.abs(xin[..., 0]) + scale * (abs(float(hb)) + np.abs(y) @ np.abs(hw.astype(np.float64))))
    assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref).max()


@pytest.mark.parametrize("n,h,w,ci,co", OPS + [(4, 256, 256, 32, 32)])
def test_mfma_conv_gradients_exact_on_bf16_inputs(n, h, w, ci, co):
    import torch
    L = diag()
    rng = np.random.default_rng(3 * ci + co)
    x = bf16_round(rng.normal(size=(n, h, w, ci)))
    W = bf16_round(rng.normal(size=(co, ci, 3, 3)) * 0.1)
    dy = bf16_round(rng.normal(size=(n, h, w, co)))
    dx_ref, dw_ref, db_ref = unet.conv3_backward(x, W, dy)
    xt = torch.tensor(x, dtype=torch.float32, device="cuda")
    wt = torch.tensor(W, dtype=torch.float32, device="cuda")
    gt = torch.tensor(dy, dtype=torch.float32, device="cuda")
    dxt = torch.empty((n, h, w, ci), dtype=torch.float32, device="cuda")
    dwt = torch.empty((co, ci, 3, 3), dtype=torch.float32, device="cuda")
    dbt = torch.empty(co, dtype=torch.float32, device="cuda")
    assert L.lbsg_diag_conv3_dgrad(gt.data_ptr(), wt.data_ptr(), dxt.data_ptr(), n, h, w, ci, co) == 0
    assert L.lbsg_diag_conv3_wgrad(xt.data_ptr(), gt.data_ptr(), dwt.data_ptr(), n, h, w, ci, co) == 0
    assert L.lbsg_diag_conv3_bgrad(xt.data_ptr(), gt.data_ptr(), dbt.data_ptr(), n, h, w, ci, co) == 0
    dx = dxt.cpu().numpy().astype(np.float64)
    dw = dwt.cpu().numpy().astype(np.float64)
    db = dbt.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(dx - dx_ref) <= 2.0 ** -8 * np.abs(dx_ref) + 1e-5 * np.abs(dx_ref).max())
    assert np.abs(dw - dw_ref).max() <= 1e-5 * np.abs(dw_ref).max()
    # FP32 sums of BF16 values: within n_terms * 2^-24 of the sum of magnitudes
    bound = (n * h * w) * 2.0 ** -24 * np.abs(dy).sum(axis=(0, 1, 2))
    assert np.all(np.abs(db - db_ref) <= bound)


@pytest.mark.parametrize("n,h,w,cu,cs,co", [(2, 32, 48, 64, 32, 32), (3, 48, 32, 32, 64, 64), (1, 64, 64, 128, 64, 128)])
def test_mfma_weight_gradient_of_upsampled_concat(n, h, w, cu, cs, co):
    import ctypes
    import torch
    L = diag()
    fn = L.lbsg_diag_conv3_wgrad_upcat
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32] * 6
    rng = np.random.default_rng(5 * cu + cs + co)
    u = bf16_round(rng.normal(size=(n, h // 2, w // 2, cu)))
    sk = bf16_round(rng.normal(size=(n, h, w, cs)))
    dy = bf16_round(rng.normal(size=(n, h, w, co)))
    W = np.zeros((co, cu + cs, 3, 3))
    _, dw_ref, _ = unet.conv3_backward(np.concatenate([unet.up2(u), sk], axis=3), W, dy)
    dev = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    ut, st, gt = dev(u), dev(sk), dev(dy)
    dwt = torch.empty((co, cu + cs, 3, 3), dtype=torch.float32, device="cuda")
    print(f"case wgrad upcat {(n, h, w, cu, cs, co)}", flush=True)
    assert fn(ut.data_ptr(), st.data_ptr(), gt.data_ptr(), dwt.data_ptr(), n, h, w, cu, cs, co) == 0
    dw = dwt.cpu().numpy().astype(np.float64)
    assert np.abs(dw - dw_ref).max() <= 1e-5 * np.abs(dw_ref).max()


# (levels, channels, side, batch): every level count the kernels serve up to the 5-level,
# 32 -> 256-channel configuration with its 16 x 16 bottom level, and the 3-level
# (32, 64, 96) net whose intermediate decoder level (upsampling adjoint into a decoder
# gradient, not the bottom encoder's) the 2-level net does not have
WHOLE_NETS = [(2, (32, 64), 32, 2), (3, (32, 64, 96), 64, 2), (4, (32, 64, 128, 128), 128, 2),
              (5, (32, 64, 128, 256, 256), 256, 2)]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("levels,chans,hw,B", WHOLE_NETS)
def test_forward_and_gradients_match_bf16_storage_reference(levels, chans, hw, B):
    # Whole-network composition (pool / upsample / concat adjoints, layer order, the fused
    # epilogues, every ReLU mask) against the float64 reference with BF16 storage at the
    # definition's tensor boundaries: what differs is FP32 against float64 accumulation
    # inside each operator.  The output and every parameter tensor's gradient within 2e-2
    # relative L2; a composition mistake (a wrong channel offset, a missing adjoint or mask)
    # gives O(1) errors.  The case is the conditioned one of run_both.  Where the
    # pre-activations sit near the ReLU kink, accumulation-order differences flip ReLU
    # decisions and BF16 roundings, the flips cascade through the later layers, and sums of
    # terms of both signs (a bias gradient under a random output gradient) magnify them: a
    # CPU emulation (the reference with its convolution results rounded to FP32) differs from
    # the reference itself by up to 5 % in the 3-level net's gradients at the
    # initialisation's parameters, and by at most 2e-4 in the conditioned case.  The
    # unconditioned case is the float64-network test below.
    print(f"case whole net levels={levels} chans={chans} side={hw} batch={B}", flush=True)
    y_gpu, y_ref, g_gpu, g_ref = run_both(levels, chans, hw, bias_shift=0.0, seed=2 + levels, B=B,
                                          conditioned=True)
    worst = max((rel(g_gpu[k], g_ref[k]), k) for k in g_ref)
    print(f"  output rel {rel(y_gpu, y_ref):.2e}, worst gradient rel {worst[0]:.2e} ({worst[1]})", flush=True)
    assert rel(y_gpu, y_ref) < 2e-2
    for name in g_ref:
        assert rel(g_gpu[name], g_ref[name]) < 2e-2, (name, rel(g_gpu[name], g_ref[name]))


def test_forward_and_gradients_against_float64_network():
    # The same composition against the plain float64 network (no storage rounding): the
    # output residual stays within a few BF16 steps; parameter gradients are sums over
    # pixels of terms of both signs, where rounding the activations to 8 bits moves the
    # typical channel by several percent, so only the typical channel and the whole tensor
    # are bounded here (the per-tensor 2e-2 bar is the test above)
    y_gpu, y_ref, g_gpu, g_ref = run_both(2, (32, 64), 32, bias_shift=0.0, seed=2, bf16=False)
    assert rel(y_gpu, y_ref) < 3e-2
    for name in g_ref:
        if name.startswith("head"):
            assert rel(g_gpu[name], g_ref[name]) < 2e-2
            continue
        a, b = g_gpu[name], g_ref[name]
        per_co = [rel(a[c], b[c]) for c in range(b.shape[0])]
        assert np.median(per_co) < 0.1 and rel(a, b) < 0.25, (name, np.median(per_co), rel(a, b))


def test_forward_with_wide_first_level():
    # 128 channels at the first level: the output head runs as its own kernel (the fused
    # epilogue covers 32 or 64), and the pooled / upsampled paths carry 128 channels
    y_gpu, y_ref, g_gpu, g_ref = run_both(2, (128, 64), 32, bias_shift=0.0, seed=4, bf16=False)
    assert rel(y_gpu, y_ref) < 3e-2
    assert rel(g_gpu["head.W"], g_ref["head.W"]) < 2e-2


def test_untrained_net_is_identity_and_training_lowers_loss():
    import torch
    from paper_2501_03759_amd import lbsg
    chans, c_in, B, hw = (32, 64), 3, 4, 32
    net = lbsg.Surrogate(chans, c_in, B, hw, hw, train=True, seed=3)
    rng = np.random.default_rng(9)
    x = rng.normal(size=(B, hw, hw, c_in)).astype(np.float32)
    # target: a fixed smooth map of the input (a learnable residual)
    target = x[..., 0] + 0.3 * np.roll(x[..., 0], 1, axis=1) - 0.2 * x[..., 1]
    xt = torch.tensor(x, device="cuda")
    tt = torch.tensor(target.astype(np.float32), device="cuda")
    out = torch.empty((B, hw, hw), dtype=torch.float32, device="cuda")
    net.forward(xt.data_ptr(), B, hw, hw, out.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), x[..., 0])
    losses = [net.train_step(xt.data_ptr(), tt.data_ptr(), B, hw, hw, 2, 2e-3) for _ in range(60)]
    assert losses[-1] < 0.3 * losses[0], losses[::10]


@pytest.mark.parametrize("chans,hw", [((32, 64), 64), ((32, 64), 96), ((32, 64, 128, 256, 256), 256), ((64, 64), 64)])
def test_predict_matches_forward_with_constant_planes(chans, hw):
    # inference reads phi and the constant planes itself (the first layer with its input
    # packed into K; at 32 first-level channels the whole first block in one launch, its
    # intermediate kept in LDS): bit for bit the forward pass on the packed input
    import torch
    from paper_2501_03759_amd import lbsg
    c_in = 4
    net = lbsg.Surrogate(chans, c_in, 1, hw, hw, train=False, seed=4)
    params = net.get_params()
    rng = np.random.default_rng(2)
    params[-(chans[0] + 1):] = rng.normal(size=chans[0] + 1).astype(np.float32) * 0.1
    net.set_params(params)
    phi = rng.normal(size=(hw, hw)).astype(np.float32)
    cond = [0.2, -0.5, 0.75]
    x = np.concatenate([phi[..., None], np.broadcast_to(np.array(cond, np.float32), (hw, hw, 3))], axis=2)[None]
    xt = torch.tensor(np.ascontiguousarray(x), device="cuda")
    a = torch.empty((1, hw, hw), dtype=torch.float32, device="cuda")
    b = torch.empty((hw, hw), dtype=torch.float32, device="cuda")
    net.forward(xt.data_ptr(), 1, hw, hw, a.data_ptr())
    pt = torch.tensor(phi, device="cuda")
    net.predict(pt.data_ptr(), cond, hw, hw, b.data_ptr())
    torch.cuda.synchronize()
    got = b.cpu().numpy()
    assert np.array_equal(a.cpu().numpy()[0], got)
    assert np.abs(got - phi).max() > 1e-3          # the network's residual is not trivially zero


def test_trained_network_gains_over_the_jump_without_it():
    # Trained on lattice Boltzmann pairs (phi(t), phi(t + K)) of seeded spinodal runs, the network
    # predicts held-out runs much better than the jump without it (phi(t + K) ~ phi(t)).  Trained
    # on the residual of the rate-extrapolated jump, it is measured against the extrapolation alone
    # (reported; it must not make the jump worse).
    import torch
    from paper_2501_03759_amd import lbsg, surrogate_train as st
    stream = torch.cuda.Stream()
    side, K = 128, 100
    with torch.cuda.stream(stream):
        runs, held = st.draw_runs(48, seed=11), st.draw_runs(6, seed=12)
        out = {}
        for extrap in (False, True):
            kw = dict(stream=stream, log=lambda m: None, amp=0.5, extrapolate=extrap)
            X, Y = st.generate(runs, side, 1500, 5500, 250, K, side, 1, seed=1, **kw)
            Xh, Yh = st.generate(held, side, 1750, 5250, 500, K, side, 1, seed=2, **kw)
            net = lbsg.Surrogate((32, 32), 5, 16, side, side, train=True, seed=0, stream=stream, out_scale=0.02)
            st.train(net, X, Y, epochs=20, batch=16, lr=1e-3, margin=0, log=lambda m: None)
            out[extrap] = st.evaluate(net, Xh, Yh, margin=0)
            net.close()
            del X, Y, Xh, Yh
    (rn, ri), (re_, rl) = out[False], out[True]
    print(f"held-out rel-L2: network {rn:.3e} vs no jump {ri:.3e}; "
          f"extrapolation + network {re_:.3e} vs extrapolation alone {rl:.3e}")
    assert rn < 0.7 * ri
    assert re_ < 1.2 * rl

