"""The warm-start network's layers on the GPU against the FP64 oracle (oracle/nn_oracle.py).

Inputs and weights are rounded to bfloat16 first, so both sides start from identical
values; the GPU accumulates in binary32 on the matrix cores and rounds its bf16 outputs
to nearest (relative error <= 2^-9), which sets the tolerances."""
import sys

import numpy as np
import pytest
import torch

from oracle import nn_oracle as N
from paper_1410_1921_amd import nn
from paper_1410_1921_amd.nn import View
from paper_1410_1921_amd.unet import LEVELS, UNet

pytestmark = pytest.mark.gpu
BF = 2.0 ** -8  # bf16 spacing relative to the value (rounding error <= half of it)


def say(*a):
    print("[gpu-nn]", *a, flush=True)
    sys.stdout.flush()


def bf16(a):
    """float64 array rounded to bfloat16 values (as float64)."""
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def to_dev_cl(a_cf, cs=None, off=0):
    """channels-first float64 [C, Z, Y, X] -> channels-last bf16 device tensor [nvox, cs]."""
    c = a_cf.shape[0]
    cs = c if cs is None else cs
    t = torch.zeros((int(np.prod(a_cf.shape[1:])), cs), dtype=torch.bfloat16)
    t[:, off:off + c] = torch.from_numpy(a_cf.reshape(c, -1).T.copy()).to(torch.bfloat16)
    return t.cuda()


def from_dev_cl(t, shape, off=0, c=None):
    c = t.shape[1] - off if c is None else c
    a = t.float().cpu().numpy()[:, off:off + c].astype(np.float64)
    return a.T.reshape((c,) + tuple(shape))


def w_dev(w):
    """oracle weights [27, Co, Ci] -> bf16 device [27][co][ci]."""
    return torch.from_numpy(np.ascontiguousarray(w, np.float32)).to(torch.bfloat16).reshape(-1).cuda()


def close(gpu, ref, rel=BF, floor=1e-3):
    err = np.abs(gpu - ref)
    bound = rel * np.abs(ref) + floor * np.abs(ref).max()
    return bool((err <= bound).all()), float(err.max()), float(np.abs(ref).max())


# sizes not all divisible by 4 take the per-voxel-tile kernel, the others the brick
# kernel (input halo staged in LDS)
@pytest.mark.parametrize("shape,cin,cout", [((6, 8, 10), 16, 16), ((4, 6, 8), 32, 48),
                                            ((3, 4, 8), 192, 64), ((2, 4, 4), 64, 128),
                                            ((5, 4, 4), 96, 32), ((8, 12, 16), 16, 16),
                                            ((4, 8, 4), 32, 48), ((12, 12, 12), 128, 128),
                                            ((4, 4, 8), 192, 64), ((8, 4, 4), 96, 32)])
def test_conv3d_forward(shape, cin, cout):
    rng = np.random.default_rng(cin * 7 + cout)
    x = bf16(rng.standard_normal((cin,) + shape))
    w = bf16(rng.standard_normal((27, cout, cin)) * (2.0 / (27 * cin)) ** 0.5)
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    say("conv fwd", shape, cin, cout)
    xd = to_dev_cl(x, cs=cin + 16, off=16)  # a view at channel offset 16
    y = torch.zeros((x[0].size, cout + 32), dtype=torch.bfloat16, device="cuda")
    nn.lbm_nn_conv3d(shape, View(xd, 16, cin), cin, w_dev(w),
                     torch.from_numpy(b.astype(np.float32)).cuda(), View(y, 32, cout), cout,
                     nn.LBM_NN_RELU)
    ref = N.relu(N.conv3d(x, w, b))
    got = from_dev_cl(y, shape, 32, cout)
    ok, err, scale = close(got, ref)
    say("worst", err, "scale", scale)
    assert ok
    # channels outside the view are untouched
    assert (y[:, :32].float() == 0).all()


@pytest.mark.parametrize("shape,cin,cout", [((4, 6, 8), 48, 16), ((2, 4, 6), 192, 64),
                                            ((4, 4, 4), 16, 32), ((8, 8, 12), 32, 16),
                                            ((12, 12, 12), 64, 128)])
def test_conv3d_input_gradient(shape, cin, cout):
    rng = np.random.default_rng(3 + cin)
    w = bf16(rng.standard_normal((27, cout, cin)) * 0.1)
    gy = bf16(rng.standard_normal((cout,) + shape))
    say("conv bwd-data", shape, cin, cout)
    wt = torch.zeros(27 * cin * cout, dtype=torch.bfloat16, device="cuda")
    nn.lbm_nn_transpose_weights(w_dev(w), cout, cin, wt)
    gx = torch.zeros((gy[0].size, cin), dtype=torch.bfloat16, device="cuda")
    nn.lbm_nn_conv3d(shape, View(to_dev_cl(gy)), cout, wt, None, View(gx), cin, nn.LBM_NN_FLIP)
    ref, _, _ = N.conv3d_bwd(np.zeros((cin,) + shape), w, gy)
    ok, err, scale = close(from_dev_cl(gx, shape), ref)
    say("worst", err, "scale", scale)
    assert ok


# grids with a size not divisible by 4 take the per-tap kernel; the others the brick
# kernel (operands staged in LDS), also through strided channel views (x_off, g_off:
# channel offsets of the views in wider tensors, as for the decoder's concatenations)
@pytest.mark.parametrize("shape,cin,cout,x_off,g_off",
                         [((6, 8, 10), 16, 16, 0, 0), ((4, 6, 8), 96, 32, 0, 0),
                          ((2, 4, 6), 64, 128, 0, 0), ((8, 8, 8), 48, 16, 0, 0),
                          ((8, 12, 16), 16, 16, 0, 0), ((4, 8, 12), 32, 64, 16, 0),
                          ((12, 12, 12), 128, 128, 0, 0), ((4, 4, 4), 192, 64, 0, 32),
                          ((8, 4, 12), 48, 16, 16, 16), ((4, 4, 8), 16, 16, 4, 0)])
def test_conv3d_weight_gradient(shape, cin, cout, x_off, g_off):
    rng = np.random.default_rng(11 + cout)
    x = bf16(rng.standard_normal((cin,) + shape))
    g = bf16(rng.standard_normal((cout,) + shape))
    say("conv wgrad", shape, cin, cout, x_off, g_off)
    dw = torch.zeros(27 * cout * cin, dtype=torch.float32, device="cuda")
    db = torch.zeros(cout, dtype=torch.float32, device="cuda")
    ws = torch.empty(nn.lbm_nn_wgrad_workspace(shape, cin, cout), dtype=torch.uint8, device="cuda")
    xd = View(to_dev_cl(x, cin + x_off, x_off), x_off, cin)
    gd = View(to_dev_cl(g, cout + g_off, g_off), g_off, cout)
    nn.lbm_nn_conv3d_wgrad(shape, xd, cin, gd, cout, dw, db, ws)
    _, gw, gb = N.conv3d_bwd(x, np.zeros((27, cout, cin)), g)
    gw_gpu = dw.cpu().numpy().astype(np.float64).reshape(27, cout, cin)
    # binary32 sums of bf16 products: ~1e-6 of the sum of |terms|
    tol = 1e-5 * np.sqrt(x[0].size) * 4
    assert np.abs(gw_gpu - gw).max() <= tol, np.abs(gw_gpu - gw).max()
    assert np.abs(db.cpu().numpy() - gb).max() <= tol
    # accumulate adds
    nn.lbm_nn_conv3d_wgrad(shape, xd, cin, gd, cout, dw, db, ws, accumulate=True)
    assert np.abs(dw.cpu().numpy().astype(np.float64).reshape(27, cout, cin) - 2 * gw).max() <= 2 * tol


# c = 16: four channels per thread; c = 6: one (the channel count is not a multiple of 4)
@pytest.mark.parametrize("c", [16, 6])
def test_pool_and_upsample(c):
    rng = np.random.default_rng(7)
    shape = (4, 6, 8)
    x = bf16(rng.standard_normal((c,) + shape))
    xc = bf16(rng.standard_normal((c, 2, 3, 4)))
    y = torch.zeros((2 * 3 * 4, c), dtype=torch.bfloat16, device="cuda")
    nn.lbm_nn_pool2(shape, c, View(to_dev_cl(x)), View(y))
    assert close(from_dev_cl(y, (2, 3, 4)), N.avgpool2(x))[0]
    gx = torch.zeros((x[0].size, c), dtype=torch.bfloat16, device="cuda")
    nn.lbm_nn_pool2_bwd(shape, c, View(to_dev_cl(xc)), View(gx))
    assert close(from_dev_cl(gx, shape), N.avgpool2_bwd(xc))[0]
    nn.lbm_nn_pool2_bwd(shape, c, View(to_dev_cl(xc)), View(gx), accumulate=True)
    assert close(from_dev_cl(gx, shape), 2 * N.avgpool2_bwd(xc))[0]
    u = torch.zeros((x[0].size, c + 16), dtype=torch.bfloat16, device="cuda")
    nn.lbm_nn_up2(shape, c, View(to_dev_cl(xc)), View(u, 16, c))
    assert np.array_equal(from_dev_cl(u, shape, 16, c), N.upsample2(xc))
    gu = torch.zeros((2 * 3 * 4, c), dtype=torch.bfloat16, device="cuda")
    nn.lbm_nn_up2_bwd(shape, c, View(to_dev_cl(x)), View(gu))
    assert close(from_dev_cl(gu, (2, 3, 4)), N.upsample2_bwd(x))[0]


@pytest.mark.parametrize("c", [16, 6])
def test_relu_gradient(c):
    # g = gy where y > 0 (exactly: a selection of bf16 values), through strided views
    rng = np.random.default_rng(5)
    shape = (4, 6, 8)
    y = bf16(rng.standard_normal((c,) + shape))
    y[:, 0, 0, :2] = 0.0  # zeros pass nothing
    gy = bf16(rng.standard_normal((c,) + shape))
    g = torch.zeros((y[0].size, c + 8), dtype=torch.bfloat16, device="cuda")
    nn.lbm_nn_relu_bwd(c, View(to_dev_cl(y)), View(to_dev_cl(gy)), View(g, 8, c))
    assert np.array_equal(from_dev_cl(g, shape, 8, c), np.where(y > 0, gy, 0.0))
    assert (g[:, :8].float() == 0).all()


def test_head_loss_and_gradients():
    rng = np.random.default_rng(9)
    shape = (4, 8, 6)
    nvox = int(np.prod(shape))
    no = 5
    x = bf16(rng.standard_normal((16,) + shape))
    wh = rng.standard_normal((no, 16)).astype(np.float32).astype(np.float64)
    bh = rng.standard_normal(no).astype(np.float32).astype(np.float64)
    tgt = rng.standard_normal((no,) + shape).astype(np.float32).astype(np.float64)
    mask = (rng.random(shape) < 0.6).astype(np.uint8)
    wt = np.array([1.0, 1.0, 1.0, 0.5, 2.0])
    out = torch.zeros((no, nvox), dtype=torch.float32, device="cuda")
    gx = torch.zeros((nvox, 16), dtype=torch.bfloat16, device="cuda")
    gwh = torch.zeros(no * 16, dtype=torch.float32, device="cuda")
    gbh = torch.zeros(no, dtype=torch.float32, device="cuda")
    ws = torch.empty(nn.lbm_nn_head_workspace(nvox, no), dtype=torch.uint8, device="cuda")
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    loss = nn.lbm_nn_head(View(to_dev_cl(x)), no, f32(wh), f32(bh), out=out,
                          target=f32(tgt.reshape(no, -1)), mask=torch.from_numpy(mask.reshape(-1)).cuda(),
                          wt=f32(wt), n_mask=float(mask.sum()), gx=View(gx), gwh=gwh, gbh=gbh, ws=ws)
    ref_out = N.head(x, wh, bh)
    ref_loss, g = N.masked_mse(ref_out, tgt, mask.astype(float), wt)
    assert np.allclose(out.cpu().numpy().reshape((no,) + shape), ref_out, rtol=1e-5, atol=1e-5)
    assert loss == pytest.approx(ref_loss, rel=1e-5)
    gw_ref = np.tensordot(g, x, axes=([1, 2, 3], [1, 2, 3]))
    assert np.allclose(gwh.cpu().numpy().reshape(no, 16), gw_ref, rtol=1e-4, atol=1e-6)
    assert np.allclose(gbh.cpu().numpy(), g.sum(axis=(1, 2, 3)), rtol=1e-4, atol=1e-6)
    gx_ref = np.tensordot(wh, g, axes=([0], [0]))
    assert close(from_dev_cl(gx, shape), gx_ref)[0]


def _oracle_params(net):
    """The network's bf16-rounded weights in the oracle's layout (first layer: the 2 used
    input channels)."""
    p = net.params()
    q = {}
    for k, v in p.items():
        q[k] = bf16(v) if k.endswith(".w") and not k.startswith("head") else v
    q["enc0a.w"] = q["enc0a.w"][:, :, :2]
    return q


def test_unet_gradient_against_oracle():
    shape = (16, 16, 32)
    rng = np.random.default_rng(21)
    net = UNet(n_out=5, seed=3)
    x = np.zeros((16,) + shape)
    x[0] = (rng.random(shape) < 0.5)
    x[1] = bf16(rng.random(shape) * 2.0)
    tgt = rng.standard_normal((5,) + shape) * 0.1
    mask = (x[0] > 0).astype(np.uint8)
    wt = np.array([1.0, 1.0, 1.0, 1.0, 1.0])
    say("unet gradient", shape)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    loss = net.loss_and_grad(shape, to_dev_cl(x), f32(tgt.reshape(5, -1)),
                             torch.from_numpy(mask.reshape(-1)).cuda(), f32(wt), float(mask.sum()))
    g_gpu = net.grads()
    q = _oracle_params(net)
    out, cache = N.unet_forward(q, x[:2])
    ref_loss, gout = N.masked_mse(out, tgt.astype(np.float32).astype(np.float64), mask.astype(float), wt)
    g_ref = N.unet_backward(q, cache, gout)
    say("loss", loss, ref_loss)
    assert loss == pytest.approx(ref_loss, rel=2e-2)
    worst = 0.0
    for k in g_ref:
        a, r = g_gpu[k], g_ref[k]
        if k == "enc0a.w":
            a = a[:, :, :2]
        rel = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
        cos = float((a * r).sum() / (np.linalg.norm(a) * np.linalg.norm(r) + 1e-30))
        worst = max(worst, rel)
        # bf16 activations between layers: a few percent of each layer's gradient
        assert rel < 0.1 and cos > 0.99, (k, rel, cos)
    say("worst relative gradient error", worst)


def test_unet_trains_and_is_deterministic():
    shape = (16, 16, 32)
    rng = np.random.default_rng(5)
    net = UNet(n_out=2, seed=1)
    x = np.zeros((16,) + shape)
    x[0] = 1.0
    x[1] = bf16(rng.random(shape))
    # a smooth target the network can fit: a ramp and the scaled diameter channel
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    tgt = np.stack([xx / shape[2], 0.5 * x[1]])
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    xd, td = to_dev_cl(x), f32(tgt.reshape(2, -1))
    mask = torch.ones(int(np.prod(shape)), dtype=torch.uint8, device="cuda")
    wt = f32([1.0, 1.0])
    o1 = net.forward(shape, xd).clone()
    o2 = net.forward(shape, xd).clone()
    assert torch.equal(o1, o2)
    losses = []
    for it in range(60):
        losses.append(net.loss_and_grad(shape, xd, td, mask, wt, float(mask.numel())))
        net.adam(lr=3e-3)
    say("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.2 * losses[0]
