"""Thin binding of include/lbm_nn.h (the layers of the warm-start network): argument
marshalling only, every layer runs in liblbm.so's kernels.

A ``View`` is a channels-last bf16 tensor view: a torch.bfloat16 tensor [nvox, cs]
plus a channel offset and a channel count, the layout the kernels expect."""
import ctypes as C

import torch

from .lbm import _check, _n3, _ptr, _stream, load

LBM_NN_RELU, LBM_NN_FLIP = 1, 2


class View:
    __slots__ = ("t", "off", "c")

    def __init__(self, t, off=0, c=None):
        if not (t.is_cuda and t.dtype == torch.bfloat16 and t.dim() == 2 and t.is_contiguous()):
            raise ValueError("a View needs a contiguous 2-D bfloat16 CUDA tensor [nvox, cs]")
        self.t, self.off = t, off
        self.c = t.shape[1] - off if c is None else c
        if off < 0 or off % 4 or off + self.c > t.shape[1]:
            raise ValueError("View: channel range outside the tensor or misaligned")

    @property
    def ptr(self):
        return C.c_void_p(self.t.data_ptr() + 2 * self.off)

    @property
    def cs(self):
        return self.t.shape[1]

    @property
    def nvox(self):
        return self.t.shape[0]


def _need(ok, what):
    if not ok:
        raise ValueError(what)


def _nv(shape):
    nz, ny, nx = shape
    return nz * ny * nx


def _len(t, n):
    return t is None or t.numel() == n


def _bf(t):
    if t is None:
        return C.c_void_p(0)
    if not (t.is_cuda and t.dtype == torch.bfloat16 and t.is_contiguous()):
        raise ValueError("expected a contiguous bfloat16 CUDA tensor")
    return _ptr(t)


def _f32(t):
    if t is None:
        return C.c_void_p(0)
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return _ptr(t)


def lbm_nn_conv3d(shape, x, cin, w, bias, y, cout, flags):
    _need(x.nvox == y.nvox == _nv(shape) and cin <= x.c and cout <= y.c,
          "lbm_nn_conv3d: views do not hold the grid's voxels and channels")
    _need(w.numel() == 27 * cin * cout and _len(bias, cout), "lbm_nn_conv3d: weight sizes")
    _check(load().lbm_nn_conv3d(_n3(shape), x.ptr, x.cs, cin, _bf(w), _f32(bias), y.ptr, y.cs,
                                cout, flags, _stream()), "lbm_nn_conv3d")


def lbm_nn_wgrad_workspace(shape, cin, cout):
    return int(load().lbm_nn_wgrad_workspace(_n3(shape), cin, cout))


def lbm_nn_conv3d_wgrad(shape, x, cin, g, cout, dw, db, ws, accumulate=False):
    _need(x.nvox == g.nvox == _nv(shape) and cin <= x.c and cout <= g.c,
          "lbm_nn_conv3d_wgrad: views do not hold the grid's voxels and channels")
    _need(dw.numel() == 27 * cin * cout and _len(db, cout), "lbm_nn_conv3d_wgrad: gradient sizes")
    _check(load().lbm_nn_conv3d_wgrad(_n3(shape), x.ptr, x.cs, cin, g.ptr, g.cs, cout, _f32(dw),
                                      _f32(db), int(accumulate), _ptr(ws), ws.numel(), _stream()),
           "lbm_nn_conv3d_wgrad")


def lbm_nn_transpose_weights(w, cout, cin, wt):
    _need(w.numel() == wt.numel() == 27 * cin * cout, "lbm_nn_transpose_weights: sizes")
    _check(load().lbm_nn_transpose_weights(_bf(w), cout, cin, _bf(wt), _stream()),
           "lbm_nn_transpose_weights")


def lbm_nn_pool2(shape_fine, c, x, y, accumulate=False):
    _need(x.nvox == _nv(shape_fine) and 8 * y.nvox == _nv(shape_fine) and c <= min(x.c, y.c),
          "lbm_nn_pool2: views do not hold the fine and coarse grids")
    _check(load().lbm_nn_pool2(_n3(shape_fine), c, x.ptr, x.cs, y.ptr, y.cs, int(accumulate),
                               _stream()), "lbm_nn_pool2")


def lbm_nn_pool2_bwd(shape_fine, c, gy, gx, accumulate=False):
    _need(8 * gy.nvox == _nv(shape_fine) and gx.nvox == _nv(shape_fine) and c <= min(gy.c, gx.c),
          "lbm_nn_pool2_bwd: views do not hold the coarse and fine grids")
    _check(load().lbm_nn_pool2_bwd(_n3(shape_fine), c, gy.ptr, gy.cs, gx.ptr, gx.cs,
                                   int(accumulate), _stream()), "lbm_nn_pool2_bwd")


def lbm_nn_up2(shape_fine, c, x, y):
    _need(8 * x.nvox == _nv(shape_fine) and y.nvox == _nv(shape_fine) and c <= min(x.c, y.c),
          "lbm_nn_up2: views do not hold the coarse and fine grids")
    _check(load().lbm_nn_up2(_n3(shape_fine), c, x.ptr, x.cs, y.ptr, y.cs, _stream()),
           "lbm_nn_up2")


def lbm_nn_up2_bwd(shape_fine, c, gy, gx):
    _need(gy.nvox == _nv(shape_fine) and 8 * gx.nvox == _nv(shape_fine) and c <= min(gy.c, gx.c),
          "lbm_nn_up2_bwd: views do not hold the fine and coarse grids")
    _check(load().lbm_nn_up2_bwd(_n3(shape_fine), c, gy.ptr, gy.cs, gx.ptr, gx.cs, _stream()),
           "lbm_nn_up2_bwd")


def lbm_nn_relu_bwd(c, y, gy, g):
    _need(y.nvox == gy.nvox == g.nvox and c <= min(y.c, gy.c, g.c), "lbm_nn_relu_bwd: views differ")
    _check(load().lbm_nn_relu_bwd(y.nvox, c, y.ptr, y.cs, gy.ptr, gy.cs, g.ptr, g.cs, _stream()),
           "lbm_nn_relu_bwd")


def lbm_nn_head_workspace(nvox, no):
    return int(load().lbm_nn_head_workspace(nvox, no))


def lbm_nn_head(x, no, wh, bh, out=None, target=None, mask=None, wt=None, n_mask=0.0, gx=None,
                gwh=None, gbh=None, ws=None):
    """Returns the loss (with a target) or None."""
    nv = x.nvox
    _need(x.c >= 16 and wh.numel() == 16 * no and _len(bh, no) and _len(out, no * nv)
          and _len(target, no * nv) and _len(mask, nv) and _len(wt, no)
          and (gx is None or (gx.nvox == nv and gx.c >= 16)), "lbm_nn_head: sizes")
    loss = C.c_double(0.0)
    _check(load().lbm_nn_head(x.nvox, x.ptr, x.cs, no, _f32(wh), _f32(bh), _f32(out), _f32(target),
                              _ptr(mask), _f32(wt), float(n_mask),
                              gx.ptr if gx is not None else C.c_void_p(0),
                              gx.cs if gx is not None else 16, _f32(gwh), _f32(gbh),
                              C.byref(loss), _ptr(ws), 0 if ws is None else ws.numel(), _stream()),
           "lbm_nn_head")
    return loss.value if target is not None else None


def lbm_nn_adam(w, g, m, v, w_bf16, lr, beta1, beta2, eps, step):
    _need(g.numel() == m.numel() == v.numel() == w.numel() and _len(w_bf16, w.numel()),
          "lbm_nn_adam: sizes")
    _check(load().lbm_nn_adam(w.numel(), _f32(w), _f32(g), _f32(m), _f32(v), _bf(w_bf16), lr, beta1,
                              beta2, eps, step, _stream()), "lbm_nn_adam")


def lbm_nn_to_bf16(src, dst):
    _need(dst.numel() == src.numel(), "lbm_nn_to_bf16: sizes")
    _check(load().lbm_nn_to_bf16(src.numel(), _f32(src), _bf(dst), _stream()), "lbm_nn_to_bf16")


def lbm_nn_make_input(mask, diam, d_scale, x):
    if not (mask.dtype == torch.uint8 and diam.dtype == torch.float64 and mask.is_cuda
            and diam.is_cuda and mask.numel() == diam.numel() == x.nvox):
        raise ValueError("lbm_nn_make_input: uint8 mask and float64 diameters of the grid")
    _check(load().lbm_nn_make_input(x.nvox, _ptr(mask), _ptr(diam), float(d_scale), x.ptr, x.cs,
                                    _stream()), "lbm_nn_make_input")


def lbm_nn_to_fields(out, mask, scale, fields):
    nk = out.shape[0]
    _need(out.numel() == nk * mask.numel() and fields.numel() >= nk * mask.numel()
          and scale.numel() >= nk, "lbm_nn_to_fields: sizes")
    _check(load().lbm_nn_to_fields(mask.numel(), nk, _f32(out), _ptr(mask), _f32(scale),
                                   _f32(fields), _stream()), "lbm_nn_to_fields")
