"""FP64 CPU oracle for the learned warm start (test infrastructure, like the rest of
``oracle/``: only the tests may import it).

The network is a 3D U-Net that maps a voxel geometry (pore mask and pore-diameter map)
to initial flow and concentration fields.  The paper has no such part; the oracle holds
the plain definitions the GPU kernels must reproduce:

* ``conv3d``: 3x3x3 cross-correlation with zero padding, y[co, v] = b[co] +
  sum_t sum_ci w[t, co, ci] x[ci, v + d_t], tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1).
* ``avgpool2`` / ``upsample2``: 2x2x2 mean, and nearest-neighbour copy to the 8 children.
* ``head``: 1x1x1 linear map to the output channels; ``masked_mse``: the mean over
  fluid voxels of sum_o wt_o (out_o - target_o)^2.
* ``unet_forward`` / ``unet_backward``: 4 levels (16, 32, 64, 128 channels), two
  ReLU convolutions per level, skip connections concatenated as [skip, upsampled].

Pins (tests/test_oracle_nn.py): conv3d against ``scipy.ndimage.correlate`` channel by
channel; every backward against central finite differences of its forward;
``avgpool2`` / ``upsample2`` adjointness and constant preservation.
Arrays are channels-first [C, Z, Y, X] in float64.
"""
import numpy as np

LEVELS = (16, 32, 64, 128)


def _taps():
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shifted(x, dz, dy, dx):
    """s[..., z, y, x] = x[..., z + dz, y + dy, x + dx], zero outside."""
    out = np.zeros_like(x)
    Z, Y, X = x.shape[-3:]
    zs, ys, xs = slice(max(0, -dz), min(Z, Z - dz)), slice(max(0, -dy), min(Y, Y - dy)), \
        slice(max(0, -dx), min(X, X - dx))
    zt, yt, xt = slice(max(0, dz), min(Z, Z + dz)), slice(max(0, dy), min(Y, Y + dy)), \
        slice(max(0, dx), min(X, X + dx))
    out[..., zs, ys, xs] = x[..., zt, yt, xt]
    return out


def conv3d(x, w, b=None):
    """x [Ci, Z, Y, X], w [27, Co, Ci], b [Co] -> y [Co, Z, Y, X]."""
    co = w.shape[1]
    y = np.zeros((co,) + x.shape[1:])
    for t, (dz, dy, dx) in enumerate(_taps()):
        xs = _shifted(x, dz, dy, dx)
        y += np.tensordot(w[t], xs, axes=([1], [0]))
    if b is not None:
        y += b[:, None, None, None]
    return y


def conv3d_bwd(x, w, gy):
    """Gradients of sum(gy * conv3d(x, w, b)) with respect to x, w and b."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for t, (dz, dy, dx) in enumerate(_taps()):
        xs = _shifted(x, dz, dy, dx)
        gw[t] = np.tensordot(gy, xs, axes=([1, 2, 3], [1, 2, 3]))
        # y[v] uses x[v + d]; the adjoint moves gy back by -d
        gx += _shifted(np.tensordot(w[t], gy, axes=([0], [0])), -dz, -dy, -dx)
    gb = gy.sum(axis=(1, 2, 3))
    return gx, gw, gb


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    C, Z, Y, X = x.shape
    return x.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).mean(axis=(2, 4, 6))


def avgpool2_bwd(gy):
    return np.repeat(np.repeat(np.repeat(gy, 2, 1), 2, 2), 2, 3) / 8.0


def upsample2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 1), 2, 2), 2, 3)


def upsample2_bwd(gy):
    C, Z, Y, X = gy.shape
    return gy.reshape(C, Z // 2, 2, Y // 2, 2, X // 2, 2).sum(axis=(2, 4, 6))


def head(x, wh, bh):
    """1x1x1 map: x [16, Z, Y, X], wh [No, 16], bh [No] -> [No, Z, Y, X]."""
    return np.tensordot(wh, x, axes=([1], [0])) + bh[:, None, None, None]


def masked_mse(out, target, mask, wt):
    """Loss and its gradient with respect to out."""
    n = max(float(mask.sum()), 1.0)
    d = (out - target) * mask[None]
    loss = float((wt[:, None, None, None] * d * d).sum() / n)
    g = 2.0 * wt[:, None, None, None] * d / n
    return loss, g


def unet_init(rng, c_in=2, c_out=5, levels=LEVELS):
    """He-normal weights in the oracle's layout (a dict of float64 arrays)."""
    p = {}

    def conv(name, ci, co):
        p[name + ".w"] = rng.standard_normal((27, co, ci)) * np.sqrt(2.0 / (27 * ci))
        p[name + ".b"] = np.zeros(co)

    prev = c_in
    for i, c in enumerate(levels):
        conv(f"enc{i}a", prev, c)
        conv(f"enc{i}b", c, c)
        prev = c
    for i in range(len(levels) - 2, -1, -1):
        conv(f"dec{i}a", levels[i] + levels[i + 1], levels[i])
        conv(f"dec{i}b", levels[i], levels[i])
    p["head.w"] = rng.standard_normal((c_out, levels[0])) * np.sqrt(1.0 / levels[0])
    p["head.b"] = np.zeros(c_out)
    return p


def unet_forward(p, x, levels=LEVELS):
    """Returns the output and the cache the backward needs."""
    cache = {}
    h = x
    skips = []
    L = len(levels)
    for i in range(L):
        if i > 0:
            h = avgpool2(h)
        for s in "ab":
            cache[f"enc{i}{s}.in"] = h
            h = relu(conv3d(h, p[f"enc{i}{s}.w"], p[f"enc{i}{s}.b"]))
            cache[f"enc{i}{s}.out"] = h
        skips.append(h)
    for i in range(L - 2, -1, -1):
        h = np.concatenate([skips[i], upsample2(h)], axis=0)
        for s in "ab":
            cache[f"dec{i}{s}.in"] = h
            h = relu(conv3d(h, p[f"dec{i}{s}.w"], p[f"dec{i}{s}.b"]))
            cache[f"dec{i}{s}.out"] = h
    cache["head.in"] = h
    return head(h, p["head.w"], p["head.b"]), cache


def unet_backward(p, cache, gout, levels=LEVELS):
    """Gradients of sum(gout * out) with respect to every parameter."""
    g = {}
    L = len(levels)
    x = cache["head.in"]
    g["head.w"] = np.tensordot(gout, x, axes=([1, 2, 3], [1, 2, 3]))
    g["head.b"] = gout.sum(axis=(1, 2, 3))
    gh = np.tensordot(p["head.w"], gout, axes=([0], [0]))
    gskip = [None] * L

    def conv_back(name, gh):
        out = cache[name + ".out"]
        gpre = gh * (out > 0)
        gx, g[name + ".w"], g[name + ".b"] = conv3d_bwd(cache[name + ".in"], p[name + ".w"], gpre)
        return gx

    for i in range(L - 1):
        gh = conv_back(f"dec{i}b", gh)
        gh = conv_back(f"dec{i}a", gh)
        c = levels[i]
        gskip[i] = gh[:c]
        gh = upsample2_bwd(gh[c:])
    for i in range(L - 1, -1, -1):
        if gskip[i] is not None:
            gh = gh + gskip[i]
        gh = conv_back(f"enc{i}b", gh)
        gh = conv_back(f"enc{i}a", gh)
        if i > 0:
            gh = avgpool2_bwd(gh)
    return g
