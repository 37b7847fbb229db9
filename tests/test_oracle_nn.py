"""Pins of the warm-start network oracle: the convolution against scipy's
cross-correlation, every backward against central finite differences of its forward,
and the pooling / upsampling adjoint pair."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import nn_oracle as N


def test_conv3d_is_zero_padded_cross_correlation():
    rng = np.random.default_rng(1)
    ci, co = 3, 2
    x = rng.standard_normal((ci, 5, 6, 7))
    w = rng.standard_normal((27, co, ci))
    b = rng.standard_normal(co)
    y = N.conv3d(x, w, b)
    for o in range(co):
        ref = np.full(x.shape[1:], b[o])
        for i in range(ci):
            k = w[:, o, i].reshape(3, 3, 3)  # [dz + 1, dy + 1, dx + 1]
            ref += ndimage.correlate(x[i], k, mode="constant", cval=0.0)
        assert np.allclose(y[o], ref, rtol=1e-13, atol=1e-13)


def test_conv3d_single_tap_shifts():
    # a one-hot kernel at offset d returns x shifted by d (zero beyond the box)
    x = np.arange(4 * 5 * 6, dtype=float).reshape(1, 4, 5, 6)
    for t, (dz, dy, dx) in enumerate(N._taps()):
        w = np.zeros((27, 1, 1))
        w[t] = 1.0
        y = N.conv3d(x, w)[0]
        for z, yy, xx in [(0, 0, 0), (3, 4, 5), (2, 1, 3)]:
            zz, y2, x2 = z + dz, yy + dy, xx + dx
            inside = 0 <= zz < 4 and 0 <= y2 < 5 and 0 <= x2 < 6
            assert y[z, yy, xx] == (x[0, zz, y2, x2] if inside else 0.0)


def _fd_check(f, args, grads, rng, eps=1e-6, rel=1e-6):
    """Directional finite differences of the scalar f along random directions of each
    argument against the analytic gradients."""
    for k, (a, g) in enumerate(zip(args, grads)):
        d = rng.standard_normal(a.shape)
        plus = [x.copy() for x in args]
        minus = [x.copy() for x in args]
        plus[k] = a + eps * d
        minus[k] = a - eps * d
        fd = (f(*plus) - f(*minus)) / (2 * eps)
        an = float((g * d).sum())
        assert fd == pytest.approx(an, rel=rel, abs=1e-9), k


def test_conv3d_backward_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 5, 3))
    w = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(2)
    gy = rng.standard_normal((2, 4, 5, 3))
    gx, gw, gb = N.conv3d_bwd(x, w, gy)
    _fd_check(lambda x, w, b: float((gy * N.conv3d(x, w, b)).sum()), [x, w, b], [gx, gw, gb], rng)


def test_pool_upsample_adjoint_and_constants():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 4, 6, 8))
    y = rng.standard_normal((2, 2, 3, 4))
    assert np.dot(N.avgpool2(x).ravel(), y.ravel()) == pytest.approx(
        np.dot(x.ravel(), N.avgpool2_bwd(y).ravel()), rel=1e-13)
    assert np.dot(N.upsample2(y).ravel(), x.ravel()) == pytest.approx(
        np.dot(y.ravel(), N.upsample2_bwd(x).ravel()), rel=1e-13)
    c = np.full((1, 4, 4, 4), 2.5)
    assert np.all(N.avgpool2(c) == 2.5) and np.all(N.upsample2(N.avgpool2(c)) == 2.5)
    # mean of the 8 children, by hand for one parent
    assert N.avgpool2(x)[1, 1, 2, 3] == pytest.approx(x[1, 2:4, 4:6, 6:8].mean(), rel=1e-15)


def test_masked_mse_and_head_gradients():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((4, 3, 3, 2))
    wh = rng.standard_normal((3, 4))
    bh = rng.standard_normal(3)
    tgt = rng.standard_normal((3, 3, 3, 2))
    mask = (rng.random((3, 3, 2)) < 0.6).astype(float)
    wt = np.array([1.0, 0.5, 2.0])

    def f(x, wh, bh):
        return N.masked_mse(N.head(x, wh, bh), tgt, mask, wt)[0]

    loss, g = N.masked_mse(N.head(x, wh, bh), tgt, mask, wt)
    gx = np.tensordot(wh, g, axes=([0], [0]))
    gw = np.tensordot(g, x, axes=([1, 2, 3], [1, 2, 3]))
    gb = g.sum(axis=(1, 2, 3))
    _fd_check(f, [x, wh, bh], [gx, gw, gb], rng)
    # voxels outside the mask do not count
    assert loss == pytest.approx(float((wt[:, None, None, None] * ((N.head(x, wh, bh) - tgt)
                                                                  * mask) ** 2).sum()
                                       / mask.sum()), rel=1e-14)


def test_unet_backward_finite_differences():
    rng = np.random.default_rng(5)
    levels = (2, 3, 4, 5)
    p = N.unet_init(rng, c_in=2, c_out=2, levels=levels)
    x = rng.standard_normal((2, 8, 8, 8))
    gout = rng.standard_normal((2, 8, 8, 8))
    out, cache = N.unet_forward(p, x, levels)
    g = N.unet_backward(p, cache, gout, levels)
    assert set(g) == set(p)
    names = sorted(p)

    def f(*vals):
        q = dict(zip(names, vals))
        return float((gout * N.unet_forward(q, x, levels)[0]).sum())

    # eps 1e-6: truncation error ~eps^2, roundoff ~1e-16 |f| / eps; small enough that no
    # ReLU input crosses zero along the probe
    _fd_check(f, [p[k] for k in names], [g[k] for k in names], rng, eps=1e-6, rel=1e-4)
