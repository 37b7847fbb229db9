"""Pins of the oracle's reconstruction step (Section 2, Steps 1-3) against the published
SplitMix64 outputs, closed forms of the lens volume, Monte-Carlo, and brute-force
re-checks of every acceptance rule."""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_hex(name):
    vals = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            vals.append(int(line, 16))
    return vals


def test_splitmix64_published_outputs(orc):
    ref = _golden_hex("splitmix64_seed0.txt")
    assert orc.splitmix64(0, len(ref)) == ref


def test_uniform_and_normal_draws(orc):
    u = orc.uniforms(7, 20000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / len(u))
    z = orc.normals(11, 20000)
    assert abs(z.mean()) < 4 / math.sqrt(len(z))
    assert abs(z.var() - 1.0) < 4 * math.sqrt(2 / len(z))
    # the polar method's normals: tail fractions of N(0,1)
    assert abs((np.abs(z) > 1.96).mean() - 0.05) < 0.01


def test_lens_volume_closed_forms(orc):
    r = 3.0
    # disjoint and tangent spheres share nothing
    assert orc.lens_volume(r, 2.0, 5.0) == 0.0
    assert orc.lens_volume(r, 2.0, 7.0) == 0.0
    # containment: the smaller sphere
    assert orc.lens_volume(4.0, 1.5, 1.0) == pytest.approx(4 / 3 * math.pi * 1.5 ** 3, rel=1e-15)
    assert orc.lens_volume(2.0, 2.0, 0.0) == pytest.approx(4 / 3 * math.pi * 8, rel=1e-15)
    # equal spheres: V = pi (4r + s)(2r - s)^2 / 12 (textbook two-cap form)
    for s in (0.5, 2.0, 4.5, 5.9):
        ref = math.pi * (4 * r + s) * (2 * r - s) ** 2 / 12
        assert orc.lens_volume(r, r, s) == pytest.approx(ref, rel=1e-13)
    # sum of two spherical caps of heights h1, h2 (cap volume pi h^2 (3 rho - h) / 3)
    r1, r2, s = 3.0, 2.0, 3.5
    a = (s * s + r1 * r1 - r2 * r2) / (2 * s)        # plane of the lens from centre 1
    h1, h2 = r1 - a, r2 - (s - a)
    caps = math.pi * h1 ** 2 * (3 * r1 - h1) / 3 + math.pi * h2 ** 2 * (3 * r2 - h2) / 3
    assert orc.lens_volume(r1, r2, s) == pytest.approx(caps, rel=1e-13)
    assert orc.sphere_volume(2.0) == pytest.approx(4 / 3 * math.pi * 8, rel=1e-15)


def test_lens_volume_monte_carlo(orc):
    rng = np.random.default_rng(5)
    for r1, r2, s in ((3.0, 2.5, 3.0), (1.0, 2.0, 2.2), (4.0, 4.0, 1.0)):
        lo = np.array([-r1, -r1, -r1])
        hi = np.array([r1, r1, r1])
        pts = rng.uniform(lo, hi, size=(400_000, 3))
        in1 = (pts ** 2).sum(1) <= r1 * r1
        in2 = ((pts - np.array([s, 0, 0])) ** 2).sum(1) <= r2 * r2
        frac = (in1 & in2).mean()
        est = frac * (2 * r1) ** 3
        sd = math.sqrt(frac * (1 - frac) / len(pts)) * (2 * r1) ** 3
        assert abs(orc.lens_volume(r1, r2, s) - est) < 5 * sd + 1e-9


def _voxelise(spheres, n):
    """Brute-force marking of the spheres (1/1024-voxel fixed point) on an n^3 grid."""
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = np.zeros((nz, ny, nx), bool)
    for cx, cy, cz, dq in spheres:
        ex = 1024 * x + 512 - cx
        ey = 1024 * y + 512 - cy
        ez = 1024 * z + 512 - cz
        m |= 4 * (ex * ex + ey * ey + ez * ez) <= dq * dq
    return m.astype(np.uint8)


@pytest.mark.parametrize("xi,p0,seed", [(0.5, 0.5, 1), (0.1, 0.9, 2), (0.0, 0.5, 3), (1.0, 0.5, 4)])
def test_reconstruction_rules(orc, xi, p0, seed):
    n = (24, 20, 16)
    eps = 0.3
    pore, sph, info = orc.reconstruct(n, eps, 6.0, 1.5, 1.0, xi, p0, seed)
    nvox = 24 * 20 * 16
    target = math.ceil(eps * nvox)
    # stop rule: target reached by the last sphere, not before it
    assert int(pore.sum()) == info["n_pore"] >= target
    assert int(_voxelise(sph[:-1], n).sum()) < target
    # voxelisation: exactly the union of the accepted spheres
    assert np.array_equal(_voxelise(sph, n), pore)
    # pairwise overlap tolerance against both spheres' volumes
    m = len(sph)
    c = sph[:, :3].astype(np.float64) / 1024.0
    r = sph[:, 3].astype(np.float64) / 2048.0
    assert (r >= 0.5).all()  # d >= d_min = 1 voxel
    for i in range(m):
        for j in range(i):
            s = float(np.sqrt(((c[i] - c[j]) ** 2).sum()))
            v = orc.lens_volume(r[i], r[j], s)
            vmin = orc.sphere_volume(min(r[i], r[j]))
            assert v <= xi * vmin * (1 + 1e-12)
            if xi == 0.0:
                assert s >= r[i] + r[j] - 1e-12


def test_forced_overlap(orc):
    # p0 = 1: every sphere after the first overlaps an earlier one
    _, sph, _ = orc.reconstruct((24, 24, 24), 0.2, 6.0, 1.5, 1.0, 0.4, 1.0, 9)
    c = sph[:, :3] / 1024.0
    r = sph[:, 3] / 2048.0
    for i in range(1, len(sph)):
        s = np.sqrt(((c[:i] - c[i]) ** 2).sum(1))
        assert (s < r[:i] + r[i]).any()


def test_determinism_and_seed(orc):
    a = orc.reconstruct(20, 0.3, 5.0, 1.0, seed=5)[0]
    b = orc.reconstruct(20, 0.3, 5.0, 1.0, seed=5)[0]
    c = orc.reconstruct(20, 0.3, 5.0, 1.0, seed=6)[0]
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_stall(orc):
    # non-overlapping spheres cannot fill 90% of the box
    with pytest.raises(orc.OracleError) as e:
        orc.reconstruct(16, 0.9, 6.0, 1.0, 1.0, 0.0, 0.0, 1, max_trials=5000)
    assert e.value.status == orc.E_STALL


def test_invalid(orc):
    with pytest.raises(orc.OracleError):
        orc.reconstruct(16, 1.2, 6.0, 1.0)
