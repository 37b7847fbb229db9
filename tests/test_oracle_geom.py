"""Pins of the oracle's characterisation (Section 4.1): 18-neighbour labelling against
scipy.ndimage.label and hand cases; 13-direction chords against closed values and an
explicit walk; squared EDT against scipy.ndimage and O(N^6) brute force; the
maximum-inscribed-sphere map against slit widths and brute force."""
import itertools
import math

import numpy as np
import pytest
from scipy import ndimage

from paper_1410_1921_amd import workloads as W

S2, S3 = math.sqrt(2.0), math.sqrt(3.0)


def _same_partition(lab_a, lab_b, mask):
    a = lab_a[mask.astype(bool)]
    b = lab_b[mask.astype(bool)]
    pairs = set(zip(a.tolist(), b.tolist()))
    return len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


@pytest.mark.parametrize("seed,p", [(1, 0.3), (2, 0.45), (3, 0.6)])
def test_label18_matches_scipy(orc, seed, p):
    m = W.random_mask((14, 13, 15), p, seed)
    # solid y and z faces: periodic wrap cannot join anything, so scipy's open
    # labelling with the 18-neighbour structure is the reference
    m[0], m[-1], m[:, 0], m[:, -1] = 0, 0, 0, 0
    lab, tr, info = orc.label18(m)
    ref, nref = ndimage.label(m, structure=ndimage.generate_binary_structure(3, 2))
    assert _same_partition(lab, ref, m)
    assert info["n_components"] == nref
    # canonical labels: the smallest linear index of each component
    flat = np.arange(m.size).reshape(m.shape)
    for k in range(1, nref + 1):
        sel = ref == k
        assert (lab[sel] == flat[sel].min()).all()
    assert (lab[m == 0] == -1).all()
    # transport components touch x = 0 and x = nx-1
    for k in range(1, nref + 1):
        sel = ref == k
        both = sel[:, :, 0].any() and sel[:, :, -1].any()
        assert (tr[sel] == int(both)).all()
    assert info["n_transport"] == int(tr.sum())
    assert info["n_pore"] == int(m.sum())


def test_label18_neighbourhood_and_wrap(orc):
    m = np.zeros((6, 6, 6), np.uint8)
    m[2, 2, 2] = m[2, 3, 3] = 1            # edge neighbours (dy, dx) = (1, 1): joined
    m[4, 4, 4] = m[5, 5, 5] = 1            # corner only: separate
    lab, _, info = orc.label18(m)
    assert lab[2, 2, 2] == lab[2, 3, 3]
    assert lab[4, 4, 4] != lab[5, 5, 5]
    assert info["n_components"] == 3
    # periodic in y: voxels at y = 0 and y = ny-1 are neighbours
    m = np.zeros((6, 6, 6), np.uint8)
    m[3, 0, 3] = m[3, 5, 3] = 1
    lab, _, info = orc.label18(m)
    assert info["n_components"] == 1
    # periodic in z, with an edge step in y
    m = np.zeros((6, 6, 6), np.uint8)
    m[0, 2, 3] = m[5, 3, 3] = 1
    assert orc.label18(m)[2]["n_components"] == 1
    # open in x: x = 0 and x = nx-1 are not neighbours
    m = np.zeros((6, 6, 6), np.uint8)
    m[3, 3, 0] = m[3, 3, 5] = 1
    assert orc.label18(m)[2]["n_components"] == 2


def test_label18_transport_channel(orc):
    m = np.zeros((8, 8, 10), np.uint8)
    m[3, 3, :] = 1                          # straight channel along x: transport
    m[6, 6, 2:5] = 1                        # short dead bar
    lab, tr, info = orc.label18(m)
    assert tr[3, 3, :].all() and not tr[6, 6, 2:5].any()
    assert info["n_transport"] == 10 and info["n_pore"] == 13


def _walk_chords(m):
    """Explicit chord walk per voxel and per direction (tiny masks only)."""
    nz, ny, nx = m.shape
    dirs = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1),
            (0, 1, 1), (0, 1, -1), (1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1)]
    out = np.zeros(m.shape)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        if not m[z, y, x]:
            continue
        tot = 0.0
        for d in dirs:
            cnt = 1
            for sgn in (1, -1):
                xx, yy, zz = x, y, z
                while True:
                    xx += sgn * d[0]; yy += sgn * d[1]; zz += sgn * d[2]
                    if not (0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz) or not m[zz, yy, xx]:
                        break
                    cnt += 1
            tot += cnt * math.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
        out[z, y, x] = tot / 13.0
    return out


def test_chords13_closed_values(orc):
    # an isolated pore voxel: every chord is one voxel long
    m = np.zeros((5, 5, 5), np.uint8)
    m[2, 2, 2] = 1
    d = orc.chords13(m)
    assert d[2, 2, 2] == pytest.approx((3 + 6 * S2 + 4 * S3) / 13, rel=1e-15)
    assert d.sum() == d[2, 2, 2]
    # a bar of L voxels along x: the x chord is L, the other 12 are 1
    m = np.zeros((5, 5, 9), np.uint8)
    m[2, 2, 1:8] = 1
    d, cnt = orc.chords13(m, want_counts=True)
    assert (d[2, 2, 1:8] == pytest.approx((7 + 2 + 6 * S2 + 4 * S3) / 13, rel=1e-15))
    assert (cnt[2, 2, 1:8] == [9, 6, 4]).all()
    # an all-pore cube n^3: the centre voxel has axis chords n, face chords n, body chords n
    n = 7
    m = np.ones((n, n, n), np.uint8)
    d, cnt = orc.chords13(m, want_counts=True)
    assert list(cnt[3, 3, 3]) == [3 * n, 6 * n, 4 * n]
    assert d[3, 3, 3] == pytest.approx(n * (3 + 6 * S2 + 4 * S3) / 13, rel=1e-15)
    # the corner voxel: axes n, face diagonals n (2 in the corner's planes) or 1, body 1 or n
    assert list(cnt[0, 0, 0]) == [3 * n, 3 * n + 3, n + 3]


@pytest.mark.parametrize("seed", [1, 2])
def test_chords13_explicit_walk(orc, seed):
    m = W.random_mask((5, 6, 7), 0.6, seed)
    assert np.allclose(orc.chords13(m), _walk_chords(m), rtol=1e-14, atol=0)


@pytest.mark.parametrize("seed,p", [(1, 0.7), (2, 0.9), (3, 0.5)])
def test_edt2_matches_scipy(orc, seed, p):
    m = W.random_mask((17, 19, 23), p, seed)
    e2 = orc.edt2(m)
    ref = ndimage.distance_transform_edt(m)
    assert np.array_equal(e2, np.rint(ref ** 2).astype(np.int64))


def test_edt2_brute_force(orc):
    m = W.random_mask((6, 7, 5), 0.75, 4)
    e2 = orc.edt2(m)
    pts = np.argwhere(m == 0)
    for z, y, x in itertools.product(range(6), range(7), range(5)):
        best = ((pts - [z, y, x]) ** 2).sum(1).min()
        assert e2[z, y, x] == best


def test_edt2_no_solid(orc):
    with pytest.raises(orc.OracleError):
        orc.edt2(np.ones((4, 4, 4), np.uint8))


@pytest.mark.parametrize("h", [1, 3, 4, 5, 8, 9])
def test_mis_slit_width(orc, h):
    m = W.slit(12, h + 6, 10, h, axis=1)
    d = orc.mis(m)
    want = h if h % 2 == 1 else h - 1
    assert (d[m == 1] == want).all()
    assert (d[m == 0] == 0).all()


def test_mis_brute_force(orc):
    m = W.blob_mask((9, 10, 11), 0.55, 7)
    e2 = orc.edt2(m)
    d = orc.mis(m, e2)
    pore = np.argwhere(m == 1)
    for z, y, x in pore:
        dd = ((pore - [z, y, x]) ** 2).sum(1)
        cand = e2[pore[:, 0], pore[:, 1], pore[:, 2]]
        best = cand[dd < cand].max()
        assert d[z, y, x] == 2.0 * math.sqrt(best) - 1.0


def test_mis_ball(orc):
    # a voxelised ball (centre distance^2 < 25) in an otherwise solid box: the nearest
    # solid voxel centre to the ball's centre is 5 away, so its width is 2*5 - 1
    n = 15
    c = n // 2
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    m = (((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2) < 25).astype(np.uint8)
    e2 = orc.edt2(m)
    d = orc.mis(m, e2)
    assert e2[c, c, c] == 25
    assert d[c, c, c] == 9.0
    assert d[m == 1].max() == 9.0 and d[m == 1].min() >= 1.0
    # every voxel of the ball lies within the centre's open ball, so all get width 9
    assert (d[m == 1] == 9.0).all()
