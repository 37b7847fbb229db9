"""Pins of the oracle's mass-transport solve on the paper's D3Q19 lattice (Section 3.2,
Eq. 10; boundaries of Section 3.3).

* On a box that is fluid everywhere, with tau_g varying only along x, the state stays
  uniform in y and z and the 19 populations collapse, by the sign of e_x, into a
  one-dimensional three-velocity lattice with weights 2/3 (rest), 1/6, 1/6.  That 1D
  lattice is iterated here with numpy, from its definition, and must give the same
  concentration profile and outlet flux.
* The steady straight channel: D_eff = c_s^2 (tau - 1/2) (nx + 1)/(nx - 1 + 2 tau) with
  c_s^2 = 1/3, tortuosity exactly 1 at tau = 1.
* A staircase of voxels that touch only along edges carries flux on D3Q19 and none on
  D3Q7 (the paper's reason for D3Q19: reduced lattices cut the void space's
  connectivity).
* Collision conserves C and keeps the equilibrium; swapping and rescaling C_in, C_out;
  mirror symmetry; one node's update from its neighbourhood equals the solve's.
"""
import numpy as np
import pytest

from paper_1410_1921_amd import workloads as W

E19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1],
                [1, 0, -1], [-1, 0, -1], [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]])
A19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def d1q3(tau_x, c_in, c_out, steps):
    """The 1D lattice: rest weight 2/3, +-x weights 1/6, BGK with tau per x, ghost
    nodes at x = -1 and x = nx holding the equilibrium of C_in and C_out.  Returns the
    concentration after the last collision and the outlet flux of that state."""
    nx = len(tau_x)
    w = np.array([2 / 3, 1 / 6, 1 / 6])
    g = np.zeros((nx, 3))
    for _ in range(steps):
        gin = np.empty_like(g)
        gin[:, 0] = g[:, 0]
        gin[1:, 1] = g[:-1, 1]
        gin[0, 1] = w[1] * c_in
        gin[:-1, 2] = g[1:, 2]
        gin[-1, 2] = w[2] * c_out
        c = gin.sum(axis=1)
        g = gin - (gin - w[None, :] * c[:, None]) / tau_x[:, None]
    return c, g[-1, 1] - w[2] * c_out


def test_all_fluid_reduces_to_one_dimension(orc):
    nz, ny, nx = 3, 4, 12
    m = np.ones((nz, ny, nx), np.uint8)
    tau_x = 0.6 + 0.05 * np.arange(nx)
    tg = np.broadcast_to(tau_x[None, None, :], m.shape)
    steps = 700
    r = orc.diffusion19_solve(m, tg, 0.9, 0.2, fixed_steps=steps, check_every=100)
    c1, flux1 = d1q3(tau_x, 0.9, 0.2, steps)
    assert np.allclose(r["c"], c1[None, None, :], rtol=0, atol=1e-13)
    assert r["phi_out"] == pytest.approx(flux1 * ny * nz, rel=1e-11)


@pytest.mark.parametrize("tau", [0.7, 1.0, 1.6])
def test_straight_channel_closed_form(orc, tau):
    nx = 14
    m = np.ones((2, 3, nx), np.uint8)
    r = orc.diffusion19_solve(m, tau, 1.0, 0.0, max_steps=400_000, check_every=100, tol=1e-14)
    assert r["converged"]
    want = (tau - 0.5) / 3 * (nx + 1) / (nx - 1 + 2 * tau)
    assert r["Deff_lattice"] == pytest.approx(want, rel=1e-9)
    if tau == 1.0:  # tortuosity eps D_ref / D_eff = 1
        assert 1.0 * (tau - 0.5) / 3 / r["Deff_lattice"] == pytest.approx(1.0, rel=1e-9)
    # every link plane carries the same flux at steady state
    assert np.allclose(r["plane_flux"], r["plane_flux"][0], rtol=1e-9)


def test_edge_connected_staircase(orc):
    nx, ny, nz = 10, 10, 1
    m = np.zeros((nz, ny, nx), np.uint8)
    for x in range(nx):
        m[0, x % ny, x] = 1  # voxel (x, x): consecutive voxels share an edge only
    kw = dict(max_steps=200_000, check_every=100, tol=1e-13)
    r19 = orc.diffusion19_solve(m, 1.0, 1.0, 0.0, **kw)
    r7 = orc.knudsen_solve(m, 1.0, 1.0, 0.0, **kw)
    assert r19["converged"] and r7["converged"]
    assert r19["Deff_lattice"] > 1e-3
    assert abs(r7["Deff_lattice"]) < 1e-12


def test_collision(orc):
    rng = np.random.default_rng(5)
    for _ in range(4):
        gin = A19 * (0.3 + rng.random(19))
        gout, c = orc.collide19_diff(gin, 0.83)
        assert c == pytest.approx(gin.sum(), rel=1e-15)
        assert gout.sum() == pytest.approx(gin.sum(), rel=1e-14)
        geq, _ = orc.collide19_diff(A19 * 0.7, 0.83)
        assert np.allclose(geq, A19 * 0.7, rtol=0, atol=2e-16)


def test_swap_and_linearity(orc):
    # the steady problem is linear in (C_in, C_out): 1 - C solves the swapped one, and
    # a + b C the rescaled one (from a zero start the transients are not)
    m = W.blob_mask((6, 9, 11), 0.6, 3)
    tg = np.where(m == 1, 0.6 + W.hash_field(m.shape, 2, 0.0, 0.8), 1.0)
    kw = dict(max_steps=400_000, check_every=100, tol=1e-14)
    a = orc.diffusion19_solve(m, tg, 1.0, 0.0, **kw)
    b = orc.diffusion19_solve(m, tg, 0.0, 1.0, **kw)
    c = orc.diffusion19_solve(m, tg, 0.7, 0.3, **kw)  # 0.3 + 0.4 * (first)
    assert b["phi_out"] == pytest.approx(-a["phi_out"], rel=1e-8)
    assert c["phi_out"] == pytest.approx(0.4 * a["phi_out"], rel=1e-8)
    assert c["Deff_lattice"] == pytest.approx(a["Deff_lattice"], rel=1e-8)
    assert a["converged"] and b["converged"] and c["converged"]
    assert np.allclose(b["c"], (1.0 - a["c"]) * m, rtol=0, atol=1e-10)
    assert np.allclose(c["c"], (0.3 + 0.4 * a["c"]) * m, rtol=0, atol=1e-10)


def test_mirror_symmetry(orc):
    m = W.blob_mask((5, 8, 9), 0.6, 7)
    tg = np.where(m == 1, 0.6 + W.hash_field(m.shape, 4, 0.0, 0.8), 1.0)
    kw = dict(fixed_steps=300, check_every=100)
    a = orc.diffusion19_solve(m, tg, 1.0, 0.0, **kw)
    b = orc.diffusion19_solve(m[:, ::-1, :].copy(), tg[:, ::-1, :].copy(), 1.0, 0.0, **kw)
    c = orc.diffusion19_solve(m[::-1, :, :].copy(), tg[::-1, :, :].copy(), 1.0, 0.0, **kw)
    assert np.allclose(b["c"], a["c"][:, ::-1, :], rtol=0, atol=1e-13)
    assert np.allclose(c["c"], a["c"][::-1, :, :], rtol=0, atol=1e-13)
    assert b["Deff_lattice"] == pytest.approx(a["Deff_lattice"], rel=1e-12)


def test_single_node_update_matches_solve(orc):
    m = W.blob_mask((4, 5, 6), 0.7, 9)
    nz, ny, nx = m.shape
    rng = np.random.default_rng(1)
    c0 = rng.random(m.shape)
    g0 = orc.diffusion19_init(m, c0)
    g0 = g0 + 1e-3 * rng.standard_normal(g0.shape) * m[..., None]
    tau = 0.9
    r = orc.diffusion19_solve(m, tau, 0.8, 0.1, fixed_steps=1, g=g0.copy(), want_planes=False)
    for z, y, x in [(0, 0, 0), (1, 2, 5), (3, 4, 2), (2, 1, 3)]:
        if not m[z, y, x]:
            continue
        kind = np.zeros(19, np.uint8)
        nb = np.zeros((19, 19))
        for i, e in enumerate(E19):
            sx, sy, sz = x - e[0], (y - e[1]) % ny, (z - e[2]) % nz
            if sx < 0:
                kind[i] = 2
            elif sx >= nx:
                kind[i] = 3
            elif not m[sz, sy, sx]:
                kind[i] = 1
            else:
                nb[i] = g0[sz, sy, sx]
        nb[0] = g0[z, y, x]
        # bounce-back reads the node's own opposite population from row 0
        gout, _ = orc.diffusion19_update_node(kind, nb, tau, 0.8, 0.1)
        assert np.allclose(gout, r["g"][z, y, x], rtol=0, atol=1e-15)
