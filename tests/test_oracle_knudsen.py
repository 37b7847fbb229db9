"""Pins of the oracle's D3Q7 Knudsen solve (Section 3.2, Eqs. 10-12; boundaries,
Section 3.3; Eq. 14) against closed forms and invariants.

Straight channel.  With C depending on x only, the steady BGK solution between the two
equilibrium ghost planes is linear in the interior with slope dC/(n_x - 1 + 2 tau) and
carries the lattice diffusivity c_s^2 (tau - 1/2) (c_s^2 = 1/4 on D3Q7 with rest weight
1/4): per fluid column the flux is c_s^2 (tau - 1/2) dC / (n_x - 1 + 2 tau).  With the
ghost-plane distance n_x + 1 in Eq. 14 this gives D_eff = eps c_s^2 (tau - 1/2)
(n_x + 1)/(n_x - 1 + 2 tau), so at tau = 1 the tortuosity eps D / D_eff is exactly 1.
"""
import numpy as np
import pytest

from paper_1410_1921_amd import workloads as W


def _duct(nx, side=2, pad=1):
    return W.square_duct(nx, side, pad)


@pytest.mark.parametrize("tau", [0.55, 0.6, 1.0, 1.5])
def test_straight_duct_exact(orc, tau):
    nx = 10
    m = _duct(nx)
    r = orc.knudsen_solve(m, tau, 1.0, 0.0, max_steps=2_000_000, tol=1e-14)
    eps = m.mean()
    cs2 = 0.25
    want = eps * cs2 * (tau - 0.5) * (nx + 1) / (nx - 1 + 2 * tau)
    assert r["converged"]
    assert r["Deff_lattice"] == pytest.approx(want, rel=1e-9)
    # every link plane carries the same flux at steady state
    pf = r["plane_flux"]
    assert np.allclose(pf, pf[0], rtol=1e-9)
    assert r["phi_in"] == pytest.approx(r["phi_out"], rel=1e-9)


def test_tortuosity_one_at_tau_one(orc):
    nx = 13
    m = W.slit(nx, 8, 3, 4, axis=1)
    r = orc.knudsen_solve(m, 1.0, 1.0, 0.0, max_steps=2_000_000, tol=1e-14)
    eps = m.mean()
    tort = eps * 0.25 * 0.5 / r["Deff_lattice"]
    assert tort == pytest.approx(1.0, rel=1e-9)


def test_parallel_columns(orc):
    # separated columns with different uniform tau add up their own closed forms
    nx = 9
    m = np.zeros((5, 5, nx), np.uint8)
    tg = np.full(m.shape, 0.8)
    cols = [((1, 1), 0.6), ((1, 3), 1.0), ((3, 1), 1.4), ((3, 3), 0.75)]
    want = 0.0
    for (z, y), t in cols:
        m[z, y, :] = 1
        tg[z, y, :] = t
        want += 0.25 * (t - 0.5) * (nx + 1) / (nx - 1 + 2 * t)
    want /= 25.0
    r = orc.knudsen_solve(m, tg, 1.0, 0.0, max_steps=3_000_000, tol=1e-14)
    assert r["Deff_lattice"] == pytest.approx(want, rel=1e-9)


def test_mass_conservation_closed_box(orc):
    # x faces solid: no link reaches a ghost plane, so sum(C) stays at its start value
    m = W.blob_mask((8, 9, 10), 0.6, 2)
    m[:, :, 0] = 0
    m[:, :, -1] = 0
    rng = np.random.default_rng(3)
    c0 = rng.random(m.shape) * m
    g = orc.knudsen_init(m, c0)
    tg = 0.55 + rng.random(m.shape)
    r = orc.knudsen_solve(m, tg, 1.0, 0.0, fixed_steps=300, g=g)
    assert r["sum_c"] == pytest.approx(c0.sum(), rel=1e-13)


def test_swap_and_linearity(orc):
    m = W.blob_mask((10, 10, 12), 0.6, 4)
    tg = 0.6 + 0.5 * W.random_mask(m.shape, 0.5, 9)
    a = orc.knudsen_solve(m, tg, 1.0, 0.0, fixed_steps=400)
    # C -> 1 - C maps the run onto the one with the faces swapped (from C = 1): the flux
    # reverses and D_eff stays
    g = orc.knudsen_init(m, 1.0 * m)
    b = orc.knudsen_solve(m, tg, 0.0, 1.0, fixed_steps=400, g=g)
    assert b["phi_out"] == pytest.approx(-a["phi_out"], rel=1e-10)
    assert b["Deff_lattice"] == pytest.approx(a["Deff_lattice"], rel=1e-10)
    # C -> 0.5 + 2 C: faces 2.5 / 0.5 from C = 0.5; flux doubles, D_eff stays
    g = orc.knudsen_init(m, 0.5 * m)
    c = orc.knudsen_solve(m, tg, 2.5, 0.5, fixed_steps=400, g=g)
    assert c["phi_out"] == pytest.approx(2 * a["phi_out"], rel=1e-10)
    assert c["Deff_lattice"] == pytest.approx(a["Deff_lattice"], rel=1e-10)


def test_single_node_update_matches_solve(orc):
    m = W.blob_mask((6, 7, 8), 0.6, 5)
    rng = np.random.default_rng(2)
    tg = 0.52 + rng.random(m.shape)
    g0 = orc.knudsen_init(m, rng.random(m.shape) * m)
    g = g0.copy()
    orc.knudsen_solve(m, tg, 0.9, 0.1, fixed_steps=1, g=g)
    e = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    nz, ny, nx = m.shape
    for z, y, x in np.argwhere(m == 1)[::3]:
        kind = np.zeros(7, np.uint8)
        nbg = np.zeros((7, 7))
        for i, (ex, ey, ez) in enumerate(e):
            sx = x - ex
            if sx < 0:
                kind[i] = 2
                continue
            if sx >= nx:
                kind[i] = 3
                continue
            s = ((z - ez) % nz, (y - ey) % ny, sx)
            kind[i] = 0 if m[s] else 1
            nbg[i] = g0[s]
        nbg[0] = g0[z, y, x]
        out, _ = orc.knudsen_update_node(kind, nbg, tg[z, y, x], 0.9, 0.1)
        assert np.array_equal(out, g[z, y, x])


def test_collision_conserves(orc):
    gin = np.array([0.3, 0.1, 0.05, 0.2, 0.12, 0.07, 0.16])
    gout, c = orc.collide7(gin, 0.77)
    assert c == pytest.approx(gin.sum(), abs=1e-16)
    assert gout.sum() == pytest.approx(gin.sum(), abs=1e-15)
    # at tau = 1 the output is the equilibrium w_i C
    gout, c = orc.collide7(gin, 1.0)
    w = np.array([0.25] + [0.125] * 6)
    assert np.allclose(gout, w * c, atol=1e-16)


def test_plane_mean_estimator(orc):
    # D_eff from the mean link-plane flux: equal to the outlet's at steady state, and
    # nearer to the steady value during the approach (the flux profile of each decaying
    # mode along x averages out over the planes)
    pore = W.square_duct(30, 3, pad=1)
    nx = pore.shape[2]
    tau = 1.0
    want = pore.mean() * 0.25 * (tau - 0.5) * (nx + 1) / (nx - 1 + 2 * tau)
    tg = np.where(pore == 1, tau, 1.0)
    early = orc.knudsen_solve(pore, tg, 1.0, 0.0, fixed_steps=300, want_c=False)
    assert abs(early["Deff_planes"] / want - 1) < 0.2 * abs(early["Deff_lattice"] / want - 1)
    done = orc.knudsen_solve(pore, tg, 1.0, 0.0, tol=1e-13, max_steps=200_000, want_c=False)
    assert done["Deff_planes"] == pytest.approx(want, rel=1e-9)
    assert done["Deff_lattice"] == pytest.approx(want, rel=1e-9)
