"""Pins of the oracle's D3Q19 flow solve (Section 3.1, Eqs. 1-3, 8-9; half-way
bounce-back, Section 3.3; Darcy, Eq. 13) against closed forms and invariants.

Discrete plane Poiseuille.  For BGK with half-way bounce-back and a body force F, the
steady profile across a slit of H fluid nodes (wall half a link beyond the last node)
is the parabola u(y) = F/(2 nu) (H^2/4 - y^2) plus a wall slip F (16 L - 3)/(24 nu),
where L = (tau - 1/2)^2 (the slip vanishes at the well-known L = 3/16).  The node mean
then gives the permeability per fluid node (H^2 + 8 L - 1)/12; over the whole box of
n_y rows (superficial velocity) it is scaled by H/n_y.
"""
import math

import numpy as np
import pytest

from paper_1410_1921_amd import workloads as W

TAU_MAGIC = 0.5 + math.sqrt(3.0 / 16.0)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0])
@pytest.mark.parametrize("h", [6, 9])
def test_slit_exact(orc, tau, h):
    m = W.slit(2, h + 2, 2, h, axis=1)
    r = orc.flow_solve(m, tau=tau, force=(1e-6, 0, 0), max_steps=200_000, check_every=100,
                       tol=1e-13, want_u=False)
    lam = (tau - 0.5) ** 2
    k = h / (h + 2) * (h * h + 8 * lam - 1) / 12
    assert r["converged"]
    assert r["k_lattice"] == pytest.approx(k, rel=1e-8)


def test_slit_along_z_walls(orc):
    # walls normal to z, force along x: the same closed form
    h, tau = 7, 0.8
    m = W.slit(2, 2, h + 2, h, axis=2)
    r = orc.flow_solve(m, tau=tau, force=(1e-6, 0, 0), max_steps=200_000, tol=1e-13, want_u=False)
    lam = (tau - 0.5) ** 2
    assert r["k_lattice"] == pytest.approx(h / (h + 2) * (h * h + 8 * lam - 1) / 12, rel=1e-8)


def _duct_series(a):
    """Mean-velocity permeability of a square duct of side a (Boussinesq series):
    k = a^2/12 * (1 - 192/pi^5 * sum_{n odd} tanh(n pi / 2) / n^5)."""
    s = sum(math.tanh(n * math.pi / 2) / n ** 5 for n in range(1, 200, 2))
    return a * a / 12 * (1 - 192 / math.pi ** 5 * s)


def test_square_duct_series(orc):
    # at L = 3/16 the bounce-back wall sits half a link out; the corner error falls as
    # 1/a^2 (about 2.4 % at a = 6, 0.65 % at a = 12)
    errs = []
    for a in (6, 12):
        m = W.square_duct(2, a)
        r = orc.flow_solve(m, tau=TAU_MAGIC, force=(1e-6, 0, 0), max_steps=400_000, tol=1e-12,
                           want_u=False)
        k_int = r["k_lattice"] * m.size / m.sum()
        errs.append(abs(k_int / _duct_series(a) - 1))
    assert errs[1] < errs[0] / 3.5
    assert errs[1] < 8e-3


def test_tube_eq27(orc):
    # Eq. 27: k = (d/2)^2 / 8 for a tube; the staircase wall converges with the radius
    errs = []
    for rad in (4.5, 9.5):
        m = W.tube(2, rad)
        r = orc.flow_solve(m, tau=TAU_MAGIC, force=(1e-6, 0, 0), max_steps=400_000, tol=1e-11,
                           want_u=False)
        k_int = r["k_lattice"] * m.size / m.sum()
        # compare against the tube of equal area, the natural radius of a voxelised disk
        r_eq = math.sqrt(m[:, :, 0].sum() / math.pi)
        errs.append(abs(k_int / (r_eq ** 2 / 8) - 1))
    assert errs[1] < errs[0]
    assert errs[1] < 0.03


def test_momentum_balance_no_solid(orc):
    # all fluid, periodic: each step adds F per node, so <rho u> = F (t - 1/2) at step t
    m = np.ones((4, 5, 6), np.uint8)
    F = (2e-6, -1e-6, 5e-7)
    for t in (1, 7, 40):
        r = orc.flow_solve(m, tau=0.7, force=F, fixed_steps=t, want_u=False)
        assert np.allclose(r["mean_rho_u"], np.array(F) * (t - 0.5), rtol=1e-10, atol=0)


def test_mass_conservation(orc):
    m = W.blob_mask((12, 12, 12), 0.5, 3)
    r = orc.flow_solve(m, tau=0.8, force=(1e-4, 0, 0), fixed_steps=500, want_u=False)
    assert abs(r["mass_dev"]) < 1e-11 * m.sum()


def test_mirror_symmetry(orc):
    m = W.blob_mask((10, 11, 12), 0.55, 5)
    base = orc.flow_solve(m, fixed_steps=300, want_u=False)["k_lattice"]
    ky = orc.flow_solve(np.ascontiguousarray(m[:, ::-1, :]), fixed_steps=300, want_u=False)
    kz = orc.flow_solve(np.ascontiguousarray(m[::-1, :, :]), fixed_steps=300, want_u=False)
    # mirrored along x with the force reversed: the same permeability
    kx = orc.flow_solve(np.ascontiguousarray(m[:, :, ::-1]), force=(-1e-6, 0, 0), fixed_steps=300,
                        want_u=False)
    for r in (ky, kz, kx):
        assert r["k_lattice"] == pytest.approx(base, rel=1e-10)


def test_stokes_linearity(orc):
    m = W.blob_mask((10, 10, 10), 0.6, 8)
    k1 = orc.flow_solve(m, force=(1e-6, 0, 0), fixed_steps=400, want_u=False)["k_lattice"]
    k2 = orc.flow_solve(m, force=(2e-6, 0, 0), fixed_steps=400, want_u=False)["k_lattice"]
    assert k2 == pytest.approx(k1, rel=1e-5)


def test_single_node_update_matches_solve(orc):
    # one step of the solve equals the node update fed with each node's neighbourhood
    m = W.blob_mask((6, 7, 8), 0.6, 2)
    rng = np.random.default_rng(1)
    f0 = orc.flow_init(m) + 1e-3 * rng.standard_normal(m.shape + (19,)) * m[..., None]
    f = f0.copy()
    orc.flow_solve(m, tau=0.9, force=(1e-5, 2e-6, 0), fixed_steps=1, f=f, want_u=False)
    e = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
         (1, 1, 0), (-1, 1, 0), (1, -1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, 1), (1, 0, -1),
         (-1, 0, -1), (0, 1, 1), (0, -1, 1), (0, 1, -1), (0, -1, -1)]
    nz, ny, nx = m.shape
    for z, y, x in np.argwhere(m == 1)[::5]:
        nbf = np.zeros((19, 19))
        nbm = np.zeros(19, np.uint8)
        for i, (ex, ey, ez) in enumerate(e):
            s = ((z - ez) % nz, (y - ey) % ny, (x - ex) % nx)
            nbm[i] = m[s]
            nbf[i] = f0[s]
        out, _ = orc.flow_update_node(nbm, nbf, 0.9, (1e-5, 2e-6, 0))
        assert np.array_equal(out, f[z, y, x])


def test_collision_invariants(orc):
    rng = np.random.default_rng(4)
    fin = 1 / 19 + 1e-3 * rng.standard_normal(19)
    F = np.array([3e-5, -1e-5, 2e-5])
    fout, mom = orc.collide19(fin, 0.73, F)
    e = np.array([(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                  (1, 1, 0), (-1, 1, 0), (1, -1, 0), (-1, -1, 0), (1, 0, 1), (-1, 0, 1),
                  (1, 0, -1), (-1, 0, -1), (0, 1, 1), (0, -1, 1), (0, 1, -1), (0, -1, -1)])
    # mass conserved; momentum gains exactly F
    assert fout.sum() == pytest.approx(fin.sum(), abs=1e-15)
    assert np.allclose(fout @ e, fin @ e + F, rtol=0, atol=1e-16)
    assert mom[0] == pytest.approx(fin.sum(), abs=1e-15)
    assert np.allclose(mom[1:], fin @ e + F / 2, rtol=0, atol=1e-16)


def test_init_equilibrium_moments(orc):
    # the D3Q19 equilibrium (Eq. 3) has density rho, momentum rho u and momentum flux
    # rho (I/3 + u u) exactly; the initial state must carry those moments at every node
    rng = np.random.default_rng(5)
    m = W.blob_mask((6, 7, 8), 0.6, 2)
    u = 0.05 * rng.standard_normal((3,) + m.shape)
    dr = 0.02 * rng.standard_normal(m.shape)
    f = orc.flow_init(m, u, dr)
    e = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                  [1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1],
                  [1, 0, -1], [-1, 0, -1], [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]], float)
    fl = m.astype(bool)
    rho = f.sum(-1)
    j = np.einsum("zyxi,ia->azyx", f, e)
    pi = np.einsum("zyxi,ia,ib->abzyx", f, e, e)
    r_ref = 1.0 + dr
    assert np.allclose(rho[fl], r_ref[fl], rtol=0, atol=1e-14)
    assert np.allclose(j[:, fl], (r_ref * u)[:, fl], rtol=0, atol=1e-14)
    want = r_ref * (np.eye(3)[:, :, None, None, None] / 3 + u[:, None] * u[None, :])
    assert np.allclose(pi[:, :, fl], want[:, :, fl], rtol=0, atol=1e-14)
    assert (f[~fl] == 0).all()
