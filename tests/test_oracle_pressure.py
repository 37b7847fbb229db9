"""Pins of the oracle's pressure boundaries (Section 3.3: Guo's non-equilibrium
extrapolation at x = -1 and x = nx, periodic in y and z).

* A slit driven by a small density difference gives the closed-form slit permeability of
  the body-force drive, the pressure drop taken over the nx + 1 spacings between the
  ghost planes: (H/n_y)(H^2 + 8 (tau - 1/2)^2 - 1)/12 for BGK, (H/n_y)(H^2 + 1/2)/12 for
  the MRT of Eq. 7 (and its TRT form) at any tau.
* No density difference, no flow.
* At steady state the discrete mass flux through every link plane (populations crossing
  x + 1/2 between fluid nodes) is the same.
* Mirror symmetry in y and z.
"""
import numpy as np
import pytest

from paper_1410_1921_amd import workloads as W

E19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0], [1, 0, 1], [-1, 0, 1],
                [1, 0, -1], [-1, 0, -1], [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]])
DRHO = 2e-5


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.4])
def test_slit_bgk(orc, tau):
    h = 6
    m = W.slit(12, h + 2, 2, h, axis=1)
    r = orc.flow_solve(m, tau=tau, force=(0, 0, 0), pressure=(1 + DRHO / 2, 1 - DRHO / 2),
                       max_steps=400_000, check_every=100, tol=1e-13, want_u=False)
    assert r["converged"]
    k = h / (h + 2) * (h * h + 8 * (tau - 0.5) ** 2 - 1) / 12
    assert r["k_lattice"] == pytest.approx(k, rel=2e-5)


@pytest.mark.parametrize("collision", ["MRT", "TRT"])
@pytest.mark.parametrize("tau", [0.6, 1.2])
def test_slit_mrt_viscosity_independent(orc, collision, tau):
    h = 6
    m = W.slit(10, h + 2, 2, h, axis=1)
    r = orc.flow_solve(m, tau=tau, force=(0, 0, 0), pressure=(1 + DRHO / 2, 1 - DRHO / 2),
                       max_steps=400_000, check_every=100, tol=1e-13, want_u=False,
                       collision=getattr(orc, collision))
    assert r["converged"]
    assert r["k_lattice"] == pytest.approx(h / (h + 2) * (h * h + 0.5) / 12, rel=2e-5)


def test_no_difference_no_flow(orc):
    m = W.blob_mask((6, 7, 9), 0.6, 4)
    r = orc.flow_solve(m, force=(0, 0, 0), pressure=(1.0, 1.0), fixed_steps=300, check_every=100)
    assert np.abs(r["u"]).max() < 1e-14  # rounding of the weights only


def link_plane_fluxes(m, f):
    """Mass crossing each plane x + 1/2 (x = 0..nx-2) per step: populations with e_x = +1
    leaving fluid (x, y, z) for fluid (x+1, .), less those with e_x = -1 leaving fluid
    (x+1, y, z) for fluid (x, .)."""
    nz, ny, nx = m.shape
    out = np.zeros(nx - 1)
    for x in range(nx - 1):
        s = 0.0
        for i, e in enumerate(E19):
            if e[0] == 0:
                continue
            src = x if e[0] == 1 else x + 1
            dst = src + e[0]
            for z in range(nz):
                for y in range(ny):
                    ty, tz = (y + e[1]) % ny, (z + e[2]) % nz
                    if m[z, y, src] and m[tz, ty, dst]:
                        s += e[0] * f[z, y, src, i]
        out[x] = s
    return out


def test_steady_flux_through_every_plane(orc):
    m = W.blob_mask((5, 8, 10), 0.65, 6)
    r = orc.flow_solve(m, tau=0.9, force=(0, 0, 0), pressure=(1 + DRHO / 2, 1 - DRHO / 2),
                       max_steps=400_000, check_every=100, tol=1e-11, want_u=False)
    assert r["converged"]
    phi = link_plane_fluxes(m, r["f"])
    assert abs(phi.mean()) > 1e-9
    assert np.allclose(phi, phi.mean(), rtol=1e-7, atol=0)


def test_mirror_symmetry(orc):
    m = W.blob_mask((6, 8, 9), 0.6, 2)
    kw = dict(tau=0.8, force=(0, 0, 0), pressure=(1 + DRHO, 1.0), fixed_steps=400,
              check_every=100)
    a = orc.flow_solve(m, **kw)
    b = orc.flow_solve(m[:, ::-1, :].copy(), **kw)
    c = orc.flow_solve(m[::-1, :, :].copy(), **kw)
    assert np.allclose(b["u"][0], a["u"][0][:, ::-1, :], rtol=0, atol=1e-14)  # rounding at the population scale
    assert np.allclose(b["u"][1], -a["u"][1][:, ::-1, :], rtol=0, atol=1e-14)  # rounding at the population scale
    assert np.allclose(c["u"][2], -a["u"][2][::-1, :, :], rtol=0, atol=1e-14)  # rounding at the population scale
    assert b["k_lattice"] == pytest.approx(a["k_lattice"], rel=1e-12)
