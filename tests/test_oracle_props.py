"""Pins of the closed forms used for units and properties (Eqs. 11, 12, 15-17, 26-29;
Section 4.2)."""
import math
import os

import numpy as np
import pytest

from paper_1410_1921_amd import workloads as W

R_GAS = 8.314462618
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "props_worked_examples.txt")


def _worked_examples():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                name, *vals = line.split()
                rows.append((name, [float(v) for v in vals[:-1]], float(vals[-1])))
    return rows


@pytest.mark.parametrize("name,args,expected", _worked_examples())
def test_worked_examples(orc, name, args, expected):
    # values worked out by hand (arithmetic beside each line of the golden file)
    assert getattr(orc, name)(*args) == pytest.approx(expected, rel=1e-13)


def test_knudsen_diffusivity_printed_value(orc):
    # Section 4.2 prints D_K,ref = 1.31e-5 (m^2/s) for d = 60 nm, T = 323 K, methane
    dk = orc.knudsen_diffusivity(60e-9, 323.0, 0.016043)
    assert dk == pytest.approx(1.31e-5, rel=5e-3)
    # linear in d, sqrt in T
    assert orc.knudsen_diffusivity(30e-9, 323.0) == pytest.approx(dk / 2, rel=1e-14)
    assert orc.knudsen_diffusivity(60e-9, 4 * 323.0) == pytest.approx(2 * dk, rel=1e-14)


@pytest.mark.parametrize("d,T,mu,P", [(20e-9, 323.0, 1.73e-5, 17236893.0),
                                      (60e-9, 400.0, 1.2e-5, 1e6), (5e-9, 300.0, 1e-5, 3e5)])
def test_eq28_coefficient(orc, d, T, mu, P):
    # Eqs. 11, 26, 27, 29 combine into f_c = 1 + 64/(3 pi) Kn with Kn = lambda / radius
    Dk = orc.knudsen_diffusivity(d, T)
    k = (d / 2) ** 2 / 8
    fc = orc.fc_dgm(Dk, mu, k, P)
    lam = orc.mean_free_path(mu, P, T)
    assert fc - 1 == pytest.approx(64 / (3 * math.pi) * lam / (d / 2), rel=1e-12)
    assert 64 / (3 * math.pi) == pytest.approx(6.7906, abs=1e-4)


@pytest.mark.parametrize("d,eps", [(45e-9, 0.4), (10e-9, 0.1), (80e-9, 0.6)])
def test_kozeny_carman_from_hydraulic_radius(orc, d, eps):
    # Carman's form k = eps^3 / (K0 S0^2 (1 - eps)^2) with the Kozeny constant K0 = 5 and
    # S0 the surface per solid volume of the grains; for spheres of diameter d, S0 is the
    # derivative of the sphere volume over the volume, taken here numerically from the
    # oracle's own sphere volume (no 180 anywhere)
    r = d / 2
    h = r * 1e-5
    area = (orc.sphere_volume(r + h) - orc.sphere_volume(r - h)) / (2 * h)
    s0 = area / orc.sphere_volume(r)
    k_carman = eps ** 3 / (5.0 * s0 ** 2 * (1 - eps) ** 2)
    assert orc.k_kozeny_carman(d, eps) == pytest.approx(k_carman, rel=1e-8)


@pytest.mark.parametrize("eps,ratio", [(0.25, 0.01), (0.4, 0.05), (0.1, 0.003)])
def test_bruggeman_and_tortuosity_agree(orc, eps, ratio):
    # D_eff/D = eps^alpha and D_eff/D = eps/tau: eps^alpha gives the ratio back, and
    # tau = eps^(1 - alpha)
    a = orc.bruggeman_alpha(ratio, eps)
    assert eps ** a == pytest.approx(ratio, rel=1e-12)
    tau = orc.tortuosity(eps, 1.0, ratio)
    assert tau == pytest.approx(eps ** (1 - a), rel=1e-12)


@pytest.mark.parametrize("tau", [1.0, 1.4])
def test_straight_duct_tortuosity(orc, tau):
    # a straight square duct along x (bounce-back side walls) of uniform tau: the D3Q7
    # solve gives eps c_s^2 (tau - 1/2) (nx + 1)/(nx - 1 + 2 tau), so Eq. 16 gives
    # tortuosity (nx - 1 + 2 tau)/(nx + 1): exactly 1 at tau = 1
    pore = W.square_duct(12, 3, pad=1)
    nx = pore.shape[2]
    eps = pore.mean()
    r = orc.knudsen_solve(pore, np.where(pore == 1, tau, 1.0), 1.0, 0.0, tol=1e-13,
                          max_steps=200_000, want_c=False, want_planes=False)
    t = orc.tortuosity(eps, orc.lattice_diffusivity(0.25, tau), r["Deff_lattice"])
    assert t == pytest.approx((nx - 1 + 2 * tau) / (nx + 1), rel=1e-9)


def test_reference_pores_diffuse_at_eps_dk(orc):
    # Eqs. 11, 12, 15 together: straight channels whose every pore has the reference
    # diameter relax at tau_ref = 1 and carry, in physical units, eps times the Knudsen
    # diffusivity of that diameter (tortuosity 1)
    d_ref_nm, voxel_nm, T = 60.0, 2.0, 400.0
    pore = W.square_duct(10, 4, pad=1)
    d_ref = d_ref_nm / voxel_nm
    tg = np.where(pore == 1, orc.tau_g(np.full(pore.shape, d_ref), d_ref, 1.0), 1.0)
    assert np.all(tg[pore == 1] == 1.0)
    r = orc.knudsen_solve(pore, tg, 1.0, 0.0, tol=1e-13, max_steps=200_000, want_c=False,
                          want_planes=False)
    dk = orc.knudsen_diffusivity(d_ref_nm * 1e-9, T)
    d_phys = orc.deff_physical(r["Deff_lattice"], 0.25, 1.0, dk)
    assert d_phys == pytest.approx(pore.mean() * dk, rel=1e-9)


def test_permeability_units_resolution_invariant(orc):
    # one physical slit (12 nm of fluid in a 16 nm period) at 2 nm and at 1 nm voxels:
    # Eq. 15's k dx^2 gives the same physical permeability, near the continuum
    # eps H^2/12 = 0.75 (12 nm)^2 / 12 = 9e-18 m^2, the finer grid the closer
    out = []
    for h, n, dx in ((6, 8, 2e-9), (12, 16, 1e-9)):
        pore = W.slit(2, n, 2, h, axis=1)
        r = orc.flow_solve(pore, tau=0.8, force=(1e-6, 0.0, 0.0), tol=1e-12, max_steps=400_000,
                           want_u=False)
        out.append(orc.k_physical(r["k_lattice"], dx))
    assert out[0] == pytest.approx(9e-18, rel=1e-2)
    assert out[1] == pytest.approx(9e-18, rel=3e-3)
    assert abs(out[1] - 9e-18) < abs(out[0] - 9e-18)
    assert orc.m2_to_mD(out[1]) == pytest.approx(out[1] / 9.869233e-16, rel=1e-15)


def test_tau_g_eq12(orc):
    # tau_g = tau_ref at d = d_ref, 1/2 at d = 0, linear in between
    assert orc.tau_g(40.0, 40.0, 1.0) == 1.0
    assert orc.tau_g(0.0, 40.0, 1.0) == 0.5
    d = np.array([1.0, 10.0, 20.0, 80.0])
    assert np.allclose(orc.tau_g(d, 40.0, 1.0), 0.5 + 0.5 * d / 40.0, rtol=1e-15)
