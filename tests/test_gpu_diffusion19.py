"""Mass transport on the paper's D3Q19 lattice (Section 3.2) on the GPU against the FP64
oracle: element-wise C and D_eff at equal step count, sampled populations, link-plane
fluxes, the straight-channel closed form, the edge-connected staircase that D3Q7 cannot
cross, identical fields across kernel variants, and the paper's validation case (a
solid sphere inscribed in a 100^3 cube, Section 3.5)."""
import sys

import numpy as np
import pytest
import torch

from paper_1410_1921_amd import lbm
from paper_1410_1921_amd import workloads as W

pytestmark = pytest.mark.gpu
Q19 = lbm.LBM_LATTICE_D3Q19


def say(*a):
    print("[gpu-d3q19]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("shape,seed", [((19, 10, 14), 2), ((33, 7, 5), 8), ((1, 9, 30), 4),
                                        ((12, 30, 41), 9)])
def test_parity_ragged(orc, shape, seed):
    m = W.blob_mask(shape, 0.6, seed)
    diam = W.hash_field(shape, seed, 1.0, 40.0).astype(np.float64) * m
    tg = np.where(m == 1, orc.tau_g(diam, 20.0, 1.0), 1.0)
    say("ragged", shape)
    r = lbm.lbm_knudsen_solve(dev(m), dev(diam), d_ref_nm=30.0, voxel_nm=1.5, c_in=0.8, c_out=0.3,
                              fixed_steps=400, check_every=50, want_c=True, lattice=Q19)
    o = orc.diffusion19_solve(m, tg, 0.8, 0.3, fixed_steps=400, check_every=50)
    assert r["steps"] == o["steps"] == 400
    assert np.abs(r.field.cpu().numpy() - o["c"]).max() < 1e-5
    assert r["Deff_lattice"] == pytest.approx(o["Deff_lattice"], rel=1e-4)
    assert r["phi_in"] == pytest.approx(o["phi_in"], rel=1e-4, abs=1e-7)
    # link-plane fluxes of the final state
    assert np.allclose(r["plane_flux"], o["plane_flux"], rtol=1e-4,
                       atol=1e-5 * np.abs(o["plane_flux"]).max())
    # populations (stored deviation + a_i C_ref) at every fluid voxel
    vox = np.flatnonzero(m.reshape(-1))[:4000]
    g, tau, flag = lbm.lbm_knudsen_sample(r.workspace, vox)
    assert flag.all() and g.shape == (len(vox), 19)
    assert np.abs(g - o["g"].reshape(-1, 19)[vox]).max() < 2e-6
    assert np.allclose(tau, tg.reshape(-1)[vox], rtol=1e-6)


def test_parity_32(orc):
    w = W.SMALL_32
    rp, kp = w["recon"], w["knudsen"]
    pore_g, _, _ = lbm.lbm_reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                       rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    d_g = lbm.lbm_pore_diameter(pore_g, lbm.LBM_PSD_CHORD13)
    pore, d = pore_g.cpu().numpy(), d_g.cpu().numpy()
    d_ref = kp["d_ref_nm"] / w["voxel_nm"]
    tg = np.where(pore == 1, orc.tau_g(d, d_ref, kp["tau_ref"]), 1.0)
    say("32^3 reconstruction")
    r = lbm.lbm_knudsen_solve(pore_g, d_g, tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"],
                              voxel_nm=w["voxel_nm"], c_in=kp["c_in"], c_out=kp["c_out"],
                              fixed_steps=kp["fixed_steps"], check_every=kp["check_every"],
                              want_c=True, lattice=Q19)
    o = orc.diffusion19_solve(pore, tg, kp["c_in"], kp["c_out"], fixed_steps=kp["fixed_steps"],
                              check_every=kp["check_every"])
    assert np.abs(r.field.cpu().numpy() - o["c"]).max() < 1e-5
    assert r["Deff_lattice"] == pytest.approx(o["Deff_lattice"], rel=1e-4)
    assert r["residual"] == pytest.approx(o["residual"], rel=1e-3)
    say("Deff", r["Deff_lattice"], o["Deff_lattice"])


@pytest.mark.parametrize("tau", [0.7, 1.0, 1.6])
def test_straight_channel_closed_form(tau):
    nx = 14
    m = np.ones((2, 3, nx), np.uint8)
    d = np.full(m.shape, (tau - 0.5) / 0.5 * 40.0)  # d_ref = 40 voxels, tau_ref = 1
    # a fixed 30 000 steps, some 90 relaxation times of the slowest mode (a residual
    # criterion bounds the change per step, not the distance to steady state)
    r = lbm.lbm_knudsen_solve(dev(m), dev(d), d_ref_nm=60.0, voxel_nm=1.5, fixed_steps=30_000,
                              lattice=Q19)
    want = (tau - 0.5) / 3 * (nx + 1) / (nx - 1 + 2 * tau)
    say("channel tau", tau, r["Deff_lattice"], want, r["steps"])
    assert r["Deff_lattice"] == pytest.approx(want, rel=2e-6)
    if tau == 1.0:
        assert r["tortuosity"] == pytest.approx(1.0, rel=2e-6)


def test_edge_connected_staircase(orc):
    nx = ny = 10
    m = np.zeros((1, ny, nx), np.uint8)
    for x in range(nx):
        m[0, x, x] = 1
    d = 40.0 * m.astype(np.float64)
    kw = dict(d_ref_nm=60.0, voxel_nm=1.5, max_steps=200_000, tol=1e-8)
    r19 = lbm.lbm_knudsen_solve(dev(m), dev(d), lattice=Q19, **kw)
    r7 = lbm.lbm_knudsen_solve(dev(m), dev(d), **kw)
    o = orc.diffusion19_solve(m, 1.0, 1.0, 0.0, max_steps=200_000, tol=1e-12)
    say("staircase D_eff d3q19", r19["Deff_lattice"], "oracle", o["Deff_lattice"], "d3q7",
        r7["Deff_lattice"])
    assert r19["Deff_lattice"] == pytest.approx(o["Deff_lattice"], rel=1e-4)
    assert r19["Deff_lattice"] > 1e-3 and abs(r7["Deff_lattice"]) < 1e-9


def test_variants_identical_and_resume():
    m = W.blob_mask((21, 30, 40), 0.55, 12)
    d = W.hash_field(m.shape, 3, 2.0, 50.0).astype(np.float64) * m
    E = lbm.LBM_VARIANT_EXPLICIT
    fm, fd = dev(m), dev(d)
    runs = [lbm.lbm_knudsen_solve(fm, fd, fixed_steps=250, check_every=50, want_c=True,
                                  lattice=Q19, variant=v)
            for v in (0, E, E | lbm.LBM_VARIANT_REMAP, E | lbm.LBM_VARIANT_NTSTORE)]
    for r in runs[1:]:
        assert torch.equal(r.field, runs[0].field)
    # stepping on, and a resume with another lattice is refused
    a = runs[0]
    lbm.lbm_knudsen_step(a.workspace, 10)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_knudsen_solve(fm, fd, fixed_steps=10, workspace=a.workspace, resume=True)
    b = lbm.lbm_knudsen_solve(fm, fd, fixed_steps=40, check_every=50, workspace=a.workspace,
                              resume=True, want_c=True, lattice=Q19)
    c = lbm.lbm_knudsen_solve(fm, fd, fixed_steps=300, check_every=50, want_c=True, lattice=Q19)
    assert np.abs(b.field.cpu().numpy() - c.field.cpu().numpy()).max() < 1e-6


def test_sphere_in_cube_section_3_5():
    # the paper's validation on its D3Q19 lattice: D_eff / D = 0.3317
    m = W.sphere_in_cube(100)
    d = np.full(m.shape, 40.0)  # tau_g = tau_ref = 1
    r = lbm.lbm_knudsen_solve(dev(m), dev(d), d_ref_nm=60.0, voxel_nm=1.5, max_steps=2_000_000,
                              tol=1e-8, lattice=Q19)
    say("sphere in cube D3Q19 D_eff/D", r["Deff_over_DKref"], "steps", r["steps"],
        "mlups", r["mlups"])
    assert r["converged"]
    # measured 0.3358 (+1.2 %); Eq. 14 is read with the distance between the ghost planes,
    # nx + 1 = 101 (a straight channel then has tortuosity exactly 1); with L_x = nx the
    # same state gives 0.3325.  The paper states neither its length nor its voxelisation.
    assert r["Deff_over_DKref"] == pytest.approx(0.3317, rel=0.015)
