"""The shipped warm-start network: predictions are well formed, and on a held-out
geometry the warm-started Knudsen solve reaches steady state in fewer steps, with D_eff
within 1e-3 of the solve from rest and of a much longer solve."""
import sys

import pytest
import torch

from paper_1410_1921_amd import lbm, warmstart as WS, workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-warmstart]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def net():
    return WS.load_network()


def test_prediction_is_well_formed(net):
    rp = W.warmstart_params(6003, 32)
    pore, diam, _ = WS.geometry(rp)
    u0, c0 = WS.predict(net, pore, diam)
    assert u0.shape == (4, 32, 32, 32) and c0.shape == (32, 32, 32)
    solid = pore == 0
    assert torch.isfinite(u0).all() and torch.isfinite(c0).all()
    assert (u0[:, solid] == 0).all() and (c0[solid] == 0).all()
    u1, c1 = WS.predict(net, pore, diam)
    assert torch.equal(u0, u1) and torch.equal(c0, c1)


def test_warm_knudsen_solve_saves_steps(net):
    cfg = W.WARMSTART
    rp = W.warmstart_params(6000, cfg["edge"])
    pore, diam, rs = WS.geometry(rp)
    kp = cfg["knudsen"]

    def solve(c_init, **kw):
        return lbm.lbm_knudsen_solve(pore, diam, tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"],
                                     voxel_nm=cfg["voxel_nm"], c_in=kp["c_in"], c_out=kp["c_out"],
                                     T=kp["T"], max_steps=kp["max_steps"], c_init=c_init,
                                     n_fluid=rs["n_pore"], **kw)

    # both forms stop at residual 1e-7 with the same flux through every link plane (spread
    # <= 5e-4: D_eff within ~2.5e-4 of steady state); both are judged against a solve run
    # three times as long, and against each other at 1e-3
    plain = solve(None, tol=1e-7, steady_tol=5e-4)
    _, c0 = WS.predict(net, pore, diam)
    warm = solve(c0.contiguous(), tol=1e-7, steady_tol=5e-4)
    tight = solve(None, fixed_steps=3 * plain["steps"])
    ref = tight["Deff_lattice"]
    e_plain = abs(plain["Deff_lattice"] / ref - 1)
    e_warm = abs(warm["Deff_lattice"] / ref - 1)
    d = abs(warm["Deff_lattice"] / plain["Deff_lattice"] - 1)
    say("knudsen steps", plain["steps"], "->", warm["steps"], "(reference", tight["steps"], ")",
        "D_eff errors vs reference: plain", e_plain, "warm", e_warm, "between", d)
    assert plain["converged"] and warm["converged"]
    assert warm["steps"] < plain["steps"]
    assert e_plain < 1e-3 and e_warm < 1e-3 and d < 1e-3
