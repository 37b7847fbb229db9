"""Steady state (Section 3.4: k and D_eff are taken once the simulation is steady).

The residual alone bounds only the change per step.  With steady_tol the flow solve also
needs its estimated distance to steady state (from the decay of the residual) and the
Knudsen solve the same flux through every link plane; both are judged here against
solves run far longer, at the 1e-3 agreement the warm-started and batched forms are held
to.  Also: the warm start's fallback to the solve from rest."""
import sys

import numpy as np
import pytest
import torch

from paper_1410_1921_amd import lbm, warmstart as WS, workloads as W

pytestmark = pytest.mark.gpu

KN = dict(tau_ref=1.0, d_ref_nm=60.0, voxel_nm=2.0, c_in=1.0, c_out=0.0, T=400.0)


def say(*a):
    print("[gpu-steady]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def geom():
    torch.cuda.set_device(0)
    rp = W.warmstart_params(6000, 64)
    say("geometry", rp)
    pore, diam, rs = WS.geometry(rp)
    return pore, diam, rs["n_pore"]


def test_flow_steady_tol(geom):
    pore, _, nf = geom
    kw = dict(tau=0.8, force=(1e-6, 0, 0), max_steps=400_000, n_fluid=nf)
    plain = lbm.lbm_flow_solve(pore, tol=1e-7, **kw)
    steady = lbm.lbm_flow_solve(pore, tol=1e-7, steady_tol=1e-3, **kw)
    # the reference runs three times as long
    ref = lbm.lbm_flow_solve(pore, fixed_steps=3 * steady["steps"], **kw)
    e_plain = abs(plain["k_lattice"] / ref["k_lattice"] - 1)
    e_steady = abs(steady["k_lattice"] / ref["k_lattice"] - 1)
    say("flow steps", plain["steps"], steady["steps"], ref["steps"], "k errors", e_plain, e_steady,
        "distance estimate", steady["steady_dist"])
    assert steady["converged"]
    assert steady["steady_dist"] <= 1e-3 and steady["residual"] < 1e-7
    assert steady["steps"] >= plain["steps"]
    assert e_steady < 1e-3


def test_knudsen_flux_spread_tol(geom):
    pore, diam, nf = geom
    kw = dict(max_steps=6_000_000, n_fluid=nf, **KN)
    steady = lbm.lbm_knudsen_solve(pore, diam, tol=1e-7, steady_tol=1e-3, **kw)
    ref = lbm.lbm_knudsen_solve(pore, diam, fixed_steps=3 * steady["steps"], **kw)
    e = abs(steady["Deff_lattice"] / ref["Deff_lattice"] - 1)
    pl = steady["plane_flux"]
    say("knudsen steps", steady["steps"], ref["steps"], "spread", steady["flux_spread"],
        ref["flux_spread"], "D_eff error", e)
    assert steady["converged"]
    assert steady["flux_spread"] <= 1e-3 and ref["flux_spread"] < steady["flux_spread"]
    assert (pl.max() - pl.min()) / abs(pl.mean()) == pytest.approx(steady["flux_spread"], rel=1e-12)
    assert e < 1e-3


def test_knudsen_no_path_converges():
    # two solid walls across x: no path between the faces, every steady flux is zero;
    # the spread's floor lets the solve stop
    pore = np.ones((12, 12, 20), np.uint8)
    pore[:, :, 9:11] = 0
    p = torch.from_numpy(pore).cuda()
    d = torch.full(p.shape, 4.0, dtype=torch.float64, device="cuda")
    r = lbm.lbm_knudsen_solve(p, d, tol=1e-7, steady_tol=1e-3, max_steps=2_000_000, **KN)
    say("no path:", r["steps"], r["Deff_lattice"], r["flux_spread"])
    assert r["converged"] and abs(r["Deff_lattice"]) < 1e-9


def test_warm_and_plain_agree(geom):
    pore, diam, nf = geom
    net = WS.load_network()
    _, c0 = WS.predict(net, pore, diam)
    # each form within ~steady_tol/2 of the steady D_eff, possibly from opposite sides
    kw = dict(max_steps=6_000_000, n_fluid=nf, tol=1e-7, steady_tol=5e-4, **KN)
    plain = lbm.lbm_knudsen_solve(pore, diam, **kw)
    warm, used = WS.knudsen_warm_or_rest(pore, diam, c0.contiguous(), **kw)
    d = abs(warm["Deff_lattice"] / plain["Deff_lattice"] - 1)
    say("plain", plain["steps"], "warm", warm["steps"], "used", used, "D_eff diff", d)
    assert used and warm["converged"] and plain["converged"]
    assert warm["steps"] < plain["steps"]
    assert d < 1e-3


def test_warm_start_fallback(geom):
    pore, diam, nf = geom
    kw = dict(max_steps=6_000_000, n_fluid=nf, tol=1e-7, steady_tol=1e-3, **KN)
    plain = lbm.lbm_knudsen_solve(pore, diam, **kw)
    # a finite but wrong prediction (the reversed profile, C = 5 in the middle) does not
    # converge within the warm budget: the solve from rest is run and returned
    nx = pore.shape[2]
    x = torch.arange(nx, device="cuda", dtype=torch.float32) / (nx - 1)
    bad = (x + 4.0 * torch.sin(np.pi * x)).expand(pore.shape).contiguous() * (pore == 1)
    r, used = WS.knudsen_warm_or_rest(pore, diam, bad.float().contiguous(),
                                      warm_max_steps=plain["steps"] // 4, **kw)
    assert not used
    assert r["steps"] == plain["steps"] and r["Deff_lattice"] == plain["Deff_lattice"]
    # without the fallback (a caller whose solve from rest did not converge either) the
    # unconverged warm solve is returned as it stands
    r, used = WS.knudsen_warm_or_rest(pore, diam, bad.float().contiguous(),
                                      warm_max_steps=plain["steps"] // 4, fallback=False, **kw)
    assert used and not r["converged"] and r["steps"] <= plain["steps"] // 4
    # a non-finite prediction diverges at its first check: the same fallback
    nan = torch.full(pore.shape, float("nan"), dtype=torch.float32, device="cuda")
    r, used = WS.knudsen_warm_or_rest(pore, diam, nan, **kw)
    assert not used and r["Deff_lattice"] == plain["Deff_lattice"]


def test_batched_steady_matches_single():
    torch.cuda.set_device(0)
    geoms = []
    for seed in (6001, 6002, 6004):
        pore, diam, rs = WS.geometry(W.warmstart_params(seed, 40))
        geoms.append((pore, diam, rs["n_pore"]))
    fl = [g[0] for g in geoms]
    dm = [g[1] for g in geoms]
    nf = [g[2] for g in geoms]
    fkw = dict(tau=0.8, force=(1e-6, 0, 0), max_steps=200_000, tol=1e-7, steady_tol=1e-3)
    _, bf, _, _ = lbm.lbm_flow_solve_batch(fl, n_fluids=nf, **fkw)
    kkw = dict(max_steps=4_000_000, tol=1e-7, steady_tol=1e-3, **KN)
    _, bk, _, _ = lbm.lbm_knudsen_solve_batch(fl, dm, n_fluids=nf, **kkw)
    for i, (p, d, n) in enumerate(geoms):
        f1 = lbm.lbm_flow_solve(p, n_fluid=n, **fkw)
        k1 = lbm.lbm_knudsen_solve(p, d, n_fluid=n, **kkw)
        say("lattice", i, "flow", f1["steps"], bf[i]["steps"], "knudsen", k1["steps"], bk[i]["steps"])
        assert bf[i]["steps"] == f1["steps"] and bf[i]["converged"] == f1["converged"]
        assert bf[i]["k_lattice"] == pytest.approx(f1["k_lattice"], rel=1e-12)
        assert bk[i]["steps"] == k1["steps"] and bk[i]["converged"] == k1["converged"]
        assert bk[i]["Deff_lattice"] == pytest.approx(k1["Deff_lattice"], rel=1e-12)
