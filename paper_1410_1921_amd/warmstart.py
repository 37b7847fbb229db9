"""Learned warm start of the flow and Knudsen solves (an addition to the paper's method).

The U-Net (unet.py) maps a geometry -- pore mask and maximum-inscribed-sphere diameter
map -- to initial fields: u and rho - 1 for the D3Q19 flow solve, C for the D3Q7 Knudsen
solve.  The solves then iterate to their own residual criterion, so the network only
changes the number of steps; the solve from rest stays the reference for the result.

By default only the Knudsen solve is warm-started: on held-out geometries the predicted
C saved ~30% of the Knudsen steps, while the predicted (u, rho - 1) made the (already
short) flow solves longer than from rest; flow_warm=True applies them anyway.

Network outputs are scaled: u / U_SCALE, (rho - 1) / R_SCALE, C (a body force of 1e-6
gives speeds of order 1e-4 in pores of ten voxels); inputs are the mask and the pore
diameter / D_SCALE.
"""
import concurrent.futures as cf
import time

import numpy as np
import torch

from . import lbm, nn
from . import workloads as W
from .nn import View
from .unet import C_IN, UNet

U_SCALE = 1e-4
R_SCALE = 1e-4
D_SCALE = 20.0
N_OUT = 5
LOSS_WT = (1.0, 1.0, 1.0, 1.0, 1.0)


def geometry(rp):
    pore, _, rs = lbm.lbm_reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                      rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    diam = lbm.lbm_pore_diameter(pore, lbm.LBM_PSD_MIS)
    return pore, diam, rs


def solve_pair(pore, diam, cfg, tol, u_init=None, c_init=None, n_fluid=None, steady=(0.0, 0.0)):
    """Flow (with rho - 1 in the returned field) and Knudsen solves of one geometry to
    residual tol and the steady-state tests steady = (flow, Knudsen) (0: residual only);
    returns the two Solve objects and their wall times."""
    fp, kp = cfg["flow"], cfg["knudsen"]
    t0 = time.perf_counter()
    fr = lbm.lbm_flow_solve(pore, tau=fp["tau"], force=fp["force"], max_steps=fp["max_steps"],
                            check_every=fp["check_every"], tol=tol, voxel_nm=cfg["voxel_nm"],
                            want_u=True, with_rho=True, u_init=u_init, n_fluid=n_fluid,
                            steady_tol=steady[0])
    t1 = time.perf_counter()
    kr = lbm.lbm_knudsen_solve(pore, diam, tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"],
                               voxel_nm=cfg["voxel_nm"], c_in=kp["c_in"], c_out=kp["c_out"],
                               T=kp["T"], max_steps=kp["max_steps"],
                               check_every=kp["check_every"], tol=tol, want_c=True,
                               c_init=c_init, n_fluid=n_fluid, steady_tol=steady[1])
    torch.cuda.current_stream().synchronize()
    return fr, kr, (t1 - t0, time.perf_counter() - t1)


def knudsen_warm_or_rest(pore, diam, c_init, warm_max_steps=None, fallback=True, **kw):
    """Knudsen solve started from the network's C, with the solve from rest as the
    fallback.  The warm solve is kept only when it meets the solve's own stop rule (the
    residual and, with steady_tol, the equal flux through every link plane) within
    warm_max_steps steps (default: kw's max_steps); when it does not, or when it diverges
    (a non-finite prediction), the solve runs again from rest with kw unchanged.  With
    fallback=False (the caller knows the solve from rest does not converge within kw's
    max_steps either) a warm solve that does not converge is kept; divergence still
    falls back.  Returns (Solve, warm_used)."""
    warm_kw = dict(kw)
    if warm_max_steps is not None:
        warm_kw["max_steps"] = int(warm_max_steps)
    try:
        r = lbm.lbm_knudsen_solve(pore, diam, c_init=c_init, **warm_kw)
        if r["converged"] or not fallback:
            return r, True
    except lbm.LbmError as e:
        if e.status != lbm.LBM_E_DIVERGED:
            raise
    return lbm.lbm_knudsen_solve(pore, diam, **kw), False


def flow_warm_or_rest(pore, u_init, warm_max_steps=None, **kw):
    """The same for the flow solve: the warm start from u_init (with kw's with_rho, its
    fourth plane rho - 1) is kept only when it converges by the solve's own rule within
    warm_max_steps; otherwise the solve runs from rest.  Returns (Solve, warm_used)."""
    warm_kw = dict(kw)
    if warm_max_steps is not None:
        warm_kw["max_steps"] = int(warm_max_steps)
    try:
        r = lbm.lbm_flow_solve(pore, u_init=u_init, **warm_kw)
        if r["converged"]:
            return r, True
    except lbm.LbmError as e:
        if e.status != lbm.LBM_E_DIVERGED:
            raise
    return lbm.lbm_flow_solve(pore, **kw), False


def _scales(dev, inverse):
    s = np.array([U_SCALE, U_SCALE, U_SCALE, R_SCALE, 1.0], np.float32)
    return torch.from_numpy(1.0 / s if inverse else s).to(dev)


def targets(fr, kr, pore):
    """The network's training target from converged solves: planar float32 [5][nvox]."""
    raw = torch.cat([fr.field.reshape(4, -1), kr.field.reshape(1, -1)])
    out = torch.empty_like(raw)
    nn.lbm_nn_to_fields(raw, pore.reshape(-1), _scales(pore.device, True), out)
    return out


def network_input(pore, diam, x0=None):
    if x0 is None:
        x0 = torch.empty((pore.numel(), C_IN), dtype=torch.bfloat16, device=pore.device)
    nn.lbm_nn_make_input(pore.reshape(-1), diam.reshape(-1), D_SCALE, View(x0))
    return x0


def predict(net, pore, diam):
    """Initial fields for the solves: u_init (float32 [4][nz][ny][nx]: u and rho - 1) and
    c_init (float32 [nz][ny][nx]), zero at solids."""
    shape = tuple(pore.shape)
    out = net.forward(shape, network_input(pore, diam))
    fields = torch.empty_like(out)
    nn.lbm_nn_to_fields(out, pore.reshape(-1), _scales(pore.device, False), fields)
    return fields[:4].reshape((4,) + shape), fields[4].reshape(shape)


def make_dataset(seeds, cfg=W.WARMSTART, tol=1e-6, workers=8, flow_cap=60_000, log=print,
                 steady=(0.0, 0.0), kn_cap=None):
    """Solves each seed's geometry from rest (concurrently, one stream per worker) and
    keeps the network input and target on the device.  The flow solve stops at flow_cap
    steps: geometries without a path along x have u = 0 at steady state, where the
    relative residual measures the decay rate of the transient and never reaches tol.
    With a steady-state test (steady, as in solve_pair) the Knudsen solve stops at kn_cap
    steps (default: the configuration's), and a geometry whose Knudsen solve does not
    meet the test is left out (its target would not be the steady state)."""
    cfg = dict(cfg, flow=dict(cfg["flow"], max_steps=min(cfg["flow"]["max_steps"], flow_cap)))
    if kn_cap is not None:
        cfg["knudsen"] = dict(cfg["knudsen"], max_steps=int(kn_cap))
    data = [None] * len(seeds)
    t_start = time.perf_counter()

    def work(k):
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            rp = W.warmstart_params(seeds[k], cfg["edge"])
            pore, diam, rs = geometry(rp)
            fr, kr, (tf, tk) = solve_pair(pore, diam, cfg, tol, n_fluid=rs["n_pore"],
                                          steady=steady)
            if steady[1] > 0 and not kr["converged"]:
                s.synchronize()
                log(f"sample {k + 1}/{len(seeds)} seed {seeds[k]}: Knudsen not steady in "
                    f"{kr['steps']} steps, left out")
                return
            item = dict(seed=seeds[k], shape=tuple(pore.shape), x0=network_input(pore, diam),
                        tgt=targets(fr, kr, pore), mask=pore.reshape(-1).clone(),
                        n_mask=float(rs["n_pore"]), steps=(fr["steps"], kr["steps"]),
                        k=fr["k_lattice"], deff=kr["Deff_lattice"])
            s.synchronize()
        data[k] = item
        log(f"sample {k + 1}/{len(seeds)} seed {seeds[k]}: flow {fr['steps']} knudsen "
            f"{kr['steps']} steps ({tf:.2f} + {tk:.2f} s), {time.perf_counter() - t_start:.0f} s")

    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for f in [ex.submit(work, k) for k in range(len(seeds))]:
            f.result()
    return [d for d in data if d is not None]


def train(net, data, epochs, lr=1e-3, log=print, seed=0):
    wt = torch.tensor(LOSS_WT, dtype=torch.float32, device=net.p.device)
    rng = np.random.default_rng(seed)
    history = []
    steps = epochs * len(data)
    it = 0
    for ep in range(epochs):
        tot = 0.0
        t0 = time.perf_counter()
        for k in rng.permutation(len(data)):
            d = data[k]
            tot += net.loss_and_grad(d["shape"], d["x0"], d["tgt"], d["mask"], wt, d["n_mask"])
            # cosine decay to lr / 10
            net.adam(lr=lr * (0.1 + 0.45 * (1 + np.cos(np.pi * it / max(steps - 1, 1)))))
            it += 1
        history.append(tot / len(data))
        log(f"epoch {ep + 1}/{epochs}: mean loss {history[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
    return history


def evaluate(net, seeds, cfg=W.WARMSTART, tol=1e-7, log=print, flow_warm=False,
             steady=(0.0, 0.0)):
    """Solves each held-out geometry from rest and from the network's fields (one after
    the other, so the wall times compare) to residual tol and the steady-state tests
    `steady` (see solve_pair); the warm-started solves fall back to the solve from rest
    when they do not converge (when that solve converged: otherwise the rerun would
    repeat it).  Without flow_warm the flow starts from rest in both forms,
    one computation counted in both.  A geometry with no pore component joining x = 0 to
    x = nx - 1 (Section 4.1's connectivity) carries no flux in either solve: k = D_eff = 0
    at steady state, so it is recorded without solving (no_path).  Returns one record per
    seed."""
    fp, kp = cfg["flow"], cfg["knudsen"]
    rows = []
    for seed in seeds:
        rp = W.warmstart_params(seed, cfg["edge"])
        pore, diam, rs = geometry(rp)
        nf = rs["n_pore"]
        _, _, ls = lbm.lbm_label(pore, want_transport=False)
        if ls["n_transport"] == 0:
            rows.append(dict(seed=seed, porosity=rs["porosity"], n_fluid=nf, no_path=True,
                             plain_steps=[0, 0], warm_steps=[0, 0], plain_s=[0.0, 0.0],
                             warm_s=[0.0, 0.0], inference_s=0.0,
                             converged=[True, True, True, True], warm_used=False,
                             k_plain=0.0, k_warm=0.0, deff_plain=0.0, deff_warm=0.0))
            log(f"held-out seed {seed}: no path along x (k = D_eff = 0), not solved")
            continue
        p_f, p_k, (p_tf, p_tk) = solve_pair(pore, diam, cfg, tol, n_fluid=nf, steady=steady)
        t0 = time.perf_counter()
        u0, c0 = predict(net, pore, diam)
        torch.cuda.current_stream().synchronize()
        t_inf = time.perf_counter() - t0
        if flow_warm:
            t0 = time.perf_counter()
            w_f, _ = flow_warm_or_rest(
                pore, u0.contiguous(), tau=fp["tau"], force=fp["force"],
                max_steps=fp["max_steps"], check_every=fp["check_every"], tol=tol,
                voxel_nm=cfg["voxel_nm"], with_rho=True, n_fluid=nf, steady_tol=steady[0])
            torch.cuda.current_stream().synchronize()
            w_tf = time.perf_counter() - t0
        else:
            w_f, w_tf = p_f, p_tf
        t0 = time.perf_counter()
        w_k, used = knudsen_warm_or_rest(
            pore, diam, c0.contiguous(), tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"],
            voxel_nm=cfg["voxel_nm"], c_in=kp["c_in"], c_out=kp["c_out"], T=kp["T"],
            max_steps=kp["max_steps"], check_every=kp["check_every"], tol=tol, n_fluid=nf,
            steady_tol=steady[1], fallback=bool(p_k["converged"]))
        torch.cuda.current_stream().synchronize()
        w_tk = time.perf_counter() - t0
        row = dict(seed=seed, porosity=rs["porosity"], n_fluid=nf,
                   plain_steps=[p_f["steps"], p_k["steps"]], warm_steps=[w_f["steps"], w_k["steps"]],
                   plain_s=[p_tf, p_tk], warm_s=[w_tf, w_tk], inference_s=t_inf,
                   converged=[bool(p_f["converged"]), bool(p_k["converged"]),
                              bool(w_f["converged"]), bool(w_k["converged"])],
                   warm_used=bool(used),
                   k_plain=p_f["k_lattice"], k_warm=w_f["k_lattice"],
                   deff_plain=p_k["Deff_lattice"], deff_warm=w_k["Deff_lattice"],
                   deff_planes_plain=p_k["Deff_planes"], deff_planes_warm=w_k["Deff_planes"])
        rows.append(row)
        log(f"held-out seed {seed}: steps flow {row['plain_steps'][0]} -> {row['warm_steps'][0]}, "
            f"knudsen {row['plain_steps'][1]} -> {row['warm_steps'][1]}; time "
            f"{sum(row['plain_s']):.2f} -> {sum(row['warm_s']) + t_inf:.2f} s")
    return rows


def summary(rows):
    """Step and time ratios over the geometries that were solved (all: those with a path
    along x) and over those whose solves from rest both converged within their caps
    (converged: the time-to-converged comparison); agreement of k and of D_eff (at the
    outlet and the link-plane mean) where both forms converged; the count of geometries
    without a path."""
    no_path = [r for r in rows if r.get("no_path")]
    rows = [r for r in rows if not r.get("no_path")]

    def part(rs):
        if not rs:
            return {}
        ps = np.array([r["plain_steps"] for r in rs], float)
        ws = np.array([r["warm_steps"] for r in rs], float)
        pt = np.array([sum(r["plain_s"]) for r in rs])
        wt = np.array([sum(r["warm_s"]) + r["inference_s"] for r in rs])
        return dict(n=len(rs), flow_steps_ratio=float(ws[:, 0].sum() / ps[:, 0].sum()),
                    knudsen_steps_ratio=float(ws[:, 1].sum() / ps[:, 1].sum()),
                    knudsen_steps_ratio_median=float(np.median(ws[:, 1] / ps[:, 1])),
                    time_plain_s=float(pt.sum()), time_warm_s=float(wt.sum()),
                    speedup=float(pt.sum() / wt.sum()))
    conv = [r for r in rows if r["converged"][0] and r["converged"][1]]
    both_k = [r for r in rows if r["converged"][0] and r["converged"][2]]
    both_d = [r for r in rows if r["converged"][1] and r["converged"][3]]
    dk = np.array([abs(r["k_warm"] / r["k_plain"] - 1) for r in both_k]) if both_k else np.zeros(1)
    dd = np.array([abs(r["deff_warm"] / r["deff_plain"] - 1) for r in both_d if r["deff_plain"] > 0]) \
        if both_d else np.zeros(1)
    dp = np.array([abs(r["deff_planes_warm"] / r["deff_planes_plain"] - 1) for r in both_d
                   if r.get("deff_planes_plain", 0) > 0])
    dp = dp if dp.size else np.zeros(1)
    return dict(all=part(rows), converged=part(conv), no_path=len(no_path),
                k_rel_diff_median=float(np.median(dk)), k_rel_diff_max=float(dk.max()),
                deff_rel_diff_median=float(np.median(dd)), deff_rel_diff_max=float(dd.max()),
                deff_planes_rel_diff_median=float(np.median(dp)),
                deff_planes_rel_diff_max=float(dp.max()),
                knudsen_converged=[sum(r["converged"][1] for r in rows),
                                   sum(r["converged"][3] for r in rows)],
                warm_used=sum(bool(r.get("warm_used", True)) for r in rows))


def default_weights():
    import os
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_warmstart.npz")


def load_network(path=None):
    return UNet.load(path or default_weights())
