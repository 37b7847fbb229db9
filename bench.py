"""Benchmark of the lattice Boltzmann hot path on one MI355X.

Headline: the 512^3 workload (porosity 0.25, sphere diameters N(16, 4) voxels, overlap
tolerance 0.7, seed 3; 33.5 M fluid nodes, 5.1 GB of binary32 populations, far beyond
the 256 MB Infinity Cache).  One step = 1000 steps of the D3Q19 flow solve (BGK, Guo
body force 1e-6 along x, half-way bounce-back, binary32 storage) with a convergence check
every 100, continuing one solve on the resident geometry.  `value` = fluid-node updates
per second of the timed steps, in MLUPS.  `roofline`: the stream-collide launches of the
timed region, 152 algorithmic bytes per update over their mean duration (HIP events on
the solve's stream, inside the library).

Extra keys (each measured once, outside the timed region):
  crop         the 128^3 centre crop of the 512^3 workload: k of binary64, binary32 and
               binary16 storage against the FP64 oracle at its stored step count, and the
               time to the converged k of each (residual 1e-7 and the steady-state test)
  sweeps_512   binary16, MRT and TRT sweep times on the 512^3 workload
  pipeline_128 the 128^3 methane workload (cache-resident: its state fits the 256 MB
               Infinity Cache, so its figures are no HBM claim): reconstruction, labelling,
               pore map, flow and Knudsen solves to steady state, plain against the
               learned warm start (time to converged k and D_eff, and their agreement)
  batch        the 150-lattice batch workload at a fixed step count, batched and single
  batch_converge  time to converged k and D_eff of the first lattices of the batch, one
               solve after the other from rest against batched + warm-started
  cpu_baseline the FP64 oracle on a bounded sample of the headline workload
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & % HBM roofline; time-to-converged k and D_eff, plain vs warm-start+FP16"
HBM_PEAK_GBS = 8000.0
BYTES_D3Q19 = 152  # 19 loads + 19 stores of binary32 per fluid-node update
BYTES_D3Q19_F16 = 76  # the same in binary16
BYTES_D3Q7 = 60    # 7 loads + 7 stores of binary32 + 1/tau_g
BYTES_D3Q19D = 156  # the D3Q19 diffusion lattice: 19 loads + 19 stores + 1/tau_g
STEPS_PER_BENCH_STEP = 1000
# the solves' stop rule: residual 1e-7 and the steady-state test (flow: estimated distance
# to steady state <= 1e-3; Knudsen: link-plane flux spread <= 2e-3, which holds the outlet
# D_eff within ~1e-3 of its steady value and the plane-mean D_eff far closer)
TOL, FLOW_STEADY, KN_STEADY = 1e-7, 1e-3, 2e-3
# the batch and held-out lattices (edges up to 96, most fast to converge): flux spread
# <= 5e-4, so that each form's outlet D_eff is within ~2.5e-4 of steady state and two
# forms within 1e-3 of each other
KN_STEADY_EVAL = 5e-4
SWEEP19 = "k_sweep19<StoreF32, false, true, 0, false, unsigned int>"
SWEEP7 = "k_sweep7<false, false, unsigned int>"

# HBM bytes per launch from the committed counter runs (profiles/): FETCH_SIZE and
# WRITE_SIZE in KiB per dispatch, scaled by what the same counters read for the
# library's copy kernel on 2 GiB buffers (FETCH_SIZE reports half of the bytes read,
# WRITE_SIZE all of the bytes written).  A figure holds only while the kernel's sources
# are those that were profiled (hash of the files).
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0
COUNTERS = {
    SWEEP7: dict(
        workload="recon128_eps0.40_d12_mis_ch4_400K", fetch_kib=15340.9, write_kib=22966.8,
        files=("paper_1410_1921_amd/csrc/knudsen.hip", "paper_1410_1921_amd/csrc/lbm_internal.h",
               "paper_1410_1921_amd/csrc/common.hip"), sha="b62b1248619e5586"),
    SWEEP19: dict(
        workload="recon512_eps0.25_d16", fetch_kib=2217149.4, write_kib=2490369.7,
        files=("paper_1410_1921_amd/csrc/flow.hip", "paper_1410_1921_amd/csrc/lbm_internal.h",
               "paper_1410_1921_amd/csrc/common.hip"), sha="3613d5c4e8f11afe"),
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def traffic_gb(kernel, workload):
    """Calibrated HBM bytes per launch (GB) of `kernel` on `workload` from the committed
    counter runs, or None when there are none or the kernel's sources have changed."""
    import hashlib
    c = COUNTERS.get(kernel)
    if c is None or c["workload"] != workload:
        return None
    h = hashlib.sha256()
    for f in c["files"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != c["sha"]:
        return None
    return round((c["fetch_kib"] * FETCH_FACTOR + c["write_kib"] * WRITE_FACTOR) * 1024 / 1e9, 5)


def recon(lbm, rp):
    pore, _, rs = lbm.lbm_reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                      rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    return pore, rs


def geometry_512(lbm, W):
    """The 512^3 reconstruction and its connectivity (stage times)."""
    import torch
    w = W.LARGE_512
    t0 = time.perf_counter()
    pore, rs = recon(lbm, w["recon"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, _, ls = lbm.lbm_label(pore, want_transport=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return pore, rs, ls, {"reconstruct": round(t1 - t0, 3), "label": round(t2 - t1, 3)}


def flow_kw(w, **kw):
    fp = w["flow"]
    return dict(tau=fp["tau"], force=fp["force"], check_every=fp["check_every"],
                voxel_nm=w["voxel_nm"], **kw)


def sweep_ms(lbm, workspace, steps):
    """Mean launch time of `steps` plain sweeps of the state in `workspace` (HIP events on
    the current stream, which the library launches on)."""
    import torch
    s = torch.cuda.current_stream()
    lbm.lbm_flow_step(workspace, 10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    lbm.lbm_flow_step(workspace, steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def sweeps_512(lbm, W, pore, nf, steps):
    """Per-launch times of the binary16, MRT and TRT flow sweeps, of a step with pressure
    boundaries, and of the D3Q7 sweep on the 512^3 workload."""
    import torch
    w = W.LARGE_512
    out = {}
    for name, kw, bpu in (("fp16", dict(storage=lbm.LBM_STORE_FP16), BYTES_D3Q19_F16),
                          ("mrt", dict(collision=lbm.LBM_COLLIDE_MRT), BYTES_D3Q19),
                          ("trt", dict(collision=lbm.LBM_COLLIDE_TRT), BYTES_D3Q19)):
        r = lbm.lbm_flow_solve(pore, fixed_steps=20, n_fluid=nf, **flow_kw(w, **kw))
        ms = sweep_ms(lbm, r.workspace, steps)
        out[name] = {"ms_per_launch": round(ms, 5), "mlups": round(nf / (ms * 1e3), 1),
                     "bytes_per_update": bpu,
                     "achieved_gbs": round(nf * bpu / (ms * 1e-3) / 1e9, 1)}
        del r
        torch.cuda.empty_cache()
    # pressure boundaries in x (Section 3.3) instead of the body force: per step, the
    # ghost-plane kernel and the sweep with open x faces
    fp = w["flow"]
    r = lbm.lbm_flow_solve(pore, tau=fp["tau"], force=(0.0, 0.0, 0.0), pressure=(1.0001, 0.9999),
                           check_every=fp["check_every"], voxel_nm=w["voxel_nm"],
                           fixed_steps=20, n_fluid=nf)
    ms = sweep_ms(lbm, r.workspace, steps)
    out["pressure"] = {"ms_per_step": round(ms, 5), "mlups": round(nf / (ms * 1e3), 1),
                       "bytes_per_update": BYTES_D3Q19,
                       "achieved_gbs": round(nf * BYTES_D3Q19 / (ms * 1e-3) / 1e9, 1),
                       "note": "ghost planes + sweep with open x faces, per step"}
    del r
    torch.cuda.empty_cache()
    # the D3Q7 mass-transport sweep streaming the same lattice from HBM (tau_g from the
    # 13-direction chord map, the methane settings); HIP events around plain sweeps
    kp = W.METHANE_128["knudsen"]
    diam = lbm.lbm_pore_diameter(pore, lbm.LBM_PSD_CHORD13)
    r = lbm.lbm_knudsen_solve(pore, diam, tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"],
                              voxel_nm=w["voxel_nm"], c_in=kp["c_in"], c_out=kp["c_out"],
                              T=kp["T"], fixed_steps=20, check_every=kp["check_every"],
                              n_fluid=nf)
    s = torch.cuda.current_stream()
    lbm.lbm_knudsen_step(r.workspace, 10)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    lbm.lbm_knudsen_step(r.workspace, steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out["d3q7"] = {"kernel": "k_sweep7<false, true, unsigned int>", "ms_per_launch": round(ms, 5),
                   "mlups": round(nf / (ms * 1e3), 1), "bytes_per_update": BYTES_D3Q7,
                   "achieved_gbs": round(nf * BYTES_D3Q7 / (ms * 1e-3) / 1e9, 1),
                   "bound": "hbm"}
    del r, diam
    torch.cuda.empty_cache()
    return out


def crop_precision(lbm, W, pore):
    """The 128^3 centre crop of the 512^3 workload: each storage against the FP64 oracle at
    the oracle's stored step count, and each storage to steady state (time, steps, k and
    its error against the binary64 solve)."""
    import torch
    w = W.LARGE_512
    (z0, z1), (y0, y1), (x0, x1) = w["crop"]
    sub = pore[z0:z1, y0:y1, x0:x1].contiguous()
    nf = lbm.lbm_count(sub)
    gold = None
    path = os.path.join(ROOT, "tests", "golden", "oracle_crop.json")
    if os.path.exists(path):  # written by the oracle alone (tests/golden/make_oracle_golden.py)
        with open(path) as fh:
            gold = json.load(fh)["flow_20000"]
    out = {"crop": w["crop"], "n_fluid": nf}
    stores = (("fp64", lbm.LBM_STORE_FP64), ("fp32", lbm.LBM_STORE_FP32),
              ("fp16", lbm.LBM_STORE_FP16))
    cap = 2_000_000
    for name, st in stores:
        rec = {}
        if gold is not None:
            r = lbm.lbm_flow_solve(sub, fixed_steps=gold["steps"], n_fluid=nf,
                                   **flow_kw(w, storage=st))
            rec["k_vs_oracle_rel"] = r["k_lattice"] / gold["k_lattice"] - 1
            rec["oracle_steps"] = gold["steps"]
        if name == "fp16":  # its residual stops decaying at the rounding floor
            cap = out["fp32"]["steps"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lbm.lbm_flow_solve(sub, max_steps=cap, tol=TOL, steady_tol=FLOW_STEADY,
                               n_fluid=nf, **flow_kw(w, storage=st))
        torch.cuda.synchronize()
        rec.update(time_to_converged_s=round(time.perf_counter() - t0, 3), steps=r["steps"],
                   converged=bool(r["converged"]), k_lattice=r["k_lattice"],
                   steady_dist=r["steady_dist"], mlups=round(r["mlups"], 1))
        out[name] = rec
        log("crop", name, rec)
    k64 = out["fp64"]["k_lattice"]
    for name in ("fp32", "fp16"):
        out[name]["k_vs_fp64_converged_rel"] = out[name]["k_lattice"] / k64 - 1
    out["fp16_note"] = ("binary16 does not meet the stop rule (its residual stops decaying at "
                        "the rounding floor); its run is capped at binary32's steps")
    del sub
    torch.cuda.empty_cache()
    return out


def pipeline_128(lbm, W, net=None):
    """One pass of the whole path on the 128^3 methane workload to steady state; with the
    network, the Knudsen solve starts from its predicted C (inference inside the timing;
    the solve from rest is the fallback)."""
    import torch
    from paper_1410_1921_amd import warmstart as WS
    w = W.METHANE_128
    rp, kp = w["recon"], w["knudsen"]
    t = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pore, rs = recon(lbm, rp)
    _, _, ls = lbm.lbm_label(pore, want_transport=False)
    diam = lbm.lbm_pore_diameter(pore, lbm.LBM_PSD_MIS)
    torch.cuda.synchronize()
    t["geometry"] = time.perf_counter() - t0
    nf = ls["n_pore"]
    t1 = time.perf_counter()
    fr = lbm.lbm_flow_solve(pore, max_steps=w["flow"]["max_steps"], tol=TOL,
                            steady_tol=FLOW_STEADY, n_fluid=nf, **flow_kw(w))
    t["flow"] = time.perf_counter() - t1
    kw = dict(tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"], voxel_nm=w["voxel_nm"],
              c_in=kp["c_in"], c_out=kp["c_out"], T=kp["T"], max_steps=kp["max_steps"],
              check_every=kp["check_every"], tol=TOL, steady_tol=KN_STEADY, n_fluid=nf)
    t1 = time.perf_counter()
    warm_used = False
    if net is None:
        kr = lbm.lbm_knudsen_solve(pore, diam, **kw)
    else:
        _, c0 = WS.predict(net, pore, diam)
        kr, warm_used = WS.knudsen_warm_or_rest(pore, diam, c0.contiguous(), **kw)
    torch.cuda.synchronize()
    t["knudsen"] = time.perf_counter() - t1
    props = lbm.lbm_props(ls, fr, kr, d_mean_nm=rp["d_mean"] * w["voxel_nm"], T=kp["T"])
    t["total"] = time.perf_counter() - t0
    return dict(label=ls, flow=fr, knudsen=kr, props=props, t=t, warm_used=warm_used)


def pipelines_128(lbm, W):
    from paper_1410_1921_amd import warmstart as WS
    log("128^3 pipeline, plain")
    p = pipeline_128(lbm, W)
    log("128^3 pipeline, warm start")
    net = WS.load_network()
    q = pipeline_128(lbm, W, net)
    fr, kr, kw_ = p["flow"], p["knudsen"], q["knudsen"]
    per7 = kr["sweep_ms"] / kr["steps"]
    return {
        "workload": W.METHANE_128["name"], "n_fluid": fr["n_fluid"],
        "note": "cache-resident (state < 256 MB Infinity Cache): not an HBM figure",
        "stop_rule": {"tol": TOL, "flow_steady_dist": FLOW_STEADY, "knudsen_flux_spread": KN_STEADY},
        "plain": {"time_to_converged_s": round(p["t"]["total"], 3),
                  "stage_s": {k: round(v, 3) for k, v in p["t"].items()},
                  "flow_steps": fr["steps"], "knudsen_steps": kr["steps"],
                  "k_lattice": fr["k_lattice"], "k_mD": fr["k_mD"],
                  "Deff_lattice": kr["Deff_lattice"], "Deff_planes": kr["Deff_planes"],
                  "Deff_m2s": kr["Deff_m2s"],
                  "tortuosity": kr["tortuosity"], "flux_spread": kr["flux_spread"],
                  "flow_mlups": round(fr["mlups"], 1), "knudsen_mlups": round(kr["mlups"], 1),
                  "connectivity": p["label"]["connectivity"],
                  "bruggeman_alpha": p["props"]["bruggeman_alpha"]},
        "warm_start": {"time_to_converged_s": round(q["t"]["total"], 3),
                       "knudsen_steps": kw_["steps"], "warm_used": q["warm_used"],
                       "Deff_lattice": kw_["Deff_lattice"], "Deff_planes": kw_["Deff_planes"],
                       "flux_spread": kw_["flux_spread"],
                       "applied_to": "Knudsen C (the flow starts from rest)"},
        "speedup": round(p["t"]["total"] / q["t"]["total"], 3),
        "knudsen_speedup": round(p["t"]["knudsen"] / q["t"]["knudsen"], 3),
        "deff_rel_diff": abs(kw_["Deff_lattice"] / kr["Deff_lattice"] - 1),
        "deff_planes_rel_diff": abs(kw_["Deff_planes"] / kr["Deff_planes"] - 1),
        "k_rel_diff": abs(q["flow"]["k_lattice"] / fr["k_lattice"] - 1),
        "k_sweep7": {"kernel": SWEEP7, "ms_per_launch": per7,
                     "achieved_gbs": round(kr["n_fluid"] * BYTES_D3Q7 / (per7 * 1e-3) / 1e9, 1),
                     "bound": "cache", "traffic": traffic_gb(SWEEP7, W.METHANE_128["name"]),
                     "traffic_unit": "GB per launch"},
    }


def batch_geometry(lbm, W, count, max_edge=1024):
    """The first `count` reconstructions of the batch workload with an edge of at most
    max_edge, with their pore maps."""
    import torch
    fl, dm, nf = [], [], []
    sel = [rp for rp in W.batch_params(W.BATCH["count"]) if rp["n"][0] <= max_edge][:count]
    for rp in sel:
        pore, rs = recon(lbm, rp)
        fl.append(pore)
        nf.append(rs["n_pore"])
        dm.append(lbm.lbm_pore_diameter(pore, lbm.LBM_PSD_MIS))
    torch.cuda.synchronize()
    return fl, dm, nf


def _kn_args(W):
    b = W.BATCH
    kp = b["knudsen"]
    return dict(tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"], voxel_nm=b["voxel_nm"],
                c_in=kp["c_in"], c_out=kp["c_out"], T=kp["T"], check_every=kp["check_every"])


def batch_throughput(lbm, W, flow_steps, kn_steps):
    """The whole batch workload for a fixed number of steps: the batched solves (autotuned
    schedule, graphs) against the same lattices solved one after the other."""
    import torch
    fl, dm, nf = batch_geometry(lbm, W, W.BATCH["count"])
    fp = W.BATCH["flow"]
    ka = _kn_args(W)
    out = {"workload": W.BATCH["name"], "lattices": len(fl), "n_fluid": int(sum(nf)),
           "flow_steps": flow_steps, "knudsen_steps": kn_steps}
    t0 = time.perf_counter()
    _, res, _, sc = lbm.lbm_flow_solve_batch(fl, tau=fp["tau"], force=fp["force"],
                                             fixed_steps=flow_steps,
                                             check_every=fp["check_every"], n_fluids=nf)
    torch.cuda.synchronize()
    out["flow_batched"] = {"mlups": round(res[0]["mlups"], 1),
                           "wall_s": round(time.perf_counter() - t0, 3),
                           "group_bytes": sc["group_bytes_run"], "groups": sc["groups"]}
    t0 = time.perf_counter()
    sw = 0.0
    for f, n in zip(fl, nf):
        sw += lbm.lbm_flow_solve(f, tau=fp["tau"], force=fp["force"], fixed_steps=flow_steps,
                                 check_every=fp["check_every"], n_fluid=n)["sweep_ms"]
    torch.cuda.synchronize()
    out["flow_single"] = {"mlups": round(sum(nf) * flow_steps / (sw * 1e3), 1),
                          "wall_s": round(time.perf_counter() - t0, 3)}
    t0 = time.perf_counter()
    _, res, _, sc = lbm.lbm_knudsen_solve_batch(fl, dm, fixed_steps=kn_steps, n_fluids=nf, **ka)
    torch.cuda.synchronize()
    out["knudsen_batched"] = {"mlups": round(res[0]["mlups"], 1),
                              "wall_s": round(time.perf_counter() - t0, 3),
                              "group_bytes": sc["group_bytes_run"], "groups": sc["groups"]}
    t0 = time.perf_counter()
    sw = 0.0
    for f, d, n in zip(fl, dm, nf):
        sw += lbm.lbm_knudsen_solve(f, d, fixed_steps=kn_steps, n_fluid=n, want_planes=False,
                                    **ka)["sweep_ms"]
    torch.cuda.synchronize()
    out["knudsen_single"] = {"mlups": round(sum(nf) * kn_steps / (sw * 1e3), 1),
                             "wall_s": round(time.perf_counter() - t0, 3)}
    del fl, dm
    torch.cuda.empty_cache()
    return out


def batch_converge(lbm, W, count, net, max_edge=96):
    """Time to the converged k and D_eff (residual 1e-7 and the steady-state test) of the
    first `count` lattices of the batch workload with an edge of at most max_edge: plain
    (one solve after the other, from rest) against batched (autotuned groups, graphs)
    with the Knudsen solves warm-started by the network."""
    import torch
    from paper_1410_1921_amd import warmstart as WS
    fl, dm, nf = batch_geometry(lbm, W, count, max_edge)
    fp = W.BATCH["flow"]
    ka = _kn_args(W)
    kp = W.BATCH["knudsen"]
    fkw = dict(tau=fp["tau"], force=fp["force"], max_steps=fp["max_steps"],
               check_every=fp["check_every"], tol=TOL, steady_tol=FLOW_STEADY,
               voxel_nm=W.BATCH["voxel_nm"])
    kkw = dict(max_steps=kp["max_steps"], tol=TOL, steady_tol=KN_STEADY_EVAL, **ka)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_f = [lbm.lbm_flow_solve(f, n_fluid=n, **fkw) for f, n in zip(fl, nf)]
    torch.cuda.synchronize()
    t_pf = time.perf_counter() - t0
    plain_k = [lbm.lbm_knudsen_solve(f, d, n_fluid=n, want_planes=False, **kkw)
               for f, d, n in zip(fl, dm, nf)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    log(f"batch converge: plain {t_plain:.1f} s (flow {t_pf:.1f} s)")
    t0 = time.perf_counter()
    _, bf, _, sf = lbm.lbm_flow_solve_batch(fl, n_fluids=nf, **fkw)
    torch.cuda.synchronize()
    t_bf = time.perf_counter() - t0
    c0 = [WS.predict(net, f, d)[1].contiguous() for f, d in zip(fl, dm)]
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0 - t_bf
    _, bk, _, sk = lbm.lbm_knudsen_solve_batch(fl, dm, n_fluids=nf, c_inits=c0, **kkw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batch converge: batched + warm {t_batch:.1f} s (flow {t_bf:.1f} s)")
    # relative differences over the lattices with a pore path along x (their flow
    # converges to a nonzero k); the others have k and D_eff at round-off level
    perc = [i for i, p in enumerate(plain_f) if p["converged"] and p["k_lattice"] > 1e-12]
    dk = [abs(bf[i]["k_lattice"] / plain_f[i]["k_lattice"] - 1) for i in perc]
    dd = [abs(bk[i]["Deff_lattice"] / plain_k[i]["Deff_lattice"] - 1) for i in perc]
    ddp = [abs(bk[i]["Deff_planes"] / plain_k[i]["Deff_planes"] - 1) for i in perc]
    return {"workload": W.BATCH["name"], "lattices": len(fl), "n_fluid": int(sum(nf)),
            "selection": f"the first {len(fl)} lattices with an edge of at most {max_edge}",
            "edges": [int(f.shape[0]) for f in fl],
            "stop_rule": {"tol": TOL, "flow_steady_dist": FLOW_STEADY,
                          "knudsen_flux_spread": KN_STEADY_EVAL},
            "form": "batched + warm-started Knudsen, binary32 state; binary16 is left out "
                    "(on the 512^3 crop it is 1.19 x faster per sweep but 6e-3 off in k and "
                    "its residual stalls at its rounding floor, so it never meets the stop "
                    "rule)",
            "plain_s": round(t_plain, 2), "plain_flow_s": round(t_pf, 2),
            "batched_warm_s": round(t_batch, 2), "batched_flow_s": round(t_bf, 2),
            "inference_s": round(t_inf, 2), "speedup": round(t_plain / t_batch, 3),
            "flow_steps_plain": sum(p["steps"] for p in plain_f),
            "flow_steps_batched": sum(b["steps"] for b in bf),
            "knudsen_steps_plain": sum(p["steps"] for p in plain_k),
            "knudsen_steps_warm": sum(b["steps"] for b in bk),
            "converged": [sum(p["converged"] for p in plain_f), sum(b["converged"] for b in bf),
                          sum(p["converged"] for p in plain_k), sum(b["converged"] for b in bk)],
            "percolating": len(perc),
            "k_rel_diff_max": max(dk) if dk else 0.0,
            "deff_rel_diff_max": max(dd) if dd else 0.0,
            "deff_planes_rel_diff_max": max(ddp) if ddp else 0.0,
            "schedule": {"flow": sf, "knudsen": sk}}


def c3_converge(lbm, W, pore, nf):
    """Time to the converged k of the whole 512^3 workload, binary32 against binary16
    storage (long: the pressure field of a porosity-0.25 medium relaxes slowly)."""
    import torch
    w = W.LARGE_512
    out = {"workload": w["name"], "n_fluid": nf,
           "stop_rule": {"tol": TOL, "flow_steady_dist": FLOW_STEADY}}
    for name, st in (("fp32", lbm.LBM_STORE_FP32), ("fp16", lbm.LBM_STORE_FP16)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = lbm.lbm_flow_solve(pore, max_steps=w["flow"]["max_steps"], tol=TOL,
                               steady_tol=FLOW_STEADY, n_fluid=nf, **flow_kw(w, storage=st))
        torch.cuda.synchronize()
        out[name] = {"time_to_converged_s": round(time.perf_counter() - t0, 2),
                     "steps": r["steps"], "converged": bool(r["converged"]),
                     "k_lattice": r["k_lattice"], "k_mD": r["k_mD"], "residual": r["residual"],
                     "steady_dist": r["steady_dist"], "mlups": round(r["mlups"], 1)}
        log("c3 converge", name, out[name])
        del r
        torch.cuda.empty_cache()
    out["k_fp16_vs_fp32_rel"] = out["fp16"]["k_lattice"] / out["fp32"]["k_lattice"] - 1
    out["speedup_fp16"] = round(out["fp32"]["time_to_converged_s"] /
                                out["fp16"]["time_to_converged_s"], 3)
    return out


def warm_eval(lbm, W, seeds, weights=None):
    """The learned warm start on held-out geometries (the warm-start workload's laws at
    96^3): plain against warm-started solves, one after the other, to steady state
    (weights: another weights file than the shipped one)."""
    from paper_1410_1921_amd import warmstart as WS
    net = WS.load_network(weights)
    # flows without a path along x never meet the stop rule (u decays to 0): capped
    cfg = dict(W.WARMSTART, flow=dict(W.WARMSTART["flow"], max_steps=60_000))
    rows = WS.evaluate(net, seeds, cfg, tol=TOL, log=lambda *a: log(*a),
                       steady=(FLOW_STEADY, KN_STEADY_EVAL))
    return {"seeds": [int(s) for s in seeds], "summary": WS.summary(rows), "rows": rows}


def copy_ceiling(lbm, nbytes=1 << 30, reps=5):
    """Attainable HBM bandwidth: the library's streaming copy kernel on `nbytes` buffers,
    read + write bytes per second from HIP events on the current stream (best of reps)."""
    import torch
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    s = torch.cuda.current_stream()
    lbm.lbm_copy_probe(dst, src)
    best = 0.0
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        lbm.lbm_copy_probe(dst, src)
        e1.record(s)
        torch.cuda.synchronize()
        best = max(best, 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return round(best, 1)


def copy_sizes(lbm, sizes_mb=(8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 512, 2048), reps=50):
    """Copy rate of the library's copy kernel against the working-set size: `reps` copies
    of each size captured in one HIP graph, replayed 4 times, timed with HIP events
    (read + write bytes per second).  Sizes up to 256 MB each way fit in the Infinity
    Cache."""
    import torch
    out = {}
    for mb in sizes_mb:
        n = mb << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(7)
        dst = torch.empty_like(src)
        lbm.lbm_copy_probe(dst, src)
        torch.cuda.synchronize()
        k = reps if mb <= 256 else 10
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(k):
                lbm.lbm_copy_probe(dst, src)
        g.replay()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(4):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / (4 * k)
        assert torch.equal(dst, src)
        out[mb] = {"us": round(us, 2), "gbs": round(2 * n / (us * 1e-6) / 1e9, 1)}
        log("copy", mb, "MB each way", out[mb])
        del src, dst, g
        torch.cuda.empty_cache()
    return out


def network_timing(lbm, W, reps=10):
    """The warm-start U-Net on one 96^3 geometry of the warm-start laws: inference
    (forward) and training steps (forward, masked loss, every gradient, Adam), HIP events
    on the current stream, mean over `reps` after one untimed pass each.  FLOP: 2 x 27 x
    cin x cout per voxel and 3x3x3 convolution, three such products per training step
    (forward, input gradient, weight gradient)."""
    import torch
    from paper_1410_1921_amd import warmstart as WS
    from paper_1410_1921_amd.unet import UNet
    net = WS.load_network()
    edge = W.WARMSTART["edge"]
    pore, diam, rs = WS.geometry(W.warmstart_params(6000, edge))
    shape = tuple(pore.shape)
    x0 = WS.network_input(pore, diam)
    fwd_flop = 0
    for name, ci, co in net.layers:
        level = net._level(name)
        fwd_flop += 2 * 27 * ci * co * (edge >> level) ** 3
    s = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_inf = timed(lambda: net.forward(shape, x0))
    trainee = UNet(n_out=WS.N_OUT, seed=1)
    target = torch.zeros((WS.N_OUT, pore.numel()), dtype=torch.float32, device="cuda")
    mask = pore.reshape(-1).contiguous()
    wt = torch.tensor(WS.LOSS_WT, dtype=torch.float32, device="cuda")

    def step():
        trainee.loss_and_grad(shape, x0, target, mask, wt, float(rs["n_pore"]))
        trainee.adam(lr=1e-4)

    ms_train = timed(step)
    peak = 2500.0  # dense bf16 MFMA, TFLOP/s
    out = {"edge": edge, "layers": len(net.layers), "forward_gflop": round(fwd_flop / 1e9, 2),
           "inference_ms": round(ms_inf, 3),
           "inference_tflops": round(fwd_flop / (ms_inf * 1e-3) / 1e12, 2),
           "train_step_ms": round(ms_train, 3),
           "train_tflops": round(3 * fwd_flop / (ms_train * 1e-3) / 1e12, 2),
           "peak_tflops": peak}
    out["train_frac"] = round(out["train_tflops"] / peak, 4)
    log("network", out)
    return out


def flow_sizes(lbm, edges=(256, 320, 384, 448, 512), steps=30):
    """Time per fluid-node update of the binary32 flow sweep against lattice size
    (reconstructions drawn like the 512^3 workload), best of 2."""
    import torch
    out = {}
    for n in edges:
        pore, st = lbm.lbm_reconstruct((n, n, n), 0.25, 16.0, 4.0, 1.0, 0.7, 0.5, 3)
        nf = st["n_pore"]
        r = lbm.lbm_flow_solve(pore, tau=0.8, force=(1e-6, 0, 0), fixed_steps=20,
                               check_every=100, n_fluid=nf)
        best = min(sweep_ms(lbm, r.workspace, steps) for _ in range(2))
        out[n] = {"n_fluid": nf, "ms_per_launch": round(best, 4),
                  "ps_per_update": round(best * 1e9 / nf, 2)}
        log("flow size", n, out[n])
        del r, pore
        torch.cuda.empty_cache()
    return out


def cpu_baseline(W, w, steps, edge=128):
    """The FP64 oracle on a bounded sample of workload `w`: its own reconstruction with the
    workload's parameters on an edge^3 box (the whole lattice when the workload is no
    larger), then `steps` D3Q19 BGK steps of the flow on it."""
    import oracle as orc
    rp = dict(w["recon"])
    n = tuple(min(int(e), edge) for e in rp["n"])
    t0 = time.perf_counter()
    pore, _, info = orc.reconstruct(n, rp["porosity"], rp["d_mean"], rp["d_std"],
                                    rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    t_rec = time.perf_counter() - t0
    what = "the whole lattice" if n == tuple(rp["n"]) else \
        f"a {n[0]}x{n[1]}x{n[2]} box drawn with the workload's parameters"
    fp = w["flow"]
    t1 = time.perf_counter()
    orc.flow_solve(pore, tau=fp["tau"], force=fp["force"], fixed_steps=steps, want_u=False)
    dt = time.perf_counter() - t1
    nf = int(pore.sum())
    return {"value": round(steps * nf / dt / 1e6, 3), "unit": "MLUPS",
            "cores": orc.num_threads(), "kind": "oracle",
            "sample": f"{w['name']}: {steps} D3Q19 BGK steps of {what} ({nf} fluid nodes, "
                      f"FP64, dense lattice) in {dt:.1f} s, after the oracle's own "
                      f"reconstruction ({t_rec:.1f} s)"}


def headline(lbm, W, pore, nf, steps, warmup):
    """The timed loop: `steps` bench steps of STEPS_PER_BENCH_STEP solve steps each."""
    import torch
    w = W.LARGE_512
    r = lbm.lbm_flow_solve(pore, fixed_steps=w["flow"]["check_every"], n_fluid=nf, **flow_kw(w))
    ws = r.workspace
    kw = flow_kw(w, fixed_steps=STEPS_PER_BENCH_STEP, n_fluid=nf, workspace=ws, resume=True)
    for i in range(warmup):
        lbm.lbm_flow_solve(pore, **kw)
        log(f"warmup {i}")
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for i in range(steps):
        runs.append(lbm.lbm_flow_solve(pore, **kw).result)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    log(f"{steps} steps in {wall:.3f} s")
    return runs, wall, ws


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-steps", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="headline line only")
    ap.add_argument("--batch-steps", type=int, default=500,
                    help="fixed steps of each lattice in the batch-workload leg")
    ap.add_argument("--batch-converge", type=int, default=8, metavar="COUNT",
                    help="lattices of the batch workload (edges up to 96) in the "
                         "time-to-converged leg")
    ap.add_argument("--only-512", action="store_true",
                    help="only the 512^3 geometry and sweeps, after 2 GiB copies by the library's "
                         "copy kernel that calibrate the HBM byte counters (profiling runs)")
    ap.add_argument("--roofline-steps", type=int, default=100)
    ap.add_argument("--only-knudsen", type=int, default=0, metavar="STEPS",
                    help="only the 128^3 geometry and STEPS Knudsen sweeps (profiling runs)")
    ap.add_argument("--only-c3-converge", action="store_true",
                    help="only the time to converged k of the 512^3 workload, binary32 and "
                         "binary16")
    ap.add_argument("--only-warm-eval", type=int, default=0, metavar="COUNT",
                    help="only the learned warm start on COUNT held-out geometries")
    ap.add_argument("--warm-eval-start", type=int, default=0, metavar="INDEX",
                    help="first held-out geometry of --only-warm-eval")
    ap.add_argument("--warm-eval-weights", default=None, metavar="NPZ",
                    help="network weights for --only-warm-eval (default: the shipped ones)")
    ap.add_argument("--only-batch", action="store_true",
                    help="only the batch workload's fixed-step throughput (--batch-steps)")
    ap.add_argument("--only-batch-converge", type=int, default=0, metavar="COUNT",
                    help="only the time-to-converged leg of the batch workload")
    ap.add_argument("--only-flow-sizes", action="store_true")
    ap.add_argument("--only-network", action="store_true",
                    help="only the warm-start U-Net: inference and training-step timing")
    ap.add_argument("--only-copy-sizes", action="store_true",
                    help="only the copy kernel's rate against the working-set size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path's multi-GPU "
              "decomposition is a design, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1410_1921_amd import lbm
    from paper_1410_1921_amd import workloads as W

    torch.cuda.set_device(0)
    lbm.load()
    if args.only_flow_sizes:
        print(json.dumps({"flow_sizes": flow_sizes(lbm)}), flush=True)
        return
    if args.only_network:
        print(json.dumps({"network": network_timing(lbm, W)}), flush=True)
        return
    if args.only_copy_sizes:
        print(json.dumps({"copy_sizes": copy_sizes(lbm)}), flush=True)
        return
    if args.only_batch:
        print(json.dumps({"batch": batch_throughput(lbm, W, args.batch_steps, args.batch_steps)}),
              flush=True)
        return
    if args.only_warm_eval:
        i0 = args.warm_eval_start
        seeds = list(W.WARMSTART["test_seeds"])[i0:i0 + args.only_warm_eval]
        print(json.dumps({"warm_eval": warm_eval(lbm, W, seeds, args.warm_eval_weights)}),
              flush=True)
        return
    if args.only_batch_converge:
        from paper_1410_1921_amd import warmstart as WS
        print(json.dumps({"batch_converge": batch_converge(lbm, W, args.only_batch_converge,
                                                           WS.load_network())}), flush=True)
        return
    if args.only_knudsen:
        w = W.METHANE_128
        rp, kp = w["recon"], w["knudsen"]
        ceiling = copy_ceiling(lbm, 1 << 31, 3)
        pore, rs = recon(lbm, rp)
        diam = lbm.lbm_pore_diameter(pore, lbm.LBM_PSD_MIS)
        kr = lbm.lbm_knudsen_solve(pore, diam, tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"],
                                   voxel_nm=w["voxel_nm"], c_in=kp["c_in"], c_out=kp["c_out"],
                                   T=kp["T"], fixed_steps=args.only_knudsen,
                                   check_every=kp["check_every"], n_fluid=rs["n_pore"])
        per = kr["sweep_ms"] / kr["steps"]
        print(json.dumps({"knudsen_sweeps": {
            "kernel": SWEEP7, "workload": w["name"], "n_fluid": kr["n_fluid"],
            "steps": kr["steps"], "ms_per_launch": per,
            "achieved_gbs": round(kr["n_fluid"] * BYTES_D3Q7 / (per * 1e-3) / 1e9, 1)},
            "copy_kernel": "k_copy_probe", "copy_gbs": ceiling}), flush=True)
        return

    log("512^3 geometry")
    pore, rs, ls, geo_s = geometry_512(lbm, W)
    nf = rs["n_pore"]
    w = W.LARGE_512
    if args.only_c3_converge:
        print(json.dumps({"c3_converge": c3_converge(lbm, W, pore, nf)}), flush=True)
        return
    if args.only_512:
        ceiling = copy_ceiling(lbm, 1 << 31, 3)
        r = lbm.lbm_flow_solve(pore, fixed_steps=20, n_fluid=nf, **flow_kw(w))
        ms = sweep_ms(lbm, r.workspace, args.roofline_steps)
        del r
        torch.cuda.empty_cache()
        print(json.dumps({"fp32": {"kernel": SWEEP19, "ms_per_launch": ms,
                                   "achieved_gbs": round(nf * BYTES_D3Q19 / (ms * 1e-3) / 1e9, 1)},
                          "sweeps_512": sweeps_512(lbm, W, pore, nf, args.roofline_steps),
                          "copy_kernel": "k_copy_probe", "copy_bytes_each_way": 1 << 31,
                          "copy_gbs": ceiling}), flush=True)
        return

    log("headline: 512^3 flow solve steps")
    runs, wall, ws = headline(lbm, W, pore, nf, args.steps, args.warmup)
    n_upd = sum(r["steps"] for r in runs)
    value = nf * n_upd / wall / 1e6
    sw_ms = sum(r["sweep_ms"] for r in runs)
    per = sw_ms / n_upd
    achieved = nf * BYTES_D3Q19 / (per * 1e-3) / 1e9
    last = runs[-1]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "n": list(w["recon"]["n"]), "n_fluid": nf,
                   "lattice": "D3Q19 BGK + Guo force, half-way bounce-back, periodic",
                   "storage": "f32 offsets from linear reference densities per half row "
                              "segment",
                   "solve_steps_per_step": STEPS_PER_BENCH_STEP,
                   "check_every": w["flow"]["check_every"]},
        "roofline": {"kernel": SWEEP19, "bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_gb(SWEEP19, w["name"]), "traffic_unit": "GB per launch",
                     "bytes_per_update": BYTES_D3Q19, "n_fluid": nf, "ms_per_launch": per,
                     "share_of_step": round(sw_ms / (wall * 1e3), 4),
                     "timing": "HIP events on the solve's stream around the sweep launches"},
        "solve_state": {"steps_done": STEPS_PER_BENCH_STEP * (args.steps + args.warmup) +
                        w["flow"]["check_every"], "k_lattice": last["k_lattice"],
                        "residual": last["residual"]},
        "geometry": {"porosity": ls["porosity"], "connectivity": ls["connectivity"],
                     "n_spheres": rs["n_spheres"], "stage_s": geo_s},
    }
    del ws
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("512^3 sweep variants")
        out["sweeps_512"] = sweeps_512(lbm, W, pore, nf, args.roofline_steps)
        log("crop precision")
        out["crop"] = crop_precision(lbm, W, pore)
        del pore
        torch.cuda.empty_cache()
        out["pipeline_128"] = pipelines_128(lbm, W)
        log("batch workload")
        out["batch"] = batch_throughput(lbm, W, args.batch_steps, args.batch_steps)
        if args.batch_converge:
            from paper_1410_1921_amd import warmstart as WS
            log("batch converge")
            out["batch_converge"] = batch_converge(lbm, W, args.batch_converge,
                                                   WS.load_network())
        log("copy ceiling")
        out["attainable_copy_gbs"] = copy_ceiling(lbm)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(W, w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
