"""Benchmark of the whole transport pipeline on one MI355X.

One step = one pass of the hot path over the 128^3 methane workload (2 nm voxels,
porosity 0.40, sphere diameters N(12, 3) voxels, overlap tolerance 0.3): reconstruction,
18-neighbour labelling, maximum-inscribed-sphere pore map, the D3Q19 flow solve to
residual 1e-7 (-> k) and the D3Q7 Knudsen solve to residual 1e-7 (-> D_eff,
tortuosity), and the derived properties.  `value` is fluid-node updates (both lattices)
per second of the whole step, in MLUPS.

The JSON line also carries the roofline of the dominant sweep kernel (algorithmic bytes
per launch / mean launch time from HIP events on the solve's stream), the same figure
for the D3Q19 sweep on the 512^3 workload (working set far beyond the 256 MB Infinity
Cache), and the FP64 CPU oracle timed on a bounded sample of the workload.
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
BYTES_D3Q7 = 60    # 7 loads + 7 stores of binary32 + 1/tau_g
BYTES_D3Q19D = 156  # the D3Q19 diffusion lattice: 19 loads + 19 stores + 1/tau_g


# HBM bytes per launch from the committed counter runs (profiles/k_sweep7_recon128_methane.md,
# profiles/k_sweep19_recon512.md): FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by
# what the same counters read for the library's copy kernel on 2 GiB buffers (FETCH_SIZE
# reports half of the bytes read, WRITE_SIZE all of the bytes written).  A figure holds
# only while the kernel's sources are those that were profiled (hash of the files).
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0
COUNTERS = {
    "k_sweep7<false, false, unsigned int>": dict(
        workload="recon128_eps0.40_d12_mis_ch4_400K", fetch_kib=15341.1, write_kib=22966.8,
        files=("paper_1410_1921_amd/csrc/knudsen.hip", "paper_1410_1921_amd/csrc/lbm_internal.h",
               "paper_1410_1921_amd/csrc/common.hip"), sha="dfc6c486c8137a23"),
    "k_sweep19<StoreF32, false, true, 0, false, unsigned int>": dict(
        workload="recon512_eps0.25_d16", fetch_kib=2142213.7, write_kib=2490369.4,
        files=("paper_1410_1921_amd/csrc/flow.hip", "paper_1410_1921_amd/csrc/lbm_internal.h",
               "paper_1410_1921_amd/csrc/common.hip"), sha="2bd94a8b945f1f9e"),
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


def pipeline(lbm, W, w, net=None):
    """One pass of the hot path; returns a dict of results and per-stage timings.  With
    the warm-start network the Knudsen solve starts from its predicted C (inference
    inside the timed region)."""
    import torch
    rp = w["recon"]
    t = {}
    t0 = time.perf_counter()
    pore, _, rs = lbm.lbm_reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                      rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    t["reconstruct"] = time.perf_counter() - t0
    t1 = time.perf_counter()
    _, _, ls = lbm.lbm_label(pore, want_transport=False)
    t["label"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    method = lbm.LBM_PSD_MIS if rp["psd"] == "mis" else lbm.LBM_PSD_CHORD13
    diam = lbm.lbm_pore_diameter(pore, method)
    torch.cuda.synchronize()
    t["pore_diameter"] = time.perf_counter() - t1
    fp, kp = w["flow"], w["knudsen"]
    c_init = None
    if net is not None:
        from paper_1410_1921_amd import warmstart as WS
        t1 = time.perf_counter()
        _, c_init = WS.predict(net, pore, diam)
        c_init = c_init.contiguous()
        torch.cuda.synchronize()
        t["inference"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    fr = lbm.lbm_flow_solve(pore, tau=fp["tau"], force=fp["force"], max_steps=fp["max_steps"],
                            fixed_steps=fp["fixed_steps"], check_every=fp["check_every"],
                            tol=fp["tol"], voxel_nm=w["voxel_nm"], n_fluid=ls["n_pore"])
    t["flow"] = time.perf_counter() - t1
    t1 = time.perf_counter()
    kr = lbm.lbm_knudsen_solve(pore, diam, tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"],
                               voxel_nm=w["voxel_nm"], c_in=kp["c_in"], c_out=kp["c_out"],
                               T=kp["T"], max_steps=kp["max_steps"], fixed_steps=kp["fixed_steps"],
                               check_every=kp["check_every"], tol=kp["tol"],
                               n_fluid=ls["n_pore"], c_init=c_init)
    t["knudsen"] = time.perf_counter() - t1
    props = lbm.lbm_props(ls, fr, kr, d_mean_nm=rp["d_mean"] * w["voxel_nm"], T=kp["T"])
    torch.cuda.synchronize()
    t["total"] = time.perf_counter() - t0
    return dict(recon=rs, label=ls, flow=fr, knudsen=kr, props=props, t=t)


def roofline_512(lbm, W, steps):
    """Mean launch time of the plain D3Q19 sweep on the 512^3 workload, from HIP events
    on the current stream around `steps` launches."""
    import torch
    w = W.LARGE_512
    rp = w["recon"]
    pore, _, rs = lbm.lbm_reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                      rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    nf = rs["n_pore"]
    fp = w["flow"]
    r = lbm.lbm_flow_solve(pore, tau=fp["tau"], force=fp["force"], fixed_steps=20,
                           check_every=fp["check_every"], voxel_nm=w["voxel_nm"], n_fluid=nf)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lbm.lbm_flow_step(r.workspace, 10)
    torch.cuda.synchronize()
    e0.record(s)
    lbm.lbm_flow_step(r.workspace, steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gbs = nf * BYTES_D3Q19 / (ms * 1e-3) / 1e9
    del r
    torch.cuda.empty_cache()
    # the same sweep with binary16 storage (84 algorithmic bytes per update)
    r = lbm.lbm_flow_solve(pore, tau=fp["tau"], force=fp["force"], fixed_steps=20,
                           check_every=fp["check_every"], voxel_nm=w["voxel_nm"], n_fluid=nf,
                           storage=lbm.LBM_STORE_FP16)
    lbm.lbm_flow_step(r.workspace, 10)
    torch.cuda.synchronize()
    e0.record(s)
    lbm.lbm_flow_step(r.workspace, steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms16 = e0.elapsed_time(e1) / steps
    del r
    torch.cuda.empty_cache()
    # and with the paper's MRT collision (binary32)
    r = lbm.lbm_flow_solve(pore, tau=fp["tau"], force=fp["force"], fixed_steps=20,
                           check_every=fp["check_every"], voxel_nm=w["voxel_nm"], n_fluid=nf,
                           collision=lbm.LBM_COLLIDE_MRT)
    lbm.lbm_flow_step(r.workspace, 10)
    torch.cuda.synchronize()
    e0.record(s)
    lbm.lbm_flow_step(r.workspace, steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms_mrt = e0.elapsed_time(e1) / steps
    del r
    torch.cuda.empty_cache()
    # and the same collision in its two-relaxation-time form
    r = lbm.lbm_flow_solve(pore, tau=fp["tau"], force=fp["force"], fixed_steps=20,
                           check_every=fp["check_every"], voxel_nm=w["voxel_nm"], n_fluid=nf,
                           collision=lbm.LBM_COLLIDE_TRT)
    lbm.lbm_flow_step(r.workspace, 10)
    torch.cuda.synchronize()
    e0.record(s)
    lbm.lbm_flow_step(r.workspace, steps)
    e1.record(s)
    torch.cuda.synchronize()
    ms_trt = e0.elapsed_time(e1) / steps
    del r, pore
    torch.cuda.empty_cache()
    name = "k_sweep19<StoreF32, false, true, 0, false, unsigned int>"
    return {"kernel": name, "workload": w["name"], "n_fluid": nf,
            "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic_gb(name, w["name"]),
            "traffic_unit": "GB per launch", "ms_per_launch": ms,
            "mlups": nf / (ms * 1e3),
            "fp16": {"ms_per_launch": ms16, "mlups": nf / (ms16 * 1e3),
                     "achieved": round(nf * 84 / (ms16 * 1e-3) / 1e9, 1)},
            "mrt": {"kernel": "k_sweep19<StoreF32, false, true, 1, false, unsigned int>",
                    "ms_per_launch": ms_mrt, "mlups": nf / (ms_mrt * 1e3),
                    "achieved": round(nf * BYTES_D3Q19 / (ms_mrt * 1e-3) / 1e9, 1)},
            "trt": {"kernel": "k_sweep19<StoreF32, false, true, 2, false, unsigned int>",
                    "ms_per_launch": ms_trt, "mlups": nf / (ms_trt * 1e3),
                    "achieved": round(nf * BYTES_D3Q19 / (ms_trt * 1e-3) / 1e9, 1)}}


def batch_geometry(lbm, W, count):
    """The first `count` reconstructions of the batch workload with their pore maps."""
    import torch
    fl, dm, nf = [], [], []
    for rp in W.batch_params(W.BATCH["count"])[:count]:
        pore, _, rs = lbm.lbm_reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                          rp["d_min"], rp["overlap_tol"], rp["p_overlap"],
                                          rp["seed"])
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
    out = {"lattices": len(fl), "n_fluid": int(sum(nf)), "flow_steps": flow_steps,
           "knudsen_steps": kn_steps}
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


def batch_converge(lbm, W, count, net):
    """Time to the converged k and D_eff (residual 1e-7) of the first `count` lattices of
    the batch workload: plain (one solve after the other, from rest) against batched
    (autotuned groups, graphs) with the Knudsen solves warm-started by the network."""
    import torch
    from paper_1410_1921_amd import warmstart as WS
    fl, dm, nf = batch_geometry(lbm, W, count)
    fp = W.BATCH["flow"]
    ka = _kn_args(W)
    kp = W.BATCH["knudsen"]
    fkw = dict(tau=fp["tau"], force=fp["force"], max_steps=fp["max_steps"],
               check_every=fp["check_every"], tol=fp["tol"], voxel_nm=W.BATCH["voxel_nm"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_f = [lbm.lbm_flow_solve(f, n_fluid=n, **fkw) for f, n in zip(fl, nf)]
    torch.cuda.synchronize()
    t_pf = time.perf_counter() - t0
    plain_k = [lbm.lbm_knudsen_solve(f, d, n_fluid=n, max_steps=kp["max_steps"], tol=kp["tol"],
                                     want_planes=False, **ka) for f, d, n in zip(fl, dm, nf)]
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
    _, bk, _, sk = lbm.lbm_knudsen_solve_batch(fl, dm, n_fluids=nf, max_steps=kp["max_steps"],
                                               tol=kp["tol"], c_inits=c0, **ka)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    log(f"batch converge: batched + warm {t_batch:.1f} s (flow {t_bf:.1f} s)")
    # relative differences over the lattices with a pore path along x (their flow
    # converges); the others have k and D_eff at round-off level
    perc = [i for i, p in enumerate(plain_f) if p["converged"]]
    dk = [abs(bf[i]["k_lattice"] / plain_f[i]["k_lattice"] - 1) for i in perc]
    dd = [abs(bk[i]["Deff_lattice"] / plain_k[i]["Deff_lattice"] - 1) for i in perc]
    return {"lattices": count, "n_fluid": int(sum(nf)),
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
            "deff_plain": [p["Deff_lattice"] for p in plain_k],
            "deff_warm": [b["Deff_lattice"] for b in bk],
            "schedule": {"flow": sf, "knudsen": sk}}


def knudsen_sweeps(lbm, w, steps):
    """`steps` D3Q7 sweeps on the workload's geometry: mean launch time from the
    library's HIP events."""
    rp, kp = w["recon"], w["knudsen"]
    pore, _, rs = lbm.lbm_reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                      rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    method = lbm.LBM_PSD_MIS if rp["psd"] == "mis" else lbm.LBM_PSD_CHORD13
    diam = lbm.lbm_pore_diameter(pore, method)
    kr = lbm.lbm_knudsen_solve(pore, diam, tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"],
                               voxel_nm=w["voxel_nm"], c_in=kp["c_in"], c_out=kp["c_out"],
                               T=kp["T"], fixed_steps=steps, check_every=kp["check_every"],
                               n_fluid=rs["n_pore"])
    per = kr["sweep_ms"] / kr["steps"]
    gbs = kr["n_fluid"] * BYTES_D3Q7 / (per * 1e-3) / 1e9
    return {"kernel": "k_sweep7", "workload": w["name"], "n_fluid": kr["n_fluid"],
            "steps": kr["steps"], "ms_per_launch": per, "achieved": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def diffusion19_sweeps(lbm, w, steps):
    """`steps` sweeps of the paper's D3Q19 mass-transport lattice on the workload's
    geometry (mean launch time from the library's HIP events), beside the D3Q7 sweep."""
    rp, kp = w["recon"], w["knudsen"]
    pore, _, rs = lbm.lbm_reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                      rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    method = lbm.LBM_PSD_MIS if rp["psd"] == "mis" else lbm.LBM_PSD_CHORD13
    diam = lbm.lbm_pore_diameter(pore, method)
    kw = dict(tau_ref=kp["tau_ref"], d_ref_nm=kp["d_ref_nm"], voxel_nm=w["voxel_nm"],
              c_in=kp["c_in"], c_out=kp["c_out"], T=kp["T"], fixed_steps=steps,
              check_every=kp["check_every"], n_fluid=rs["n_pore"], want_planes=False)
    out = {"workload": w["name"], "n_fluid": rs["n_pore"], "steps": steps}
    for name, lat, bpu in (("d3q19", lbm.LBM_LATTICE_D3Q19, BYTES_D3Q19D),
                           ("d3q7", lbm.LBM_LATTICE_D3Q7, BYTES_D3Q7)):
        kr = lbm.lbm_knudsen_solve(pore, diam, lattice=lat, **kw)
        per = kr["sweep_ms"] / kr["steps"]
        out[name] = {"ms_per_launch": per, "mlups": round(kr["mlups"], 1),
                     "achieved_gbs": round(kr["n_fluid"] * bpu / (per * 1e-3) / 1e9, 1),
                     "bytes_per_update": bpu}
    out["d3q19"]["kernel"] = "k_sweep19d<false, false, unsigned int>"
    return out


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


def flow_sizes(lbm, edges=(256, 320, 384, 448, 512), steps=30):
    """Time per fluid-node update of the binary32 flow sweep against lattice size
    (reconstructions drawn like the 512^3 workload: porosity 0.25, N(16, 4) spheres,
    overlap tolerance 0.7, seed 3), from HIP events over `steps` launches, best of 2."""
    import torch
    s = torch.cuda.current_stream()
    out = {}
    for n in edges:
        pore, _, st = lbm.lbm_reconstruct((n, n, n), 0.25, 16.0, 4.0, 1.0, 0.7, 0.5, 3)
        nf = st["n_pore"]
        r = lbm.lbm_flow_solve(pore, tau=0.8, force=(1e-6, 0, 0), fixed_steps=20,
                               check_every=100, n_fluid=nf)
        best = 1e9
        for _ in range(2):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            lbm.lbm_flow_step(r.workspace, steps)
            e1.record(s)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / steps)
        out[n] = {"n_fluid": nf, "workspace_gb": round(r.workspace.nbytes / 1e9, 2),
                  "ms_per_launch": round(best, 4), "ps_per_update": round(best * 1e9 / nf, 2)}
        log("flow size", n, out[n])
        del r, pore
        torch.cuda.empty_cache()
    return out


def cpu_baseline(W, w, steps):
    """The FP64 oracle on a bounded sample of the workload: the whole geometry stage plus
    `steps` steps of each lattice (instead of running to convergence)."""
    import numpy as np
    import oracle as orc
    rp = w["recon"]
    t0 = time.perf_counter()
    pore, _, info = orc.reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                    rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    orc.label18(pore)
    d = orc.mis(pore) if rp["psd"] == "mis" else orc.chords13(pore)
    fp, kp = w["flow"], w["knudsen"]
    orc.flow_solve(pore, tau=fp["tau"], force=fp["force"], fixed_steps=steps, want_u=False)
    tg = np.where(pore == 1, orc.tau_g(d, kp["d_ref_nm"] / w["voxel_nm"], kp["tau_ref"]), 1.0)
    orc.knudsen_solve(pore, tg, kp["c_in"], kp["c_out"], fixed_steps=steps, want_c=False,
                      want_planes=False)
    dt = time.perf_counter() - t0
    updates = 2 * steps * info["n_pore"]
    return {"value": round(updates / dt / 1e6, 3), "unit": "MLUPS", "cores": orc.num_threads(),
            "kind": "oracle",
            "sample": f"{w['name']}: reconstruction + labelling + pore map + {steps} D3Q19 and "
                      f"{steps} D3Q7 steps (FP64, dense lattice), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="recon128_eps0.40_d12_mis_ch4_400K")
    ap.add_argument("--cpu-steps", type=int, default=800)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-512", action="store_true")
    ap.add_argument("--no-warm", action="store_true", help="skip the warm-started pipeline")
    ap.add_argument("--roofline-steps", type=int, default=100)
    ap.add_argument("--only-512", action="store_true",
                    help="only the 512^3 sweep roofline, after 2 GiB copies by the library's "
                         "copy kernel that calibrate the HBM byte counters (profiling runs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch-workload leg")
    ap.add_argument("--batch-steps", type=int, default=1000,
                    help="fixed steps of each lattice in the batch-workload leg")
    ap.add_argument("--only-batch", action="store_true",
                    help="only the batch-workload leg (profiling runs)")
    ap.add_argument("--batch-converge", type=int, default=0, metavar="COUNT",
                    help="only the time to converged solutions of the first COUNT lattices of "
                         "the batch workload, plain against batched + warm-started")
    ap.add_argument("--only-knudsen", type=int, default=0, metavar="STEPS",
                    help="only the geometry stages and STEPS Knudsen sweeps of the workload, "
                         "after the same copy calibration (profiling runs)")
    ap.add_argument("--only-copy-sizes", action="store_true",
                    help="only the copy rate against working-set size (cache vs HBM)")
    ap.add_argument("--only-flow-sizes", action="store_true",
                    help="only the flow sweep's time per update against lattice size")
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
    if args.only_512:
        # counter calibration: three 2 GiB copies by the library's copy kernel
        ceiling = copy_ceiling(lbm, 1 << 31, 3)
        print(json.dumps({"roofline_512": roofline_512(lbm, W, args.roofline_steps),
                          "copy_kernel": "k_copy_probe", "copy_bytes_each_way": 1 << 31,
                          "copy_copies": 4, "copy_gbs": ceiling}), flush=True)
        return
    if args.only_flow_sizes:
        print(json.dumps({"flow_sizes": flow_sizes(lbm)}), flush=True)
        return
    if args.only_copy_sizes:
        print(json.dumps({"copy_sizes_mb": copy_sizes(lbm), "copy_kernel": "k_copy_probe"}),
              flush=True)
        return
    if args.only_batch:
        print(json.dumps({"batch": batch_throughput(lbm, W, args.batch_steps, args.batch_steps),
                          "workload": W.BATCH["name"]}), flush=True)
        return
    if args.batch_converge:
        from paper_1410_1921_amd import warmstart as WS
        print(json.dumps({"batch_converge": batch_converge(lbm, W, args.batch_converge,
                                                           WS.load_network()),
                          "workload": W.BATCH["name"]}), flush=True)
        return
    w = W.WORKLOADS[args.workload]
    if args.only_knudsen:
        ceiling = copy_ceiling(lbm, 1 << 31, 3)
        print(json.dumps({"knudsen_sweeps": knudsen_sweeps(lbm, w, args.only_knudsen),
                          "copy_kernel": "k_copy_probe", "copy_bytes_each_way": 1 << 31,
                          "copy_copies": 4, "copy_gbs": ceiling}), flush=True)
        return
    log("workload", w["name"])
    for i in range(args.warmup):
        r = pipeline(lbm, W, w)
        log(f"warmup {i}: {r['t']['total']:.2f} s, flow {r['flow']['steps']} steps, "
            f"knudsen {r['knudsen']['steps']} steps")
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        runs.append(pipeline(lbm, W, w))
        log(f"step {i}: {runs[-1]['t']}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    last = runs[-1]
    nf = last["flow"]["n_fluid"]
    updates = sum((r["flow"]["steps"] + r["knudsen"]["steps"]) * nf for r in runs)
    value = updates / wall / 1e6

    # dominant kernel over the timed region, from the library's HIP events
    fl_ms = sum(r["flow"]["sweep_ms"] for r in runs)
    kn_ms = sum(r["knudsen"]["sweep_ms"] for r in runs)
    fl_n = sum(r["flow"]["steps"] for r in runs)
    kn_n = sum(r["knudsen"]["steps"] for r in runs)
    if kn_ms >= fl_ms:
        name, per, bpu, ms = "k_sweep7<false, false, unsigned int>", kn_ms / kn_n, BYTES_D3Q7, kn_ms
    else:
        name, per, bpu, ms = ("k_sweep19<StoreF32, false, false, 0, false, unsigned int>", fl_ms / fl_n,
                              BYTES_D3Q19, fl_ms)
    achieved = nf * bpu / (per * 1e-3) / 1e9
    roof = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_gb(name, w["name"]), "traffic_unit": "GB per launch",
            "bytes_per_update": bpu, "n_fluid": nf, "ms_per_launch": per,
            "share_of_step": round(ms / (wall * 1e3), 4)}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "n": list(w["recon"]["n"]), "n_fluid": nf,
                   "tol": w["flow"]["tol"], "storage": "f32 (f - w_i)", "init": "zero"},
        "time_to_converged_s": round(ms_per_step / 1e3, 3),
        "flow": {k: last["flow"][k] for k in ("steps", "k_lattice", "k_m2", "k_mD", "residual",
                                              "mlups", "gbps")},
        "knudsen": {k: last["knudsen"][k] for k in ("steps", "Deff_lattice", "Deff_over_DKref",
                                                    "Deff_m2s", "tortuosity", "residual",
                                                    "flux_spread", "mlups", "gbps")},
        "geometry": {"porosity": last["label"]["porosity"],
                     "connectivity": last["label"]["connectivity"],
                     "n_spheres": last["recon"]["n_spheres"]},
        "stage_s": {k: round(v, 4) for k, v in last["t"].items()},
        "roofline": roof,
    }
    if not args.no_warm:
        from paper_1410_1921_amd import warmstart as WS
        log("warm-started pipeline")
        net = WS.load_network()
        pipeline(lbm, W, w, net)  # buffers and kernels warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wr = pipeline(lbm, W, w, net)
        torch.cuda.synchronize()
        tw = time.perf_counter() - t0
        out["warm_start"] = {
            "time_to_converged_s": round(tw, 3),
            "speedup": round(ms_per_step / 1e3 / tw, 3),
            "flow_steps": [last["flow"]["steps"], wr["flow"]["steps"]],
            "knudsen_steps": [last["knudsen"]["steps"], wr["knudsen"]["steps"]],
            "inference_s": round(wr["t"]["inference"], 4),
            "k_rel_diff": abs(wr["flow"]["k_lattice"] / last["flow"]["k_lattice"] - 1),
            "deff_rel_diff": abs(wr["knudsen"]["Deff_lattice"] / last["knudsen"]["Deff_lattice"] - 1),
            "network": "U-Net 16-128 ch, trained 25 epochs on 400 solves of 96^3 geometries",
            "applied_to": "Knudsen C (the flow starts from rest)"}
    if not args.no_batch:
        log("batch workload")
        out["batch"] = batch_throughput(lbm, W, args.batch_steps, args.batch_steps)
        out["batch"]["workload"] = W.BATCH["name"]
    log("D3Q19 mass-transport sweeps")
    out["diffusion_d3q19"] = diffusion19_sweeps(lbm, w, 2000)
    if not args.no_512:
        log("512^3 roofline")
        out["roofline_512"] = roofline_512(lbm, W, args.roofline_steps)
    log("copy ceiling")
    out["attainable_copy_gbs"] = copy_ceiling(lbm)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(W, w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
