"""Writes the stored oracle results that the full-size parity tests compare with.

Calls only the FP64 CPU oracle (``oracle/``) and the seeded workload parameters
(``paper_1410_1921_amd/workloads.py``, which holds no step of the method).  Run from the
repository root:

    python tests/golden/make_oracle_golden.py c2     # 128^3 methane workload
    python tests/golden/make_oracle_golden.py crop   # 128^3 centre crop of the 512^3 one

Each writes ``tests/golden/oracle_<name>.json``: the result scalars at the stated step
counts, the link-plane fluxes, and the fields at 1024 seeded fluid voxels (plus 64 solid
ones), so that a GPU test can compare element by element without running the oracle; the
crop record also holds the hash of the oracle's 512^3 maximum-inscribed-sphere map.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as orc  # noqa: E402
from paper_1410_1921_amd import workloads as W  # noqa: E402


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sample_voxels(pore, seed, n_fluid=1024, n_solid=64):
    """Linear indices of seeded fluid and solid voxels (sorted)."""
    rng = np.random.default_rng(seed)
    flat = pore.reshape(-1)
    fl = np.flatnonzero(flat == 1)
    so = np.flatnonzero(flat == 0)
    pick = np.concatenate([rng.choice(fl, min(n_fluid, fl.size), replace=False),
                           rng.choice(so, min(n_solid, so.size), replace=False)])
    return np.sort(pick)


def flow_record(pore, vox, **kw):
    t0 = time.perf_counter()
    r = orc.flow_solve(pore, tau=0.8, force=(1e-6, 0.0, 0.0), check_every=100, **kw)
    u = r["u"].reshape(3, -1)[:, vox].T
    log(f"flow {kw}: {r['steps']} steps, k {r['k_lattice']:.9e}, {time.perf_counter() - t0:.0f} s")
    return {"steps": r["steps"], "k_lattice": r["k_lattice"], "residual": r["residual"],
            "converged": r["converged"], "mean_rho_u": list(r["mean_rho_u"]),
            "mass_dev": r["mass_dev"], "max_abs_u": float(np.abs(r["u"]).max()),
            "u": u.tolist()}


def mask_hash(pore):
    return hashlib.sha256(np.ascontiguousarray(pore, np.uint8).tobytes()).hexdigest()


def c2():
    w = W.METHANE_128
    rp, kp = w["recon"], w["knudsen"]
    pore, _, info = orc.reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                    rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    vox = sample_voxels(pore, 128)
    out = {"workload": w["name"], "mask_sha256": mask_hash(pore), "n_pore": info["n_pore"],
           "threads": orc.num_threads(), "vox": vox.tolist()}
    out["flow_2000"] = flow_record(pore, vox, fixed_steps=2000)
    # the oracle's own stop rule: first check with residual < 1e-7
    out["flow_converged"] = flow_record(pore, vox, max_steps=400_000, tol=1e-7)
    d = orc.mis(pore)
    tg = np.where(pore == 1, orc.tau_g(d, kp["d_ref_nm"] / w["voxel_nm"], kp["tau_ref"]), 1.0)
    steps = 100_000
    t0 = time.perf_counter()
    r = orc.knudsen_solve(pore, tg, kp["c_in"], kp["c_out"], fixed_steps=steps, check_every=100)
    log(f"knudsen {steps} steps: D_eff {r['Deff_lattice']:.9e}, {time.perf_counter() - t0:.0f} s")
    out["knudsen_100000"] = {
        "steps": r["steps"], "Deff_lattice": r["Deff_lattice"], "residual": r["residual"],
        "phi_in": r["phi_in"], "phi_out": r["phi_out"], "sum_c": r["sum_c"],
        "plane_flux": r["plane_flux"].tolist(), "c": r["c"].reshape(-1)[vox].tolist()}
    return out


def crop():
    w = W.LARGE_512
    rp = w["recon"]
    pore, _, info = orc.reconstruct(rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"],
                                    rp["d_min"], rp["overlap_tol"], rp["p_overlap"], rp["seed"])
    (z0, z1), (y0, y1), (x0, x1) = w["crop"]
    sub = np.ascontiguousarray(pore[z0:z1, y0:y1, x0:x1])
    log(f"512^3 reconstruction: {info}; crop fluid {int(sub.sum())}")
    vox = sample_voxels(sub, 512)
    out = {"workload": w["name"], "crop": [list(c) for c in w["crop"]],
           "mask_sha256_full": mask_hash(pore), "mask_sha256": mask_hash(sub),
           "n_pore": int(sub.sum()), "threads": orc.num_threads(), "vox": vox.tolist()}
    # the maximum-inscribed-sphere map of the whole 512^3 reconstruction (the map the
    # 512^3, batch and warm-start workloads read), as the hash of its binary64 values
    t0 = time.perf_counter()
    d = orc.mis(pore)
    out["mis_sha256_full"] = hashlib.sha256(np.ascontiguousarray(d, np.float64).tobytes()).hexdigest()
    log(f"512^3 MIS map: {time.perf_counter() - t0:.0f} s")
    del pore, d
    # the crop converges slowly (residual 1e-6 after ~60 000 steps): the oracle pins the
    # GPU paths at a fixed count; converged errors take the GPU binary64 path as reference
    out["flow_20000"] = flow_record(sub, vox, fixed_steps=20_000)
    return out


if __name__ == "__main__":
    which = sys.argv[1]
    rec = {"c2": c2, "crop": crop}[which]()
    path = os.path.join(HERE, f"oracle_{which}.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, separators=(",", ":"))
    log("wrote", path)
