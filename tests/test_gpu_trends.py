"""The paper's qualitative results (Section 4) reproduced on small reconstructions: means
over eight seeds of 48^3 reconstructions (sphere diameters in voxels, scaled down from
the paper's nanometres; 2 nm voxels, methane at 323 K, d_ref = 60 nm).

* Section 4.1: the connectivity of the void space rises with porosity (xi = 0.1).
* Section 4.2: the effective Knudsen diffusivity rises with porosity, with the mean pore
  diameter (xi = 0.1) and with the overlap tolerance.
* Section 4.3: the intrinsic permeability rises with porosity, mean pore diameter and
  overlap tolerance.

Flow and mass transport run on the transport voxels only (the paper's dead pores carry
no steady flux) to residual 1e-6.  A few low-porosity samples are held together by a
single narrow throat; their flow solve stops at the step limit with k near 0, which is
what it counts for in the mean.  Margins are set from a measured run: porosity
0.25/0.35/0.45 gives k x10 and x4.7, D_eff x8 and x3.2; mean diameter 5/8/12 voxels k
x1.26 and x1.30, D_eff x2.6 and x2.1; overlap tolerance 0.1/0.5/1.0 k x1.75 and x1.15,
D_eff x1.61 and x1.09.  Geometry and solves are deterministic, so are these figures.
"""
import sys

import numpy as np
import pytest

from paper_1410_1921_amd import lbm

pytestmark = pytest.mark.gpu
N = 48
SEEDS = tuple(range(1, 9))


def say(*a):
    print("[gpu-trends]", *a, flush=True)
    sys.stdout.flush()


def properties(eps, d_mean, xi, seed):
    pore, _, _ = lbm.lbm_reconstruct((N, N, N), eps, d_mean, d_mean / 4, 1.0, xi, 0.5, seed)
    _, transport, ls = lbm.lbm_label(pore)
    conn = ls["n_transport"] / ls["n_pore"]
    if ls["n_transport"] == 0:
        return conn, 0.0, 0.0
    diam = lbm.lbm_pore_diameter(pore, lbm.LBM_PSD_MIS)
    f = lbm.lbm_flow_solve(transport, tau=0.8, force=(1e-6, 0.0, 0.0), max_steps=200_000,
                           tol=1e-6)
    k = lbm.lbm_knudsen_solve(transport, diam, d_ref_nm=60.0, voxel_nm=2.0, T=323.0,
                              max_steps=4_000_000, tol=1e-6)
    assert k["converged"]
    assert f["converged"] or abs(f["k_lattice"]) < 1e-4
    return conn, f["k_lattice"], k["Deff_over_DKref"]


def sweep(points):
    means = []
    for eps, d_mean, xi in points:
        v = np.array([properties(eps, d_mean, xi, s) for s in SEEDS])
        means.append(v.mean(axis=0))
        say("eps", eps, "<d>", d_mean, "xi", xi, "connectivity, k, D_eff/D_K,ref", means[-1])
    return np.array(means)


def rising(values, factor):
    return all(b > factor * a for a, b in zip(values[:-1], values[1:]))


def test_porosity():
    m = sweep([(0.25, 8.0, 0.1), (0.35, 8.0, 0.1), (0.45, 8.0, 0.1)])
    assert rising(m[:, 0], 1.0)          # connectivity (Section 4.1)
    assert rising(m[:, 1], 2.0)          # permeability (Section 4.3)
    assert rising(m[:, 2], 2.0)          # effective diffusivity (Section 4.2)


def test_mean_pore_diameter():
    m = sweep([(0.35, 5.0, 0.1), (0.35, 8.0, 0.1), (0.35, 12.0, 0.1)])
    assert rising(m[:, 1], 1.1)
    assert rising(m[:, 2], 1.5)


def test_overlap_tolerance():
    m = sweep([(0.35, 8.0, 0.1), (0.35, 8.0, 0.5), (0.35, 8.0, 1.0)])
    assert rising(m[:, 1], 1.05)
    assert rising(m[:, 2], 1.05)
