"""Every sweep kernel variant (XCD-contiguous or plain workgroup order, ordinary or
streaming stores) computes the same state: bit-identical
fields, and k / D_eff equal up to the summation order of the FP64 check (1e-12)."""
import numpy as np
import pytest
import torch

from paper_1410_1921_amd import lbm
from paper_1410_1921_amd import workloads as W

pytestmark = pytest.mark.gpu

E = lbm.LBM_VARIANT_EXPLICIT
VARIANTS = [lbm.LBM_VARIANT_AUTO, E, E | lbm.LBM_VARIANT_REMAP, E | lbm.LBM_VARIANT_NTSTORE,
            E | lbm.LBM_VARIANT_REMAP | lbm.LBM_VARIANT_NTSTORE]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("shape,seed", [((13, 21, 10), 3), ((9, 5, 34), 4), ((2, 3, 17), 5)])
def test_flow_variants_agree(shape, seed):
    m = dev(W.blob_mask(shape, 0.55, seed))
    print("[variants] flow", shape, flush=True)
    runs = [lbm.lbm_flow_solve(m, tau=0.7, force=(1e-5, 2e-6, -1e-6), fixed_steps=250,
                               check_every=50, want_u=True, variant=v) for v in VARIANTS]
    for r in runs[1:]:
        assert torch.equal(r.field, runs[0].field)
        assert r["k_lattice"] == pytest.approx(runs[0]["k_lattice"], rel=1e-12)
        assert r["residual"] == pytest.approx(runs[0]["residual"], rel=1e-9)
    # and lbm_flow_step continues identically
    for r in runs:
        lbm.lbm_flow_step(r.workspace, 7)
    vox = np.flatnonzero(m.cpu().numpy().reshape(-1))[:50]
    ref = lbm.lbm_flow_sample(runs[0].workspace, vox)[0]
    for r in runs[1:]:
        assert np.array_equal(lbm.lbm_flow_sample(r.workspace, vox)[0], ref)


@pytest.mark.parametrize("shape,seed", [((19, 10, 14), 2), ((5, 7, 33), 8), ((3, 2, 9), 1)])
def test_knudsen_variants_agree(shape, seed):
    mk = W.blob_mask(shape, 0.6, seed)
    m = dev(mk)
    d = dev(W.hash_field(shape, seed, 1.0, 40.0).astype(np.float64) * mk)
    print("[variants] knudsen", shape, flush=True)
    runs = [lbm.lbm_knudsen_solve(m, d, d_ref_nm=30.0, voxel_nm=1.5, c_in=0.8, c_out=0.3,
                                  fixed_steps=300, check_every=50, want_c=True, variant=v)
            for v in VARIANTS]
    for r in runs[1:]:
        assert torch.equal(r.field, runs[0].field)
        assert r["Deff_lattice"] == pytest.approx(runs[0]["Deff_lattice"], rel=1e-12, abs=1e-300)
        assert np.allclose(r["plane_flux"], runs[0]["plane_flux"], rtol=1e-12, atol=1e-300)
