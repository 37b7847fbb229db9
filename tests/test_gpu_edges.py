"""Edge cases of the hot path on the GPU against the FP64 oracle.

* The largest edge the library takes (1024 voxels, coordinates packed in 10 bits) along
  each axis: geometry bit for bit, flow and mass transport element by element.
* A 1024^3 domain (the largest volume): reconstruction and labelling bit for bit; flow,
  D3Q19 and D3Q7 mass transport on sampled nodes after two steps from seeded random
  fields, with more than 2^32 population elements, so the sweeps run with 64-bit
  offsets.
* The 64-bit kernels forced on small lattices give the same bits as the 32-bit ones.
* Sizes beyond the limit are refused before any launch.
* Degenerate lattices: a single-voxel domain, a fluid voxel walled in on every side,
  fluid that reaches neither x face, and no fluid at all.
* Non-finite parameters are refused before any launch; a NaN in the starting field is
  reported as divergence by the first check.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1410_1921_amd import lbm
from paper_1410_1921_amd import workloads as W

pytestmark = pytest.mark.gpu
W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OFF64 = lbm.LBM_VARIANT_OFF64


def say(*a):
    print("[gpu-edges]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def recon(orc, rp):
    args = (rp["n"], rp["porosity"], rp["d_mean"], rp["d_std"], rp["d_min"], rp["overlap_tol"],
            rp["p_overlap"], rp["seed"])
    pore_g, sph_g, st_g = lbm.lbm_reconstruct(*args)
    pore_o, sph_o, st_o = orc.reconstruct(*args)
    assert np.array_equal(sph_g, sph_o)
    assert st_g["n_spheres"] == st_o["n_spheres"] and st_g["n_pore"] == st_o["n_pore"]
    return pore_g, pore_o, st_g


# ------------------------------------------------------------------ 1024 along one axis
@pytest.mark.parametrize("n", [(1024, 7, 6), (6, 1024, 7), (7, 6, 1024)], ids=["x", "y", "z"])
def test_edge_1024_each_axis(orc, n):
    rp = dict(n=n, porosity=0.4, d_mean=3.0, d_std=1.0, d_min=1.0, overlap_tol=0.5,
              p_overlap=0.5, seed=21)
    say("edge 1024", n)
    pore_g, pore_o, _ = recon(orc, rp)
    assert np.array_equal(pore_g.cpu().numpy(), pore_o)
    lab_g, tr_g, _ = lbm.lbm_label(pore_g)
    lab_o, tr_o, _ = orc.label18(pore_o)
    assert np.array_equal(lab_g.cpu().numpy(), lab_o)
    assert np.array_equal(tr_g.cpu().numpy(), tr_o)
    assert np.array_equal(lbm.lbm_pore_diameter(pore_g, lbm.LBM_PSD_CHORD13).cpu().numpy(),
                          orc.chords13(pore_o))
    d_g = lbm.lbm_pore_diameter(pore_g, lbm.LBM_PSD_MIS)
    d_o = orc.mis(pore_o)
    assert np.array_equal(d_g.cpu().numpy(), d_o)

    force = (1e-5, 2e-6, -3e-6)
    r = lbm.lbm_flow_solve(pore_g, tau=0.7, force=force, fixed_steps=200, check_every=50,
                           want_u=True)
    o = orc.flow_solve(pore_o, tau=0.7, force=force, fixed_steps=200, check_every=50)
    u = r.field.cpu().numpy().astype(np.float64)
    assert np.abs(u - o["u"]).max() <= 1e-5 * np.abs(o["u"]).max()
    assert np.allclose(r["mean_rho_u"], o["mean_rho_u"], rtol=1e-4, atol=1e-4 * 1e-5)

    tg = np.where(pore_o == 1, orc.tau_g(d_o, 20.0, 1.0), 1.0)
    k = lbm.lbm_knudsen_solve(pore_g, d_g, d_ref_nm=30.0, voxel_nm=1.5, c_in=0.9, c_out=0.2,
                              fixed_steps=300, check_every=50, want_c=True)
    ko = orc.knudsen_solve(pore_o, tg, 0.9, 0.2, fixed_steps=300, check_every=50)
    assert np.abs(k.field.cpu().numpy() - ko["c"]).max() < 1e-5
    assert k["phi_in"] == pytest.approx(ko["phi_in"], rel=1e-4, abs=1e-9)
    assert k["Deff_lattice"] == pytest.approx(ko["Deff_lattice"], rel=1e-4, abs=1e-9)
    say("edge 1024", n, "k", r["k_lattice"], "Deff", k["Deff_lattice"], ko["Deff_lattice"])


# ------------------------------------------------------------------ 64-bit offsets forced
@pytest.mark.parametrize("collision,storage,pressure", [
    ("BGK", lbm.LBM_STORE_FP32, False), ("MRT", lbm.LBM_STORE_FP32, False),
    ("TRT", lbm.LBM_STORE_FP32, False), ("BGK", lbm.LBM_STORE_FP16, False),
    ("BGK", lbm.LBM_STORE_FP64, False), ("BGK", lbm.LBM_STORE_FP32, True),
    ("TRT", lbm.LBM_STORE_FP64, True)])
def test_flow_off64_identical(collision, storage, pressure):
    g = dev(W.blob_mask((13, 21, 30), 0.55, 4))
    kw = dict(tau=0.7, force=(0, 0, 0) if pressure else (1e-5, 3e-6, 0), fixed_steps=150,
              check_every=50, want_u=True, storage=storage,
              collision=getattr(lbm, "LBM_COLLIDE_" + collision),
              pressure=(1.0001, 0.9999) if pressure else None)
    a = lbm.lbm_flow_solve(g, **kw)
    E = lbm.LBM_VARIANT_EXPLICIT
    for v in (OFF64, E | OFF64 | lbm.LBM_VARIANT_NTSTORE, E | OFF64 | lbm.LBM_VARIANT_REMAP):
        b = lbm.lbm_flow_solve(g, variant=v, **kw)
        assert torch.equal(a.field, b.field)
        assert a["k_lattice"] == b["k_lattice"]
    # stepping on and resuming a solve that runs the 64-bit kernels
    lbm.lbm_flow_step(b.workspace, 10)
    c = lbm.lbm_flow_solve(g, variant=OFF64, workspace=b.workspace, resume=True,
                           **{**kw, "fixed_steps": 40})
    d = lbm.lbm_flow_solve(g, **{**kw, "fixed_steps": 200})
    assert torch.equal(c.field, d.field)


@pytest.mark.parametrize("lattice", ["D3Q7", "D3Q19"])
def test_knudsen_off64_identical(lattice):
    m = W.blob_mask((21, 30, 40), 0.55, 12)
    d = W.hash_field(m.shape, 3, 2.0, 50.0).astype(np.float64) * m
    fm, fd = dev(m), dev(d)
    q = getattr(lbm, "LBM_LATTICE_" + lattice)
    kw = dict(fixed_steps=250, check_every=50, want_c=True, lattice=q)
    a = lbm.lbm_knudsen_solve(fm, fd, **kw)
    E = lbm.LBM_VARIANT_EXPLICIT
    for v in (OFF64, E | OFF64 | lbm.LBM_VARIANT_NTSTORE, E | OFF64 | lbm.LBM_VARIANT_REMAP):
        b = lbm.lbm_knudsen_solve(fm, fd, variant=v, **kw)
        assert torch.equal(a.field, b.field)
        assert a["Deff_lattice"] == b["Deff_lattice"]
        assert np.array_equal(a["plane_flux"], b["plane_flux"])


def test_batch_refuses_off64():
    m = [dev(W.blob_mask((8, 9, 10), 0.6, s)) for s in (1, 2)]
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_flow_solve_batch(m, fixed_steps=10, variant=OFF64)
    assert e.value.status == lbm.LBM_E_INVAL
    d = [torch.full(x.shape, 10.0, dtype=torch.float64, device="cuda") for x in m]
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_knudsen_solve_batch(m, d, fixed_steps=10, variant=OFF64)
    assert e.value.status == lbm.LBM_E_INVAL


# ------------------------------------------------------------------ beyond the limit
@pytest.mark.parametrize("shape", [(3, 4, 1025), (3, 1025, 4), (1025, 3, 4)])
def test_edge_beyond_limit_refused(shape):
    m = torch.ones(shape, dtype=torch.uint8, device="cuda")
    m[0, 0, 0] = 0
    d = torch.full(shape, 10.0, dtype=torch.float64, device="cuda")
    calls = [lambda: lbm.lbm_label(m),
             lambda: lbm.lbm_pore_diameter(m, lbm.LBM_PSD_CHORD13),
             lambda: lbm.lbm_pore_diameter(m, lbm.LBM_PSD_MIS),
             lambda: lbm.lbm_flow_solve(m, fixed_steps=1),
             lambda: lbm.lbm_knudsen_solve(m, d, fixed_steps=1),
             lambda: lbm.lbm_knudsen_solve(m, d, fixed_steps=1, lattice=lbm.LBM_LATTICE_D3Q19),
             lambda: lbm.lbm_reconstruct((shape[2], shape[1], shape[0]), 0.3, 3.0, 1.0)]
    for call in calls:
        with pytest.raises(lbm.LbmError) as e:
            call()
        assert e.value.status == lbm.LBM_E_INVAL


# ------------------------------------------------------------------ degenerate lattices
def test_single_voxel_domain(orc):
    m = np.ones((1, 1, 1), np.uint8)
    r = lbm.lbm_flow_solve(dev(m), tau=0.9, force=(1e-5, -2e-6, 3e-6), fixed_steps=60,
                           check_every=20, want_u=True)
    o = orc.flow_solve(m, tau=0.9, force=(1e-5, -2e-6, 3e-6), fixed_steps=60, check_every=20)
    # a node that is its own neighbour in every direction: uniform acceleration, F per
    # step (the reported velocity adds half a step's force)
    assert np.allclose(r.field.cpu().numpy(), o["u"], rtol=1e-5, atol=0)
    assert np.allclose(o["u"][:, 0, 0, 0], np.array([1e-5, -2e-6, 3e-6]) * 60, rtol=0.01)
    d = np.full(m.shape, 30.0)
    tg = orc.tau_g(d, 40.0, 1.0)  # d_ref = 60 nm / 1.5 nm
    for lattice, solve in ((lbm.LBM_LATTICE_D3Q7, orc.knudsen_solve),
                           (lbm.LBM_LATTICE_D3Q19, orc.diffusion19_solve)):
        k = lbm.lbm_knudsen_solve(dev(m), dev(d), d_ref_nm=60.0, voxel_nm=1.5, c_in=1.0, c_out=0.0,
                                  fixed_steps=200, check_every=50, want_c=True, lattice=lattice)
        ko = solve(m, tg, 1.0, 0.0, fixed_steps=200, check_every=50)
        assert np.abs(k.field.cpu().numpy() - ko["c"]).max() < 1e-6
        assert k["Deff_lattice"] == pytest.approx(ko["Deff_lattice"], rel=1e-4)


def test_walled_in_and_unreached_fluid(orc):
    # one fluid voxel walled in on every side, and a pocket that reaches neither x face
    m = np.zeros((6, 7, 9), np.uint8)
    m[1, 1, 1] = 1
    m[3:5, 2:6, 3:7] = 1
    force = (2e-5, 1e-5, 0.0)
    r = lbm.lbm_flow_solve(dev(m), tau=0.8, force=force, fixed_steps=300, check_every=50,
                           want_u=True)
    o = orc.flow_solve(m, tau=0.8, force=force, fixed_steps=300, check_every=50)
    u = r.field.cpu().numpy().astype(np.float64)
    assert np.abs(u - o["u"]).max() <= 1e-5 * np.abs(o["u"]).max()
    d = np.full(m.shape, 20.0) * m
    for lattice in (lbm.LBM_LATTICE_D3Q7, lbm.LBM_LATTICE_D3Q19):
        k = lbm.lbm_knudsen_solve(dev(m), dev(d), c_in=1.0, c_out=0.0, fixed_steps=200,
                                  check_every=50, want_c=True, lattice=lattice)
        # nothing enters: C stays 0 (up to the rounding of the stored frame), no flux, no
        # effective diffusivity
        assert k.field.abs().max().item() < 1e-6
        assert abs(k["Deff_lattice"]) < 1e-9 and abs(k["phi_in"]) < 1e-9
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_knudsen_solve(dev(np.zeros((4, 5, 6), np.uint8)), dev(np.zeros((4, 5, 6))),
                              fixed_steps=10)
    assert e.value.status == lbm.LBM_E_INVAL


# ------------------------------------------------------------------ 1024^3
BIG = dict(n=(1024, 1024, 1024), porosity=0.25, d_mean=16.0, d_std=4.0, d_min=1.0,
           overlap_tol=0.7, p_overlap=0.5, seed=5)


@pytest.fixture(scope="module")
def big(orc):
    say("reconstruct 1024^3")
    pore_g, pore_o, st = recon(orc, BIG)
    yield pore_g, pore_o, st
    del pore_g
    torch.cuda.empty_cache()


def _windows(shape, nodes, wrap_x):
    """Linear voxel indices of the 5^3 windows around `nodes` ([K, 5, 5, 5]); y and z
    wrap, x wraps (periodic flow) or is clamped (the caller keeps only in-range x)."""
    nz, ny, nx = shape
    z, y, x = np.unravel_index(nodes, shape)
    off = np.arange(-2, 3)
    zz = (z[:, None] + off) % nz
    yy = (y[:, None] + off) % ny
    xx = x[:, None] + off
    xx = xx % nx if wrap_x else np.clip(xx, 0, nx - 1)
    return (zz[:, :, None, None] * ny + yy[:, None, :, None]) * nx + xx[:, None, None, :]


def _pick(mask_at, nvox, shape, count, seed):
    """About `count` fluid voxels at random plus fluid voxels on the x faces; mask_at maps
    linear indices to mask values."""
    rng = np.random.default_rng(seed)
    cand = rng.choice(nvox, size=8 * count, replace=False)
    nz, ny, nx = shape
    yz = rng.integers(0, ny * nz, size=4 * 64)
    faces = np.concatenate([yz[:128] * nx, yz[128:] * nx + nx - 1])
    cand = np.concatenate([cand, faces])
    keep = cand[mask_at(cand) == 1]
    return np.unique(np.concatenate([keep[:count], keep[np.isin(keep, faces)]]))


def test_max_volume_1024_geometry(orc, big):
    pore_g, pore_o, st = big
    assert torch.equal(pore_g, dev(pore_o))
    say("label 1024^3")
    lab_g, tr_g, ls_g = lbm.lbm_label(pore_g)
    lab_o, tr_o, ls_o = orc.label18(pore_o)
    assert torch.equal(lab_g, dev(lab_o))
    assert torch.equal(tr_g, dev(tr_o))
    assert (ls_g["n_pore"], ls_g["n_transport"], ls_g["n_components"]) == \
        (ls_o["n_pore"], ls_o["n_transport"], ls_o["n_components"])
    del lab_g, tr_g, lab_o, tr_o
    torch.cuda.empty_cache()


def test_max_volume_1024_flow_sampled(orc, big):
    pore_g, pore_o, st = big
    nf = st["n_pore"]
    assert 19 * ((nf + 63) // 64 * 64) > 2 ** 32  # the 64-bit population offsets
    shape = pore_o.shape
    gen = torch.Generator(device="cuda").manual_seed(17)
    u0 = torch.rand((3,) + shape, generator=gen, device="cuda", dtype=torch.float32)
    u0.mul_(4e-3).sub_(2e-3)
    tau, force = 0.8, (2e-5, -1e-5, 5e-6)
    say("flow 1024^3", nf, "nodes")
    r = lbm.lbm_flow_solve(pore_g, tau=tau, force=force, fixed_steps=2, check_every=100,
                           u_init=u0, n_fluid=nf)
    nodes = _pick(lambda v: pore_o.reshape(-1)[v], pore_o.size, shape, 600, 3)
    f_g, flag = lbm.lbm_flow_sample(r.workspace, nodes)
    assert flag.all()
    win = _windows(shape, nodes, True)
    uw_all = u0.view(3, -1)[:, torch.from_numpy(win.reshape(-1)).cuda()].cpu().numpy()
    uw_all = uw_all.reshape(3, len(nodes), 5, 5, 5).astype(np.float64)
    del r, u0
    torch.cuda.empty_cache()
    worst = scale = 0.0
    for k in range(len(nodes)):
        mw = np.ascontiguousarray(pore_o.reshape(-1)[win[k]])
        f = orc.flow_init(mw, np.ascontiguousarray(uw_all[:, k]))
        orc.flow_solve(mw, tau=tau, force=force, fixed_steps=2, f=f, want_u=False)
        ref = f[2, 2, 2] - W19
        worst = max(worst, np.abs(f_g[k] - ref).max())
        scale = max(scale, np.abs(ref).max())
    say("flow 1024^3 sampled", len(nodes), "worst", worst, "scale", scale)
    assert worst <= 2e-6 * scale


def _transport_sampled(orc, fluid_g, mask_at, shape, lattice, seed, count):
    """Two steps from seeded random C and pore sizes; sampled populations against the
    oracle's solve on the window (x clamped at the faces)."""
    q = 19 if lattice == lbm.LBM_LATTICE_D3Q19 else 7
    nf = lbm.lbm_count(fluid_g)
    assert q * ((nf + 63) // 64 * 64) > 2 ** 32  # the 64-bit population offsets
    gen = torch.Generator(device="cuda").manual_seed(seed)
    c0 = torch.rand(shape, generator=gen, device="cuda", dtype=torch.float32)
    diam = torch.rand(shape, generator=gen, device="cuda", dtype=torch.float64)
    diam.mul_(39.5).add_(0.5)
    dref = 60.0 / 2.0
    say("transport 1024^3 q", q, nf, "nodes")
    r = lbm.lbm_knudsen_solve(fluid_g, diam, d_ref_nm=60.0, voxel_nm=2.0, c_in=1.0, c_out=0.0,
                              fixed_steps=2, check_every=100, c_init=c0, n_fluid=nf,
                              want_planes=False, lattice=lattice)
    nodes = _pick(mask_at, int(np.prod(shape)), shape, count, seed)
    g_g, tau_g, flag = lbm.lbm_knudsen_sample(r.workspace, nodes)
    assert flag.all()
    win = _windows(shape, nodes, False)
    idx = torch.from_numpy(win.reshape(-1)).cuda()
    cw_all = c0.view(-1)[idx].cpu().numpy().reshape(len(nodes), 5, 5, 5).astype(np.float64)
    dw_all = diam.view(-1)[idx].cpu().numpy().reshape(len(nodes), 5, 5, 5)
    mw_all = mask_at(win.reshape(-1)).reshape(len(nodes), 5, 5, 5)
    del r, c0, diam
    torch.cuda.empty_cache()
    init, solve = ((orc.diffusion19_init, orc.diffusion19_solve) if q == 19 else
                   (orc.knudsen_init, orc.knudsen_solve))
    nz, ny, nx = shape
    worst = 0.0
    for k, v in enumerate(nodes):
        x = v % nx
        xs = np.arange(x - 2, x + 3)
        keep = (xs >= 0) & (xs < nx)  # the window stops at the faces
        mw = np.ascontiguousarray(mw_all[k][:, :, keep])
        cw = np.ascontiguousarray(cw_all[k][:, :, keep])
        tw = np.where(mw == 1, orc.tau_g(dw_all[k][:, :, keep], dref, 1.0), 1.0)
        g = init(mw, cw)
        solve(mw, tw, 1.0, 0.0, fixed_steps=2, g=g, want_c=False, want_planes=False)
        ref = g[2, 2, int(np.flatnonzero(xs[keep] == x)[0])]
        worst = max(worst, np.abs(g_g[k][:q] - ref).max())
        assert tau_g[k] == pytest.approx(orc.tau_g(dw_all[k][2, 2, 2], dref, 1.0), rel=1e-6)
    say("transport 1024^3 q", q, "sampled", len(nodes), "worst", worst)
    assert worst <= 1e-6


def test_max_volume_1024_diffusion19_sampled(orc, big):
    pore_g, pore_o, _ = big
    _transport_sampled(orc, pore_g, lambda v: pore_o.reshape(-1)[v], pore_o.shape,
                       lbm.LBM_LATTICE_D3Q19, 23, 500)


def test_max_volume_1024_knudsen_d3q7_sampled(orc):
    # D3Q7 needs more than 2^32 / 7 fluid nodes for the 64-bit offsets: a seeded random
    # mask of porosity 0.62 (666 million nodes)
    shape = (1024, 1024, 1024)
    gen = torch.Generator(device="cuda").manual_seed(29)
    m = (torch.rand(shape, generator=gen, device="cuda") < 0.62).to(torch.uint8)
    flat = m.view(-1)

    def mask_at(v):
        return flat[torch.from_numpy(np.ascontiguousarray(v, np.int64)).cuda()].cpu().numpy()

    _transport_sampled(orc, m, mask_at, shape, lbm.LBM_LATTICE_D3Q7, 31, 600)
    del m, flat
    torch.cuda.empty_cache()


def test_binding_refuses_mismatched_shapes():
    # the C ABI takes bare pointers: the binding checks that companion arrays cover the
    # grid before any call reaches the library
    from paper_1410_1921_amd import nn
    from paper_1410_1921_amd.nn import View
    m = dev(W.blob_mask((8, 9, 10), 0.6, 3))
    with pytest.raises(ValueError):
        lbm.lbm_knudsen_solve(m, torch.ones((8, 9, 9), dtype=torch.float64, device="cuda"),
                              fixed_steps=10)
    with pytest.raises(ValueError):
        lbm.lbm_knudsen_solve(m, torch.ones((8, 9, 10), dtype=torch.float64, device="cuda"),
                              fixed_steps=10, c_init=torch.zeros((8, 9, 9), device="cuda"))
    with pytest.raises(ValueError):
        lbm.lbm_flow_solve(m, fixed_steps=10, u_init=torch.zeros((3, 8, 9, 9), device="cuda"))
    shape = (16, 16, 16)
    x = View(torch.zeros((16 * 16 * 16, 16), dtype=torch.bfloat16, device="cuda"))
    y_small = View(torch.zeros((16 * 16 * 8, 16), dtype=torch.bfloat16, device="cuda"))
    w = torch.zeros(27 * 16 * 16, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(ValueError):
        nn.lbm_nn_conv3d(shape, x, 16, w, None, y_small, 16, 0)
    with pytest.raises(ValueError):
        nn.lbm_nn_conv3d(shape, x, 16, w[:-1], None, x, 16, 0)
    with pytest.raises(ValueError):
        nn.lbm_nn_pool2(shape, 16, x, x)


def small_problem():
    m = W.blob_mask((16, 16, 16), 0.5, 3)
    return m, np.where(m > 0, 4.0, 0.0)


@pytest.mark.parametrize("bad", [dict(c_in=float("nan")), dict(c_out=float("inf")),
                                 dict(tau_ref=float("inf")), dict(d_ref_nm=float("inf")),
                                 dict(voxel_nm=float("nan"))])
def test_knudsen_non_finite_parameters_refused(bad):
    m, d = small_problem()
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_knudsen_solve(dev(m), dev(d), fixed_steps=10, **bad)
    assert e.value.status == lbm.LBM_E_INVAL


@pytest.mark.parametrize("bad", [dict(force=(float("nan"), 0.0, 0.0)),
                                 dict(force=(1e-6, float("inf"), 0.0)),
                                 dict(voxel_nm=0.0), dict(voxel_nm=float("inf"))])
def test_flow_non_finite_parameters_refused(bad):
    m, _ = small_problem()
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_flow_solve(dev(m), fixed_steps=10, **bad)
    assert e.value.status == lbm.LBM_E_INVAL


@pytest.mark.parametrize("lattice", ["D3Q7", "D3Q19"])
def test_knudsen_nan_start_reported_as_diverged(lattice):
    # a NaN in the initial concentration reaches the first check's sums, which report it;
    # a later solve of the same problem is unaffected
    lat = getattr(lbm, "LBM_LATTICE_" + lattice)
    m, d = small_problem()
    c0 = np.zeros(m.shape, np.float32)
    fl = np.flatnonzero(m)
    c0.flat[fl[len(fl) // 2]] = np.nan
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_knudsen_solve(dev(m), dev(d), max_steps=1000, check_every=100, c_init=dev(c0),
                              lattice=lat)
    assert e.value.status == lbm.LBM_E_DIVERGED
    r = lbm.lbm_knudsen_solve(dev(m), dev(d), fixed_steps=200, check_every=100, lattice=lat)
    say(lattice, "after a diverged solve: D_eff", r["Deff_lattice"], "steps", r["steps"])
    assert np.isfinite(r["Deff_lattice"]) and r["steps"] == 200
