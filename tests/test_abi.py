"""The C-ABI library loads, exports every entry point that include/lbm.h declares, and its
host-only paths (struct layouts, workspace sizing, argument checks, properties) behave
as documented.  No GPU needed: nothing here launches a kernel."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1410_1921_amd import lbm
    return lbm


def _declared(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    L = lib.load()
    names = _declared() + _declared(os.path.join(ROOT, "include", "lbm_nn.h"))
    assert len(names) == 21 + 15
    for name in names:
        assert hasattr(L, name), name
    # and the binding wraps each of them
    for name in names:
        assert name in lib._SIGS, name


def test_struct_layouts_match(lib):
    for i, cls in enumerate(lib.STRUCTS):
        assert lib.lbm_sizeof(i) == C.sizeof(cls), cls.__name__
    assert lib.lbm_sizeof(99) == 0
    assert len(lib.STRUCTS) == 10


def test_version(lib):
    assert "gfx950" in lib.lbm_version()


def test_workspace_sizes(lib):
    s_small = lib.lbm_workspace_size(lib.LBM_WS_FLOW, (32, 32, 32), 1000)
    s_big = lib.lbm_workspace_size(lib.LBM_WS_FLOW, (32, 32, 32), 20000)
    # two population buffers of 19 binary32 values per extra node, at least
    assert s_big - s_small >= 2 * 19 * 4 * 19000
    # n_fluid < 0 sizes for every voxel
    assert lib.lbm_workspace_size(lib.LBM_WS_FLOW, (32, 32, 32), -1) >= \
        lib.lbm_workspace_size(lib.LBM_WS_FLOW, (32, 32, 32), 32 ** 3)
    # binary16 / binary64 storage: 2 and 8 bytes per population (binary16 adds the
    # two binary32 writer-density arrays)
    s16 = [lib.lbm_workspace_size(lib.LBM_WS_FLOW_FP16, (32, 32, 32), m) for m in (1000, 20000)]
    s64 = [lib.lbm_workspace_size(lib.LBM_WS_FLOW_FP64, (32, 32, 32), m) for m in (1000, 20000)]
    assert s16[1] - s16[0] >= 2 * (19 * 2 + 4) * 19000
    assert s16[1] - s16[0] < s_big - s_small < s64[1] - s64[0]
    assert s64[1] - s64[0] >= 2 * 19 * 8 * 19000
    assert lib.lbm_workspace_size(lib.LBM_WS_KNUDSEN, (16, 16, 16), 100) > 0
    k7 = [lib.lbm_workspace_size(lib.LBM_WS_KNUDSEN, (32, 32, 32), m) for m in (1000, 20000)]
    k19 = [lib.lbm_workspace_size(lib.LBM_WS_KNUDSEN_D3Q19, (32, 32, 32), m) for m in (1000, 20000)]
    assert k19[1] - k19[0] - (k7[1] - k7[0]) >= 2 * 12 * 4 * 19000  # 12 more populations
    assert lib.lbm_workspace_size(lib.LBM_WS_LABEL, (16, 16, 16)) >= 2 * 16 ** 3
    assert lib.lbm_workspace_size(lib.LBM_WS_PORE_DIAM, (16, 16, 16)) >= 12 * 16 ** 3
    with pytest.raises(lib.LbmError) as e:
        lib.lbm_workspace_size(7, (8, 8, 8))
    assert e.value.status == lib.LBM_E_INVAL
    with pytest.raises(lib.LbmError):
        lib.lbm_workspace_size(lib.LBM_WS_FLOW, (2000, 8, 8))
    with pytest.raises(lib.LbmError):
        lib.lbm_workspace_size(lib.LBM_WS_FLOW, (8, 8, 8), 10_000)


def test_workspace_sizes_at_the_largest_volume(lib):
    # 1024^3, every voxel fluid: 2^30 nodes, population arrays far beyond 2^32 elements;
    # the sizes come out in 64-bit arithmetic, at least the population bytes, and grow
    # with the storage width
    n = (1024, 1024, 1024)
    nf = 1024 ** 3
    per_node = {lib.LBM_WS_FLOW: 2 * 19 * 4, lib.LBM_WS_FLOW_FP16: 2 * (19 * 2 + 4),
                lib.LBM_WS_FLOW_FP64: 2 * 19 * 8, lib.LBM_WS_KNUDSEN: 2 * 7 * 4,
                lib.LBM_WS_KNUDSEN_D3Q19: 2 * 19 * 4}
    for kind, b in per_node.items():
        size = lib.lbm_workspace_size(kind, n, nf)
        assert b * nf <= size < (b + 64) * nf, kind
    assert lib.lbm_workspace_size(lib.LBM_WS_FLOW_FP64, n, nf) > 2 ** 38
    assert lib.lbm_workspace_size(lib.LBM_WS_LABEL, n) >= 2 * nf
    assert lib.lbm_workspace_size(lib.LBM_WS_PORE_DIAM, n) >= 12 * nf


def test_argument_checks_before_device(lib):
    L = lib.load()
    n = (C.c_int32 * 3)(8, 8, 8)
    dummy = C.c_void_p(1)
    # tau <= 1/2 is rejected before anything touches a device
    p = lib.lbm_flow_params(0.5, (C.c_double * 3)(1e-6, 0, 0), 10, 0, 10, 0, 1e-7, 1.0, 0, 0)
    r = lib.lbm_flow_result()
    assert L.lbm_flow_solve(n, dummy, C.byref(p), C.byref(r), None, None, dummy, 1 << 20,
                            None) == lib.LBM_E_INVAL
    assert "tau" in L.lbm_last_error().decode()
    p = lib.lbm_flow_params(0.8, (C.c_double * 3)(1e-6, 0, 0), 10, 0, 0, 0, 1e-7, 1.0, 0, 0)
    assert L.lbm_flow_solve(n, dummy, C.byref(p), C.byref(r), None, None, dummy, 1 << 20,
                            None) == lib.LBM_E_INVAL
    kp = lib.lbm_knudsen_params(1.0, 60.0, 1.5, 1.0, 1.0, 323.0, 0.016, 10, 0, 10, 0, 1e-7, 0, 0)
    kr = lib.lbm_knudsen_result()
    assert L.lbm_knudsen_solve(n, dummy, dummy, C.byref(kp), C.byref(kr), None, None, None,
                               dummy, 1 << 20, None) == lib.LBM_E_INVAL
    for bad_lattice in (2, -1, 19):
        kp = lib.lbm_knudsen_params(1.0, 60.0, 1.5, 1.0, 0.0, 323.0, 0.016, 10, 0, 10, 0, 1e-7, 0,
                                    bad_lattice)
        assert L.lbm_knudsen_solve(n, dummy, dummy, C.byref(kp), C.byref(kr), None, None, None,
                                   dummy, 1 << 20, None) == lib.LBM_E_INVAL
        assert "lattice" in L.lbm_last_error().decode()
    rp = lib.lbm_recon_params((C.c_int32 * 3)(8, 8, 8), 1.5, 4.0, 1.0, 1.0, 0.5, 0.5, 1, 0)
    rs = lib.lbm_recon_stats()
    assert L.lbm_reconstruct(C.byref(rp), dummy, None, 0, C.byref(rs), None) == lib.LBM_E_INVAL
    assert L.lbm_label(n, None, None, None, None, None, 0, None) == lib.LBM_E_INVAL
    assert L.lbm_pore_diameter(n, dummy, 5, dummy, dummy, 1 << 20, None) == lib.LBM_E_INVAL
    nbad = (C.c_int32 * 3)(0, 8, 8)
    assert L.lbm_pore_diameter(nbad, dummy, 0, dummy, dummy, 1 << 20, None) == lib.LBM_E_INVAL
    # unknown storage, with_rho and collision values are rejected
    for storage, wr, col in ((3, 0, 0), (-1, 0, 0), (0, 2, 0), (0, 0, 3), (0, 0, -1)):
        p = lib.lbm_flow_params(0.8, (C.c_double * 3)(1e-6, 0, 0), 10, 0, 10, storage, 1e-7, 1.0,
                                0, 0, wr, col)
        assert L.lbm_flow_solve(n, dummy, C.byref(p), C.byref(r), None, None, dummy, 1 << 20,
                                None) == lib.LBM_E_INVAL
    # unknown boundaries, pressure boundaries with binary16 storage, non-positive
    # densities or no driving
    for storage, bc, rin, rout in ((0, 2, 1.0, 1.0), (1, 1, 1.01, 1.0), (0, 1, 0.0, 1.0),
                                   (0, 1, 1.0, 1.0)):
        p = lib.lbm_flow_params(0.8, (C.c_double * 3)(0, 0, 0), 10, 0, 10, storage, 1e-7, 1.0,
                                0, 0, 0, 0, bc, 0, rin, rout)
        assert L.lbm_flow_solve(n, dummy, C.byref(p), C.byref(r), None, None, dummy, 1 << 20,
                                None) == lib.LBM_E_INVAL
    # variant bits other than EXPLICIT | REMAP | NTSTORE are rejected by both solves
    for bad in (2, 16, 1 << 20, -1):
        p = lib.lbm_flow_params(0.8, (C.c_double * 3)(1e-6, 0, 0), 10, 0, 10, 0, 1e-7, 1.0, 0, bad)
        assert L.lbm_flow_solve(n, dummy, C.byref(p), C.byref(r), None, None, dummy, 1 << 20,
                                None) == lib.LBM_E_INVAL
        assert "variant" in L.lbm_last_error().decode()
        kp = lib.lbm_knudsen_params(1.0, 60.0, 1.5, 1.0, 0.0, 323.0, 0.016, 10, 0, 10, 0, 1e-7,
                                    bad, 0)
        assert L.lbm_knudsen_solve(n, dummy, dummy, C.byref(kp), C.byref(kr), None, None, None,
                                   dummy, 1 << 20, None) == lib.LBM_E_INVAL
        assert "variant" in L.lbm_last_error().decode()


def test_props_relations(lib, orc):
    g = dict(n_pore=400, n_transport=380, n_components=2, porosity=0.4, connectivity=0.95)
    f = dict(steps=100, n_fluid=400, converged=1, reserved=0, k_lattice=0.1, k_m2=2.25e-19,
             k_mD=2.25e-19 / 9.869233e-16, residual=1e-8, mean_rho_u=[1e-6, 0, 0], mass_dev=0.0,
             sweep_ms=1.0, mlups=1.0, gbps=1.0)
    dk = orc.knudsen_diffusivity(60e-9, 323.0)
    k = dict(steps=100, n_fluid=400, converged=1, reserved=0, Deff_lattice=0.0125,
             Deff_over_DKref=0.1, Deff_m2s=0.1 * dk, DK_ref_m2s=dk, tortuosity=4.0,
             tortuosity_local=3.0, phi_in=1.0, phi_out=1.0, flux_spread=0.0, residual=1e-8,
             sum_c=1.0, sweep_ms=1.0, mlups=1.0, gbps=1.0)
    out = lib.lbm_props(g, f, k, d_mean_nm=45.0, P=17236893.0, T=323.0, mu=1.73e-5)
    assert out["k_KC_m2"] == pytest.approx(orc.k_kozeny_carman(45e-9, 0.4), rel=1e-14)
    assert out["fc_dgm"] == pytest.approx(orc.fc_dgm(0.1 * dk, 1.73e-5, 2.25e-19, 17236893.0),
                                          rel=1e-14)
    assert out["k_apparent_m2"] == pytest.approx(2.25e-19 * out["fc_dgm"], rel=1e-14)
    assert out["mean_free_path_m"] == pytest.approx(orc.mean_free_path(1.73e-5, 17236893.0, 323.0),
                                                    rel=1e-14)
    assert out["bruggeman_alpha"] == pytest.approx(orc.bruggeman_alpha(0.1, 0.4), rel=1e-14)
    assert out["tortuosity"] == 4.0 and out["Deff_m2s"] == pytest.approx(0.1 * dk, rel=1e-15)
    partial = lib.lbm_props(g, None, None)
    assert math.isnan(partial["k_m2"]) and partial["porosity"] == 0.4


def test_batch_sizes_and_checks(lib):
    L = lib.load()
    one = lib.lbm_flow_batch_workspace([(32, 32, 32)], [1000])
    two = lib.lbm_flow_batch_workspace([(32, 32, 32), (16, 24, 40)], [1000, 3000])
    # at least the two binary32 population buffers of every block-aligned list
    assert one >= 2 * 19 * 4 * 1024
    assert two - one >= 2 * 19 * 4 * 3072
    assert lib.lbm_flow_batch_workspace([(8, 8, 2000)], [10]) == 0
    assert lib.lbm_flow_batch_workspace([(8, 8, 8)], [-1]) == 0
    n = (C.c_int32 * 6)(8, 8, 8, 8, 8, 8)
    nf = (C.c_int64 * 2)(100, 100)
    masks = (C.c_void_p * 2)(1, 1)
    res = (lib.lbm_flow_result * 2)()
    dummy = C.c_void_p(1)

    def call(count=2, **kw):
        a = dict(tau=0.8, force=(1e-6, 0, 0), max_steps=10, fixed_steps=0, check_every=10,
                 storage=0, tol=1e-7, voxel_nm=1.0, resume=0, variant=0, with_rho=0, collision=0,
                 boundary=0)
        a.update(kw)
        p = lib.lbm_flow_params(a["tau"], (C.c_double * 3)(*a["force"]), a["max_steps"],
                                a["fixed_steps"], a["check_every"], a["storage"], a["tol"],
                                a["voxel_nm"], a["resume"], a["variant"], a["with_rho"],
                                a["collision"], a["boundary"], 0, 1.01, 1.0)
        return L.lbm_flow_solve_batch(count, n, masks, nf, C.byref(p), None, res, None, dummy,
                                      1 << 30, None)

    # binary16 / binary64 storage, resume, density planes, F_x = 0, tau <= 1/2, unknown
    # variant bits and an empty batch are rejected before any device work
    for kw in (dict(storage=1), dict(storage=2), dict(resume=1), dict(with_rho=1),
               dict(boundary=1),
               dict(force=(0, 1e-6, 0)), dict(tau=0.5), dict(variant=2), dict(collision=3),
               dict(count=0)):
        assert call(**kw) == lib.LBM_E_INVAL, kw


def test_knudsen_batch_sizes_and_checks(lib):
    L = lib.load()
    one = lib.lbm_knudsen_batch_workspace([(32, 32, 32)], [1000])
    two = lib.lbm_knudsen_batch_workspace([(32, 32, 32), (16, 24, 40)], [1000, 3000])
    assert one >= 2 * 7 * 4 * 1024
    assert two - one >= 2 * 7 * 4 * 3072
    assert lib.lbm_knudsen_batch_workspace([(8, 8, 2000)], [10]) == 0
    n = (C.c_int32 * 6)(8, 8, 8, 8, 8, 8)
    nf = (C.c_int64 * 2)(100, 100)
    ptrs = (C.c_void_p * 2)(1, 1)
    res = (lib.lbm_knudsen_result * 2)()

    def call(count=2, **kw):
        a = dict(tau_ref=1.0, c_in=1.0, c_out=0.0, resume=0, variant=0, check_every=10,
                 lattice=0)
        a.update(kw)
        p = lib.lbm_knudsen_params(a["tau_ref"], 60.0, 1.5, a["c_in"], a["c_out"], 323.0, 0.016,
                                   10, 0, a["check_every"], a["resume"], 1e-7, a["variant"],
                                   a["lattice"])
        return L.lbm_knudsen_solve_batch(count, n, ptrs, ptrs, nf, C.byref(p), None, res, None,
                                         None, C.c_void_p(1), 1 << 30, None)

    for kw in (dict(resume=1), dict(c_out=1.0), dict(tau_ref=0.5), dict(variant=2),
               dict(check_every=0), dict(count=0), dict(lattice=1)):
        assert call(**kw) == lib.LBM_E_INVAL, kw
