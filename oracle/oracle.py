"""ctypes wrapper of the FP64 C oracle (test infrastructure; see the package docstring).

Arrays follow the voxel convention of the oracle: a volume is a C-ordered numpy array of
shape (nz, ny, nx), so the linear index is x + nx*(y + ny*z).  Populations are
node-major, shape (nz, ny, nx, q).  Vector fields are planar, shape (3, nz, ny, nx).
"""
import ctypes as C
import os

import numpy as np

from . import build_oracle

_lib = None

_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")

OK, W_NOT_CONVERGED, E_INVAL, E_NOMEM, E_STALL, E_DIVERGED = 0, 1, -1, -2, -4, -5


class OracleError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def _nullable(ptype):
    """An ndpointer type that also accepts None."""

    class _P(ptype):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return super().from_param(obj)

    return _P


def lib():
    global _lib
    if _lib is not None:
        return _lib
    path = build_oracle.LIB
    src = build_oracle.SRC
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
        build_oracle.build()
    L = C.CDLL(path)
    L.orc_splitmix64_next.argtypes = [C.POINTER(C.c_uint64)]
    L.orc_splitmix64_next.restype = C.c_uint64
    L.orc_uniform.argtypes = [C.POINTER(C.c_uint64)]
    L.orc_uniform.restype = C.c_double
    L.orc_normal.argtypes = [C.POINTER(C.c_uint64)]
    L.orc_normal.restype = C.c_double
    L.orc_sphere_volume.argtypes = [C.c_double]
    L.orc_sphere_volume.restype = C.c_double
    L.orc_lens_volume.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_lens_volume.restype = C.c_double
    L.orc_reconstruct.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_uint64, C.c_int64,
                                  _u8p, _nullable(_i64p), C.c_int64, _i64p]
    L.orc_reconstruct.restype = C.c_int
    L.orc_label18.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _i32p, _nullable(_u8p), _i64p]
    L.orc_label18.restype = C.c_int
    L.orc_chords13.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _f64p, _nullable(_i64p)]
    L.orc_chords13.restype = None
    L.orc_edt2.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _i64p]
    L.orc_edt2.restype = C.c_int
    L.orc_mis.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _i64p, _f64p, _nullable(_i64p)]
    L.orc_mis.restype = None
    L.orc_tau_g.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_tau_g.restype = C.c_double
    L.orc_collide19.argtypes = [_f64p, C.c_double, _f64p, _f64p, _nullable(_f64p)]
    L.orc_collide19.restype = None
    L.orc_flow_init.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _nullable(_f64p), _nullable(_f64p),
                                _f64p]
    L.orc_flow_init.restype = None
    L.orc_flow_solve.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, C.c_double, C.c_int, _f64p,
                                 C.c_int64, C.c_int64, C.c_int, C.c_double, _nullable(_f64p),
                                 _f64p, _nullable(_f64p), _f64p]
    L.orc_flow_solve.restype = C.c_int
    L.orc_flow_solve_p.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, C.c_double, C.c_int, _f64p,
                                   C.c_double, C.c_double, C.c_int64, C.c_int64, C.c_int,
                                   C.c_double, _nullable(_f64p), _f64p, _nullable(_f64p), _f64p]
    L.orc_flow_solve_p.restype = C.c_int
    L.orc_flow_update_node.argtypes = [_u8p, _f64p, C.c_double, C.c_int, _f64p, _f64p,
                                       _nullable(_f64p)]
    L.orc_flow_update_node.restype = None
    L.orc_collide19_trt.argtypes = [_f64p, C.c_double, _f64p, _f64p, _f64p]
    L.orc_collide19_trt.restype = None
    L.orc_collide19_mrt.argtypes = [_f64p, C.c_double, _nullable(_f64p), _f64p, _f64p,
                                    _nullable(_f64p)]
    L.orc_collide19_mrt.restype = None
    L.orc_mrt_matrices.argtypes = [_nullable(_f64p), _nullable(_f64p)]
    L.orc_mrt_matrices.restype = None
    L.orc_mrt_rates.argtypes = [C.c_double, _f64p]
    L.orc_mrt_rates.restype = None
    L.orc_collide7.argtypes = [_f64p, C.c_double, _f64p, C.POINTER(C.c_double)]
    L.orc_collide7.restype = None
    L.orc_knudsen_init.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _nullable(_f64p), _f64p]
    L.orc_knudsen_init.restype = None
    L.orc_knudsen_solve.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _f64p, C.c_double, C.c_double,
                                    C.c_int64, C.c_int64, C.c_int, C.c_double, _nullable(_f64p),
                                    _f64p, _nullable(_f64p), _nullable(_f64p), _f64p]
    L.orc_knudsen_solve.restype = C.c_int
    L.orc_knudsen_update_node.argtypes = [_u8p, _f64p, C.c_double, C.c_double, C.c_double, _f64p,
                                          C.POINTER(C.c_double)]
    L.orc_knudsen_update_node.restype = None
    L.orc_collide19_diff.argtypes = [_f64p, C.c_double, _f64p, C.POINTER(C.c_double)]
    L.orc_collide19_diff.restype = None
    L.orc_diffusion19_init.argtypes = [C.c_int, C.c_int, C.c_int, _u8p, _nullable(_f64p), _f64p]
    L.orc_diffusion19_init.restype = None
    L.orc_diffusion19_solve.argtypes = L.orc_knudsen_solve.argtypes
    L.orc_diffusion19_solve.restype = C.c_int
    L.orc_diffusion19_update_node.argtypes = L.orc_knudsen_update_node.argtypes
    L.orc_diffusion19_update_node.restype = None
    for name in ("orc_knudsen_diffusivity", "orc_mean_free_path"):
        getattr(L, name).restype = C.c_double
    L.orc_knudsen_diffusivity.argtypes = [C.c_double] * 3
    L.orc_mean_free_path.argtypes = [C.c_double] * 4
    L.orc_fc_dgm.argtypes = [C.c_double] * 4
    L.orc_fc_dgm.restype = C.c_double
    L.orc_k_kozeny_carman.argtypes = [C.c_double] * 2
    L.orc_k_kozeny_carman.restype = C.c_double
    for name, nargs in (("orc_lattice_diffusivity", 2), ("orc_time_step", 4),
                        ("orc_deff_physical", 4), ("orc_tortuosity", 3),
                        ("orc_bruggeman_alpha", 2), ("orc_k_physical", 2), ("orc_m2_to_mD", 1)):
        getattr(L, name).argtypes = [C.c_double] * nargs
        getattr(L, name).restype = C.c_double
    L.orc_num_threads.argtypes = []
    L.orc_num_threads.restype = C.c_int
    _lib = L
    return L


def num_threads() -> int:
    return lib().orc_num_threads()


# ---------------------------------------------------------------- random numbers
def splitmix64(seed: int, count: int):
    st = C.c_uint64(seed)
    return [lib().orc_splitmix64_next(C.byref(st)) for _ in range(count)]


def uniforms(seed: int, count: int):
    st = C.c_uint64(seed)
    return np.array([lib().orc_uniform(C.byref(st)) for _ in range(count)])


def normals(seed: int, count: int):
    st = C.c_uint64(seed)
    return np.array([lib().orc_normal(C.byref(st)) for _ in range(count)])


# ---------------------------------------------------------------- reconstruction
def sphere_volume(r):
    return lib().orc_sphere_volume(float(r))


def lens_volume(r1, r2, s):
    return lib().orc_lens_volume(float(r1), float(r2), float(s))


def _shape(n):
    if np.isscalar(n):
        n = (int(n),) * 3
    nx, ny, nz = (int(a) for a in n)
    return nx, ny, nz


def reconstruct(n, porosity, d_mean, d_std, d_min=1.0, overlap_tol=0.5, p_overlap=0.5, seed=1,
                max_trials=100_000_000, sphere_cap=1 << 20):
    """Section 2 reconstruction.  Returns (pore[nz,ny,nx] uint8, spheres[m,4] int64, info)."""
    nx, ny, nz = _shape(n)
    pore = np.zeros((nz, ny, nx), np.uint8)
    sph = np.zeros((sphere_cap, 4), np.int64)
    info = np.zeros(3, np.int64)
    st = lib().orc_reconstruct(nx, ny, nz, porosity, d_mean, d_std, d_min, overlap_tol, p_overlap,
                               seed, max_trials, pore, sph, sphere_cap, info)
    if st != OK:
        raise OracleError(st, "reconstruct")
    m = int(info[0])
    return pore, sph[:min(m, sphere_cap)].copy(), {"n_spheres": m, "n_trials": int(info[1]),
                                                    "n_pore": int(info[2])}


# ---------------------------------------------------------------- characterisation
def label18(pore):
    pore = np.ascontiguousarray(pore, np.uint8)
    nz, ny, nx = pore.shape
    label = np.zeros(pore.shape, np.int32)
    transport = np.zeros(pore.shape, np.uint8)
    info = np.zeros(3, np.int64)
    st = lib().orc_label18(nx, ny, nz, pore, label, transport, info)
    if st != OK:
        raise OracleError(st, "label18")
    return label, transport, {"n_pore": int(info[0]), "n_transport": int(info[1]),
                              "n_components": int(info[2])}


def chords13(pore, want_counts=False):
    pore = np.ascontiguousarray(pore, np.uint8)
    nz, ny, nx = pore.shape
    diam = np.zeros(pore.shape, np.float64)
    counts = np.zeros(pore.shape + (3,), np.int64) if want_counts else None
    lib().orc_chords13(nx, ny, nz, pore, diam, counts)
    return (diam, counts) if want_counts else diam


def edt2(pore):
    pore = np.ascontiguousarray(pore, np.uint8)
    nz, ny, nx = pore.shape
    e2 = np.zeros(pore.shape, np.int64)
    st = lib().orc_edt2(nx, ny, nz, pore, e2)
    if st != OK:
        raise OracleError(st, "edt2")
    return e2


def mis(pore, e2=None, want_emax=False):
    pore = np.ascontiguousarray(pore, np.uint8)
    nz, ny, nx = pore.shape
    if e2 is None:
        e2 = edt2(pore)
    diam = np.zeros(pore.shape, np.float64)
    emax = np.zeros(pore.shape, np.int64) if want_emax else None
    lib().orc_mis(nx, ny, nz, pore, np.ascontiguousarray(e2, np.int64), diam, emax)
    return (diam, emax) if want_emax else diam


def tau_g(d_p, d_ref, tau_ref=1.0):
    """Eq. 12, elementwise over numpy arrays (same arithmetic order as the C function)."""
    d_p = np.asarray(d_p, np.float64)
    return d_p / d_ref * (tau_ref - 0.5) + 0.5


# ---------------------------------------------------------------- flow (D3Q19)
def flow_init(fluid, u_init=None, drho_init=None):
    """Equilibrium populations (node-major) at rho = 1 + drho_init and u = u_init (rest
    and 1 where not given)."""
    fluid = np.ascontiguousarray(fluid, np.uint8)
    nz, ny, nx = fluid.shape
    f = np.zeros(fluid.shape + (19,), np.float64)
    ui = None if u_init is None else np.ascontiguousarray(u_init, np.float64)
    dr = None if drho_init is None else np.ascontiguousarray(drho_init, np.float64)
    lib().orc_flow_init(nx, ny, nz, fluid, ui, dr, f)
    return f


BGK, MRT, TRT = 0, 1, 2


def flow_solve(fluid, tau=0.8, force=(1e-6, 0.0, 0.0), max_steps=1_000_000, fixed_steps=0,
               check_every=100, tol=1e-7, f=None, u_prev0=None, want_u=True, collision=BGK,
               pressure=None):
    """Iterate the D3Q19 flow (see ``orc_flow_solve``) with the BGK, MRT or TRT collision.
    ``f`` (node-major state) is updated in place when given, else it starts from rest.
    pressure=(rho_in, rho_out): pressure boundaries in x (``orc_flow_solve_p``)."""
    fluid = np.ascontiguousarray(fluid, np.uint8)
    nz, ny, nx = fluid.shape
    if f is None:
        f = flow_init(fluid)
    F = np.ascontiguousarray(force, np.float64)
    u = np.zeros((3,) + fluid.shape, np.float64) if want_u else None
    out = np.zeros(8, np.float64)
    up = None if u_prev0 is None else np.ascontiguousarray(u_prev0, np.float64)
    if pressure is None:
        st = lib().orc_flow_solve(nx, ny, nz, fluid, tau, int(collision), F, max_steps,
                                  fixed_steps, check_every, tol, up, f, u, out)
    else:
        st = lib().orc_flow_solve_p(nx, ny, nz, fluid, tau, int(collision), F, float(pressure[0]),
                                    float(pressure[1]), max_steps, fixed_steps, check_every, tol,
                                    up, f, u, out)
    if st < 0:
        raise OracleError(st, "flow_solve")
    return {"status": st, "steps": int(out[0]), "k_lattice": out[1], "residual": out[2],
            "mean_rho_u": out[3:6].copy(), "mass_dev": out[6], "converged": bool(out[7]),
            "u": u, "f": f}


def collide19(fin, tau, force):
    fout = np.zeros(19)
    mom = np.zeros(4)
    lib().orc_collide19(np.ascontiguousarray(fin, np.float64), tau,
                        np.ascontiguousarray(force, np.float64), fout, mom)
    return fout, mom


def flow_update_node(nb_fluid, nb_f, tau, force, collision=BGK):
    fout = np.zeros(19)
    mom = np.zeros(4)
    lib().orc_flow_update_node(np.ascontiguousarray(nb_fluid, np.uint8),
                               np.ascontiguousarray(nb_f, np.float64), tau, int(collision),
                               np.ascontiguousarray(force, np.float64), fout, mom)
    return fout, mom


def collide19_mrt(fin, tau, force, rates=None):
    """One MRT collision (see ``orc_collide19_mrt``); rates overrides Eq. 7."""
    fout = np.zeros(19)
    mom = np.zeros(4)
    r = None if rates is None else np.ascontiguousarray(rates, np.float64)
    lib().orc_collide19_mrt(np.ascontiguousarray(fin, np.float64), tau, r,
                            np.ascontiguousarray(force, np.float64), fout, mom)
    return fout, mom


def collide19_trt(fin, tau, force):
    """The MRT collision of Eq. 7 in its two-relaxation-time form (``orc_collide19_trt``)."""
    fout = np.zeros(19)
    mom = np.zeros(4)
    lib().orc_collide19_trt(np.ascontiguousarray(fin, np.float64), tau,
                            np.ascontiguousarray(force, np.float64), fout, mom)
    return fout, mom


def mrt_matrices():
    q = np.zeros((19, 19))
    qi = np.zeros((19, 19))
    lib().orc_mrt_matrices(q, qi)
    return q, qi


def mrt_rates(tau):
    s = np.zeros(19)
    lib().orc_mrt_rates(tau, s)
    return s


# ---------------------------------------------------------------- Knudsen (D3Q7)
def knudsen_init(fluid, c_init=None):
    fluid = np.ascontiguousarray(fluid, np.uint8)
    nz, ny, nx = fluid.shape
    g = np.zeros(fluid.shape + (7,), np.float64)
    ci = None if c_init is None else np.ascontiguousarray(c_init, np.float64)
    lib().orc_knudsen_init(nx, ny, nz, fluid, ci, g)
    return g


def knudsen_solve(fluid, tau_g_field, c_in=1.0, c_out=0.0, max_steps=1_000_000, fixed_steps=0,
                  check_every=100, tol=1e-7, g=None, c_prev0=None, want_c=True, want_planes=True):
    fluid = np.ascontiguousarray(fluid, np.uint8)
    nz, ny, nx = fluid.shape
    if g is None:
        g = knudsen_init(fluid)
    tg = np.ascontiguousarray(np.broadcast_to(tau_g_field, fluid.shape), np.float64)
    c = np.zeros(fluid.shape, np.float64) if want_c else None
    planes = np.zeros(nx + 1, np.float64) if want_planes else None
    out = np.zeros(7, np.float64)
    cp = None if c_prev0 is None else np.ascontiguousarray(c_prev0, np.float64)
    st = lib().orc_knudsen_solve(nx, ny, nz, fluid, tg, c_in, c_out, max_steps, fixed_steps,
                                 check_every, tol, cp, g, c, planes, out)
    if st < 0:
        raise OracleError(st, "knudsen_solve")
    res = {"status": st, "steps": int(out[0]), "Deff_lattice": out[1], "residual": out[2],
           "phi_out": out[3], "phi_in": out[4], "sum_c": out[5], "converged": bool(out[6]),
           "c": c, "plane_flux": planes, "g": g}
    if planes is not None:
        # Eq. 14 with the mean link-plane flux in place of the outlet's
        res["Deff_planes"] = planes.mean() / (ny * nz) * (nx + 1) / (c_in - c_out)
    return res


def diffusion19_init(fluid, c_init=None):
    fluid = np.ascontiguousarray(fluid, np.uint8)
    nz, ny, nx = fluid.shape
    g = np.zeros(fluid.shape + (19,), np.float64)
    ci = None if c_init is None else np.ascontiguousarray(c_init, np.float64)
    lib().orc_diffusion19_init(nx, ny, nz, fluid, ci, g)
    return g


def diffusion19_solve(fluid, tau_g_field, c_in=1.0, c_out=0.0, max_steps=1_000_000,
                      fixed_steps=0, check_every=100, tol=1e-7, g=None, c_prev0=None,
                      want_c=True, want_planes=True):
    """The mass-transport solve on the D3Q19 lattice (Section 3.2); same returns as
    knudsen_solve."""
    fluid = np.ascontiguousarray(fluid, np.uint8)
    nz, ny, nx = fluid.shape
    if g is None:
        g = diffusion19_init(fluid)
    tg = np.ascontiguousarray(np.broadcast_to(tau_g_field, fluid.shape), np.float64)
    c = np.zeros(fluid.shape, np.float64) if want_c else None
    planes = np.zeros(nx + 1, np.float64) if want_planes else None
    out = np.zeros(7, np.float64)
    cp = None if c_prev0 is None else np.ascontiguousarray(c_prev0, np.float64)
    st = lib().orc_diffusion19_solve(nx, ny, nz, fluid, tg, c_in, c_out, max_steps, fixed_steps,
                                     check_every, tol, cp, g, c, planes, out)
    if st < 0:
        raise OracleError(st, "diffusion19_solve")
    return {"status": st, "steps": int(out[0]), "Deff_lattice": out[1], "residual": out[2],
            "phi_out": out[3], "phi_in": out[4], "sum_c": out[5], "converged": bool(out[6]),
            "c": c, "plane_flux": planes, "g": g}


def collide19_diff(gin, tau):
    gout = np.zeros(19)
    conc = C.c_double(0.0)
    lib().orc_collide19_diff(np.ascontiguousarray(gin, np.float64), tau, gout, C.byref(conc))
    return gout, conc.value


def diffusion19_update_node(nb_kind, nb_g, tau, c_in, c_out):
    gout = np.zeros(19)
    conc = C.c_double(0.0)
    lib().orc_diffusion19_update_node(np.ascontiguousarray(nb_kind, np.uint8),
                                      np.ascontiguousarray(nb_g, np.float64), tau, c_in, c_out,
                                      gout, C.byref(conc))
    return gout, conc.value


def collide7(gin, tau):
    gout = np.zeros(7)
    conc = C.c_double(0.0)
    lib().orc_collide7(np.ascontiguousarray(gin, np.float64), tau, gout, C.byref(conc))
    return gout, conc.value


def knudsen_update_node(nb_kind, nb_g, tau, c_in, c_out):
    gout = np.zeros(7)
    conc = C.c_double(0.0)
    lib().orc_knudsen_update_node(np.ascontiguousarray(nb_kind, np.uint8),
                                  np.ascontiguousarray(nb_g, np.float64), tau, c_in, c_out, gout,
                                  C.byref(conc))
    return gout, conc.value


# ---------------------------------------------------------------- closed forms
def knudsen_diffusivity(d_m, T, M=0.016043):
    return lib().orc_knudsen_diffusivity(d_m, T, M)


def mean_free_path(mu, p, T, M=0.016043):
    return lib().orc_mean_free_path(mu, p, T, M)


def fc_dgm(Deff, mu, k, P):
    return lib().orc_fc_dgm(Deff, mu, k, P)


def k_kozeny_carman(d, eps):
    return lib().orc_k_kozeny_carman(d, eps)


# ---------------------------------------------------------------- Section 4 relations, Eq. 15
def lattice_diffusivity(cs2, tau):
    """D_L = c_s^2 (tau - 1/2) (Section 3.2)."""
    return lib().orc_lattice_diffusivity(cs2, tau)


def time_step(cs2, tau_ref, dx_m, dk_ref):
    """Eq. 15: seconds per lattice step when a pore of tau_ref diffuses at dk_ref."""
    return lib().orc_time_step(cs2, tau_ref, dx_m, dk_ref)


def deff_physical(deff_lattice, cs2, tau_ref, dk_ref):
    """Eq. 15: a lattice diffusivity in m^2/s."""
    return lib().orc_deff_physical(deff_lattice, cs2, tau_ref, dk_ref)


def tortuosity(eps, d_free, deff):
    """Eq. 16: eps D / D_eff."""
    return lib().orc_tortuosity(eps, d_free, deff)


def bruggeman_alpha(deff_over_d, eps):
    """Section 4.2: alpha of D_eff / D = eps^alpha."""
    return lib().orc_bruggeman_alpha(deff_over_d, eps)


def k_physical(k_lattice, dx_m):
    """Eq. 15: permeability in m^2."""
    return lib().orc_k_physical(k_lattice, dx_m)


def m2_to_mD(k_m2):
    return lib().orc_m2_to_mD(k_m2)
