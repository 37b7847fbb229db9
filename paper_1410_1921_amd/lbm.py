"""Thin ctypes binding of liblbm.so (include/lbm.h), function for function.

The binding only marshals arguments: it turns torch tensors into device pointers, takes
the current torch stream, and provisions workspaces as torch uint8 tensors.  Every step
of the computation runs in the HIP library; if the library is missing the calls raise.

Volumes are torch tensors of shape (nz, ny, nx) on the GPU, x fastest.
"""
import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_W_NOT_CONVERGED = 0, 1
LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_RECON_STALL, LBM_E_DIVERGED = -1, -2, -3, -4, -5
LBM_PSD_CHORD13, LBM_PSD_MIS = 0, 1
LBM_WS_LABEL, LBM_WS_PORE_DIAM, LBM_WS_FLOW, LBM_WS_KNUDSEN = 0, 1, 2, 3
LBM_WS_FLOW_FP16, LBM_WS_FLOW_FP64 = 4, 5
LBM_WS_KNUDSEN_D3Q19 = 6
LBM_LATTICE_D3Q7, LBM_LATTICE_D3Q19 = 0, 1
LBM_STORE_FP32, LBM_STORE_FP16, LBM_STORE_FP64 = 0, 1, 2
LBM_COLLIDE_BGK, LBM_COLLIDE_MRT, LBM_COLLIDE_TRT = 0, 1, 2
LBM_BOUNDARY_PERIODIC, LBM_BOUNDARY_PRESSURE = 0, 1
_WS_FLOW_KIND = {LBM_STORE_FP32: LBM_WS_FLOW, LBM_STORE_FP16: LBM_WS_FLOW_FP16,
                 LBM_STORE_FP64: LBM_WS_FLOW_FP64}
LBM_VARIANT_AUTO, LBM_VARIANT_EXPLICIT, LBM_VARIANT_REMAP, LBM_VARIANT_NTSTORE = 0, 1, 4, 8
LBM_VARIANT_NOGRAPH = 16
LBM_VARIANT_OFF64 = 32  # single-lattice solves: 64-bit population offsets on any size

_STATUS = {0: "OK", 1: "W_NOT_CONVERGED", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_DEVICE",
           -4: "E_RECON_STALL", -5: "E_DIVERGED"}


class LbmError(RuntimeError):
    def __init__(self, status, what, msg):
        super().__init__(f"{what}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


# ------------------------------------------------------------------ struct mirrors
class lbm_recon_params(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("porosity", C.c_double), ("d_mean", C.c_double),
                ("d_std", C.c_double), ("d_min", C.c_double), ("overlap_tol", C.c_double),
                ("p_overlap", C.c_double), ("seed", C.c_uint64), ("max_trials", C.c_int64)]


class lbm_recon_stats(C.Structure):
    _fields_ = [("n_spheres", C.c_int64), ("n_trials", C.c_int64), ("n_pore", C.c_int64),
                ("porosity", C.c_double)]


class lbm_label_stats(C.Structure):
    _fields_ = [("n_pore", C.c_int64), ("n_transport", C.c_int64), ("n_components", C.c_int64),
                ("porosity", C.c_double), ("connectivity", C.c_double)]


class lbm_flow_params(C.Structure):
    _fields_ = [("tau", C.c_double), ("force", C.c_double * 3), ("max_steps", C.c_int64),
                ("fixed_steps", C.c_int64), ("check_every", C.c_int32), ("storage", C.c_int32),
                ("tol", C.c_double), ("voxel_nm", C.c_double), ("resume", C.c_int32),
                ("variant", C.c_int32), ("with_rho", C.c_int32), ("collision", C.c_int32),
                ("boundary", C.c_int32), ("reserved", C.c_int32), ("rho_in", C.c_double),
                ("rho_out", C.c_double), ("steady_tol", C.c_double)]


class lbm_flow_result(C.Structure):
    _fields_ = [("steps", C.c_int64), ("n_fluid", C.c_int64), ("converged", C.c_int32),
                ("reserved", C.c_int32), ("k_lattice", C.c_double), ("k_m2", C.c_double),
                ("k_mD", C.c_double), ("residual", C.c_double), ("mean_rho_u", C.c_double * 3),
                ("mass_dev", C.c_double), ("sweep_ms", C.c_double), ("mlups", C.c_double),
                ("gbps", C.c_double), ("steady_dist", C.c_double)]


class lbm_knudsen_params(C.Structure):
    _fields_ = [("tau_ref", C.c_double), ("d_ref_nm", C.c_double), ("voxel_nm", C.c_double),
                ("c_in", C.c_double), ("c_out", C.c_double), ("T_K", C.c_double),
                ("M_kg_mol", C.c_double), ("max_steps", C.c_int64), ("fixed_steps", C.c_int64),
                ("check_every", C.c_int32), ("resume", C.c_int32), ("tol", C.c_double),
                ("variant", C.c_int32), ("lattice", C.c_int32), ("steady_tol", C.c_double)]


class lbm_knudsen_result(C.Structure):
    _fields_ = [("steps", C.c_int64), ("n_fluid", C.c_int64), ("converged", C.c_int32),
                ("reserved", C.c_int32), ("Deff_lattice", C.c_double),
                ("Deff_over_DKref", C.c_double), ("Deff_m2s", C.c_double),
                ("DK_ref_m2s", C.c_double), ("tortuosity", C.c_double),
                ("tortuosity_local", C.c_double), ("phi_in", C.c_double), ("phi_out", C.c_double),
                ("flux_spread", C.c_double), ("residual", C.c_double), ("sum_c", C.c_double),
                ("sweep_ms", C.c_double), ("mlups", C.c_double), ("gbps", C.c_double),
                ("steady_dist", C.c_double), ("Deff_planes", C.c_double)]


class lbm_props_params(C.Structure):
    _fields_ = [("d_mean_nm", C.c_double), ("P_Pa", C.c_double), ("T_K", C.c_double),
                ("mu_Pa_s", C.c_double), ("M_kg_mol", C.c_double)]


class lbm_props_out(C.Structure):
    _fields_ = [(k, C.c_double) for k in (
        "porosity", "connectivity", "k_m2", "k_mD", "k_KC_m2", "Deff_m2s", "DK_ref_m2s",
        "tortuosity", "bruggeman_alpha", "mean_free_path_m", "fc_dgm", "k_apparent_m2")]


class lbm_batch_sched(C.Structure):
    _fields_ = [("group_bytes", C.c_int64), ("group_bytes_run", C.c_int64), ("groups", C.c_int32),
                ("variant", C.c_int32), ("tune_ms", C.c_double)]


STRUCTS = [lbm_recon_params, lbm_recon_stats, lbm_label_stats, lbm_flow_params, lbm_flow_result,
           lbm_knudsen_params, lbm_knudsen_result, lbm_props_params, lbm_props_out,
           lbm_batch_sched]

_P = C.c_void_p
_SIGS = {
    "lbm_reconstruct": ([C.POINTER(lbm_recon_params), _P, _P, C.c_int64,
                         C.POINTER(lbm_recon_stats), _P], C.c_int32),
    "lbm_label": ([_P, _P, _P, _P, C.POINTER(lbm_label_stats), _P, C.c_size_t, _P], C.c_int32),
    "lbm_label_noalloc": ([_P, _P, _P, _P, C.POINTER(lbm_label_stats), _P], C.c_int32),
    "lbm_pore_diameter": ([_P, _P, C.c_int32, _P, _P, C.c_size_t, _P], C.c_int32),
    "lbm_count": ([_P, _P, C.POINTER(C.c_int64), _P, C.c_size_t, _P], C.c_int32),
    "lbm_flow_solve": ([_P, _P, C.POINTER(lbm_flow_params), C.POINTER(lbm_flow_result), _P, _P,
                        _P, C.c_size_t, _P], C.c_int32),
    "lbm_flow_step": ([_P, C.c_size_t, C.c_int64, _P], C.c_int32),
    "lbm_flow_sample": ([_P, C.c_size_t, _P, C.c_int64, _P, _P, _P], C.c_int32),
    "lbm_flow_batch_workspace": ([C.c_int32, _P, _P], C.c_size_t),
    "lbm_flow_solve_batch": ([C.c_int32, _P, _P, _P, C.POINTER(lbm_flow_params),
                              C.POINTER(lbm_batch_sched), C.POINTER(lbm_flow_result), _P, _P,
                              C.c_size_t, _P], C.c_int32),
    "lbm_knudsen_solve": ([_P, _P, _P, C.POINTER(lbm_knudsen_params),
                           C.POINTER(lbm_knudsen_result), _P, _P, _P, _P, C.c_size_t, _P],
                          C.c_int32),
    "lbm_knudsen_step": ([_P, C.c_size_t, C.c_int64, _P], C.c_int32),
    "lbm_knudsen_batch_workspace": ([C.c_int32, _P, _P], C.c_size_t),
    "lbm_knudsen_solve_batch": ([C.c_int32, _P, _P, _P, _P, C.POINTER(lbm_knudsen_params),
                                 C.POINTER(lbm_batch_sched), C.POINTER(lbm_knudsen_result), _P,
                                 _P, _P, C.c_size_t, _P], C.c_int32),
    "lbm_knudsen_sample": ([_P, C.c_size_t, _P, C.c_int64, _P, _P, _P, _P], C.c_int32),
    "lbm_props": ([C.POINTER(lbm_label_stats), C.POINTER(lbm_flow_result),
                   C.POINTER(lbm_knudsen_result), C.POINTER(lbm_props_params),
                   C.POINTER(lbm_props_out)], C.c_int32),
    "lbm_workspace_size": ([C.c_int32, _P, C.c_int64, C.POINTER(C.c_size_t)], C.c_int32),
    "lbm_last_error": ([], C.c_char_p),
    "lbm_version": ([], C.c_char_p),
    "lbm_sizeof": ([C.c_int32], C.c_size_t),
    "lbm_copy_probe": ([_P, _P, C.c_size_t, _P], C.c_int32),
    # lbm_nn.h: layers of the warm-start network (wrapped in paper_1410_1921_amd.nn)
    "lbm_nn_conv3d": ([_P, _P, C.c_int32, C.c_int32, _P, _P, _P, C.c_int32, C.c_int32,
                       C.c_int32, _P], C.c_int32),
    "lbm_nn_wgrad_workspace": ([_P, C.c_int32, C.c_int32], C.c_size_t),
    "lbm_nn_conv3d_wgrad": ([_P, _P, C.c_int32, C.c_int32, _P, C.c_int32, C.c_int32, _P, _P,
                             C.c_int32, _P, C.c_size_t, _P], C.c_int32),
    "lbm_nn_transpose_weights": ([_P, C.c_int32, C.c_int32, _P, _P], C.c_int32),
    "lbm_nn_pool2": ([_P, C.c_int32, _P, C.c_int32, _P, C.c_int32, C.c_int32, _P], C.c_int32),
    "lbm_nn_pool2_bwd": ([_P, C.c_int32, _P, C.c_int32, _P, C.c_int32, C.c_int32, _P], C.c_int32),
    "lbm_nn_up2": ([_P, C.c_int32, _P, C.c_int32, _P, C.c_int32, _P], C.c_int32),
    "lbm_nn_up2_bwd": ([_P, C.c_int32, _P, C.c_int32, _P, C.c_int32, _P], C.c_int32),
    "lbm_nn_relu_bwd": ([C.c_int64, C.c_int32, _P, C.c_int32, _P, C.c_int32, _P, C.c_int32, _P],
                        C.c_int32),
    "lbm_nn_head_workspace": ([C.c_int64, C.c_int32], C.c_size_t),
    "lbm_nn_head": ([C.c_int64, _P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P, C.c_double, _P,
                     C.c_int32, _P, _P, C.POINTER(C.c_double), _P, C.c_size_t, _P], C.c_int32),
    "lbm_nn_adam": ([C.c_int64, _P, _P, _P, _P, _P, C.c_float, C.c_float, C.c_float, C.c_float,
                     C.c_int64, _P], C.c_int32),
    "lbm_nn_to_bf16": ([C.c_int64, _P, _P, _P], C.c_int32),
    "lbm_nn_make_input": ([C.c_int64, _P, _P, C.c_double, _P, C.c_int32, _P], C.c_int32),
    "lbm_nn_to_fields": ([C.c_int64, C.c_int32, _P, _P, _P, _P, _P], C.c_int32),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load liblbm.so (built in-tree by build.py).  Raises when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1410_1921_amd/build.py "
                           "(or __graft_entry__.build()) first")
    L = C.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(st, what):
    if st < 0:
        raise LbmError(st, what, load().lbm_last_error().decode())
    return st


def _n3(shape):
    nz, ny, nx = shape
    return (C.c_int32 * 3)(nx, ny, nz)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _as_dict(s):
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


def _vol(t, dtype, what):
    if not (t.is_cuda and t.dtype == dtype and t.dim() == 3 and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous 3-D {dtype} CUDA tensor (nz, ny, nx)")
    return t


class Workspace:
    """Caller-owned device workspace (a torch uint8 tensor) and its size."""

    def __init__(self, nbytes, device):
        self.nbytes = int(nbytes)
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())


def lbm_workspace_size(kind, shape, n_fluid=-1):
    out = C.c_size_t(0)
    _check(load().lbm_workspace_size(kind, _n3(shape), int(n_fluid), C.byref(out)),
           "lbm_workspace_size")
    return out.value


def lbm_version():
    return load().lbm_version().decode()


def lbm_sizeof(which):
    return load().lbm_sizeof(which)


def lbm_copy_probe(dst, src):
    """Streaming device copy of src into dst (same byte size, multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("lbm_copy_probe: sizes differ")
    _check(load().lbm_copy_probe(_ptr(dst), _ptr(src), nbytes, _stream()), "lbm_copy_probe")


# ------------------------------------------------------------------ geometry
def lbm_reconstruct(n, porosity, d_mean, d_std, d_min=1.0, overlap_tol=0.5, p_overlap=0.5,
                    seed=1, max_trials=0, sphere_cap=1 << 20, device="cuda"):
    """Section 2 reconstruction.  Returns (pore uint8 tensor (nz,ny,nx), spheres int64
    numpy [m,4] in 1/1024 voxel, stats dict)."""
    nx, ny, nz = (int(a) for a in (n if not np.isscalar(n) else (n, n, n)))
    p = lbm_recon_params((C.c_int32 * 3)(nx, ny, nz), porosity, d_mean, d_std, d_min,
                         overlap_tol, p_overlap, seed, max_trials)
    pore = torch.empty((nz, ny, nx), dtype=torch.uint8, device=device)
    sph = np.zeros((sphere_cap, 4), np.int64)
    st = lbm_recon_stats()
    _check(load().lbm_reconstruct(C.byref(p), _ptr(pore), sph.ctypes.data_as(C.c_void_p),
                                  sphere_cap, C.byref(st), _stream()), "lbm_reconstruct")
    m = min(st.n_spheres, sphere_cap)
    return pore, sph[:m].copy(), _as_dict(st)


def lbm_count(mask):
    _vol(mask, torch.uint8, "mask")
    ws = torch.empty(256, dtype=torch.uint8, device=mask.device)
    out = C.c_int64(0)
    _check(load().lbm_count(_n3(mask.shape), _ptr(mask), C.byref(out), _ptr(ws), 256, _stream()),
           "lbm_count")
    return out.value


def lbm_label(pore, want_transport=True):
    """Section 4.1 labelling.  Returns (label int32, transport uint8 or None, stats dict)."""
    _vol(pore, torch.uint8, "pore")
    label = torch.empty(pore.shape, dtype=torch.int32, device=pore.device)
    tr = torch.empty(pore.shape, dtype=torch.uint8, device=pore.device) if want_transport else None
    ws = Workspace(lbm_workspace_size(LBM_WS_LABEL, pore.shape), pore.device)
    st = lbm_label_stats()
    _check(load().lbm_label(_n3(pore.shape), _ptr(pore), _ptr(label), _ptr(tr), C.byref(st),
                            ws.ptr, ws.nbytes, _stream()), "lbm_label")
    return label, tr, _as_dict(st)


def lbm_label_noalloc(pore, want_transport=True):
    """lbm_label on the library's static scratch (no workspace; volumes up to 256^3)."""
    _vol(pore, torch.uint8, "pore")
    label = torch.empty(pore.shape, dtype=torch.int32, device=pore.device)
    tr = torch.empty(pore.shape, dtype=torch.uint8, device=pore.device) if want_transport else None
    st = lbm_label_stats()
    _check(load().lbm_label_noalloc(_n3(pore.shape), _ptr(pore), _ptr(label), _ptr(tr),
                                    C.byref(st), _stream()), "lbm_label_noalloc")
    return label, tr, _as_dict(st)


def lbm_pore_diameter(pore, method=LBM_PSD_CHORD13):
    """Pore diameter map (voxels, float64 tensor)."""
    _vol(pore, torch.uint8, "pore")
    diam = torch.empty(pore.shape, dtype=torch.float64, device=pore.device)
    ws = Workspace(lbm_workspace_size(LBM_WS_PORE_DIAM, pore.shape), pore.device)
    _check(load().lbm_pore_diameter(_n3(pore.shape), _ptr(pore), int(method), _ptr(diam), ws.ptr,
                                    ws.nbytes, _stream()), "lbm_pore_diameter")
    return diam


# ------------------------------------------------------------------ flow
class Solve:
    """Result of a solve: `result` (dict of the C result struct), `status`, the field
    tensor (or None), and the workspace that keeps the state for step/sample/resume."""

    def __init__(self, status, result, field, workspace, shape):
        self.status = status
        self.result = result
        self.field = field
        self.workspace = workspace
        self.shape = shape

    def __getitem__(self, k):
        return self.result[k]


def lbm_flow_solve(fluid, tau=0.8, force=(1e-6, 0.0, 0.0), max_steps=1_000_000, fixed_steps=0,
                   check_every=100, tol=1e-7, voxel_nm=1.0, want_u=False, u_init=None,
                   workspace=None, resume=False, n_fluid=None, variant=LBM_VARIANT_AUTO,
                   storage=LBM_STORE_FP32, with_rho=False, collision=LBM_COLLIDE_BGK,
                   pressure=None, steady_tol=0.0):
    """D3Q19 flow solve.  With with_rho the velocity field (want_u) and u_init carry a
    fourth plane, rho - 1.  pressure=(rho_in, rho_out): pressure boundaries in x.
    steady_tol > 0: convergence also needs the estimated distance to steady state."""
    _vol(fluid, torch.uint8, "fluid")
    if n_fluid is None:
        n_fluid = lbm_count(fluid)
    if workspace is None:
        workspace = Workspace(lbm_workspace_size(_WS_FLOW_KIND.get(storage, LBM_WS_FLOW),
                                                 fluid.shape, n_fluid), fluid.device)
    planes = 4 if with_rho else 3
    bc = LBM_BOUNDARY_PERIODIC if pressure is None else LBM_BOUNDARY_PRESSURE
    rho_in, rho_out = (1.0, 1.0) if pressure is None else (float(pressure[0]), float(pressure[1]))
    p = lbm_flow_params(tau, (C.c_double * 3)(*force), max_steps, fixed_steps, check_every,
                        int(storage), tol, voxel_nm, int(bool(resume)), int(variant),
                        int(bool(with_rho)), int(collision), bc, 0, rho_in, rho_out,
                        float(steady_tol))
    r = lbm_flow_result()
    u = torch.empty((planes,) + tuple(fluid.shape), dtype=torch.float32, device=fluid.device) \
        if want_u else None
    if u_init is not None and not (u_init.is_cuda and u_init.dtype == torch.float32 and
                                   u_init.is_contiguous() and
                                   u_init.numel() == planes * fluid.numel()):
        raise ValueError(f"u_init must be a contiguous float32 CUDA tensor ({planes}, nz, ny, nx)")
    st = _check(load().lbm_flow_solve(_n3(fluid.shape), _ptr(fluid), C.byref(p), C.byref(r),
                                      _ptr(u), _ptr(u_init), workspace.ptr, workspace.nbytes,
                                      _stream()), "lbm_flow_solve")
    return Solve(st, _as_dict(r), u, workspace, tuple(fluid.shape))


def lbm_flow_step(workspace, steps):
    _check(load().lbm_flow_step(workspace.ptr, workspace.nbytes, int(steps), _stream()),
           "lbm_flow_step")


def lbm_flow_sample(workspace, vox):
    """Post-collision f_i - w_i (float64 [count, 19]) and fluid flags at voxels `vox`."""
    vox = np.ascontiguousarray(vox, np.int64)
    f = np.zeros((len(vox), 19), np.float64)
    flag = np.zeros(len(vox), np.uint8)
    _check(load().lbm_flow_sample(workspace.ptr, workspace.nbytes, vox.ctypes.data_as(C.c_void_p),
                                  len(vox), f.ctypes.data_as(C.c_void_p),
                                  flag.ctypes.data_as(C.c_void_p), _stream()), "lbm_flow_sample")
    return f, flag


def lbm_flow_batch_workspace(shapes, n_fluids):
    """Workspace bytes of lbm_flow_solve_batch for lattices of these (nz, ny, nx) shapes
    and fluid counts (0: invalid sizes)."""
    n = np.array([[s[2], s[1], s[0]] for s in shapes], np.int32)
    nf = np.ascontiguousarray(n_fluids, np.int64)
    return load().lbm_flow_batch_workspace(len(n), n.ctypes.data_as(C.c_void_p),
                                           nf.ctypes.data_as(C.c_void_p))


def lbm_flow_solve_batch(fluids, tau=0.8, force=(1e-6, 0.0, 0.0), max_steps=1_000_000,
                         fixed_steps=0, check_every=100, tol=1e-7, voxel_nm=1.0, want_u=False,
                         n_fluids=None, variant=LBM_VARIANT_AUTO, collision=LBM_COLLIDE_BGK,
                         group_bytes=0, workspace=None, steady_tol=0.0):
    """D3Q19 flow solves of several lattices in one batch (binary32 storage).
    group_bytes: 0 autotuned, < 0 one group, > 0 the group budget.  Returns (status, list
    of result dicts, list of velocity fields or None, schedule dict)."""
    for m in fluids:
        _vol(m, torch.uint8, "fluid")
    if n_fluids is None:
        n_fluids = [lbm_count(m) for m in fluids]
    count = len(fluids)
    n = np.array([[m.shape[2], m.shape[1], m.shape[0]] for m in fluids], np.int32)
    nf = np.ascontiguousarray(n_fluids, np.int64)
    if workspace is None:
        workspace = Workspace(lbm_flow_batch_workspace([m.shape for m in fluids], nf),
                              fluids[0].device)
    p = lbm_flow_params(tau, (C.c_double * 3)(*force), max_steps, fixed_steps, check_every,
                        LBM_STORE_FP32, tol, voxel_nm, 0, int(variant), 0, int(collision),
                        LBM_BOUNDARY_PERIODIC, 0, 1.0, 1.0, float(steady_tol))
    res = (lbm_flow_result * count)()
    us = [torch.empty((3,) + tuple(m.shape), dtype=torch.float32, device=m.device)
          for m in fluids] if want_u else None
    masks = (C.c_void_p * count)(*[m.data_ptr() for m in fluids])
    u_ptrs = (C.c_void_p * count)(*[u.data_ptr() for u in us]) if want_u else None
    sched = lbm_batch_sched(int(group_bytes))
    st = _check(load().lbm_flow_solve_batch(count, n.ctypes.data_as(C.c_void_p), masks,
                                            nf.ctypes.data_as(C.c_void_p), C.byref(p),
                                            C.byref(sched), res, u_ptrs, workspace.ptr,
                                            workspace.nbytes, _stream()), "lbm_flow_solve_batch")
    return st, [_as_dict(r) for r in res], us, _as_dict(sched)


# ------------------------------------------------------------------ Knudsen
def lbm_knudsen_solve(fluid, pore_diam, tau_ref=1.0, d_ref_nm=60.0, voxel_nm=1.5, c_in=1.0,
                      c_out=0.0, T=323.0, M=0.016043, max_steps=1_000_000, fixed_steps=0,
                      check_every=100, tol=1e-7, want_c=False, c_init=None, want_planes=True,
                      workspace=None, resume=False, n_fluid=None, variant=LBM_VARIANT_AUTO,
                      lattice=LBM_LATTICE_D3Q7, steady_tol=0.0):
    """Mass-transport solve on the D3Q7 lattice or (lattice=LBM_LATTICE_D3Q19) the
    paper's D3Q19 lattice.  steady_tol > 0: convergence also needs the spread of the
    link-plane fluxes at or below it."""
    _vol(fluid, torch.uint8, "fluid")
    _vol(pore_diam, torch.float64, "pore_diam")
    if pore_diam.shape != fluid.shape:
        raise ValueError("pore_diam and fluid shapes differ")
    if c_init is not None and _vol(c_init, torch.float32, "c_init").shape != fluid.shape:
        raise ValueError("c_init and fluid shapes differ")
    if n_fluid is None:
        n_fluid = lbm_count(fluid)
    if workspace is None:
        kind = LBM_WS_KNUDSEN_D3Q19 if lattice == LBM_LATTICE_D3Q19 else LBM_WS_KNUDSEN
        workspace = Workspace(lbm_workspace_size(kind, fluid.shape, n_fluid), fluid.device)
    p = lbm_knudsen_params(tau_ref, d_ref_nm, voxel_nm, c_in, c_out, T, M, max_steps, fixed_steps,
                           check_every, int(bool(resume)), tol, int(variant), int(lattice),
                           float(steady_tol))
    r = lbm_knudsen_result()
    c = torch.empty(fluid.shape, dtype=torch.float32, device=fluid.device) if want_c else None
    nx = fluid.shape[2]
    planes = np.zeros(nx + 1, np.float64) if want_planes else None
    if c_init is not None:
        _vol(c_init, torch.float32, "c_init")
    st = _check(load().lbm_knudsen_solve(
        _n3(fluid.shape), _ptr(fluid), _ptr(pore_diam), C.byref(p), C.byref(r), _ptr(c),
        _ptr(c_init), None if planes is None else planes.ctypes.data_as(C.c_void_p),
        workspace.ptr, workspace.nbytes, _stream()), "lbm_knudsen_solve")
    workspace.lattice = int(lattice)
    res = _as_dict(r)
    res["plane_flux"] = planes
    return Solve(st, res, c, workspace, tuple(fluid.shape))


def lbm_knudsen_batch_workspace(shapes, n_fluids):
    """Workspace bytes of lbm_knudsen_solve_batch (0: invalid sizes)."""
    n = np.array([[s[2], s[1], s[0]] for s in shapes], np.int32)
    nf = np.ascontiguousarray(n_fluids, np.int64)
    return load().lbm_knudsen_batch_workspace(len(n), n.ctypes.data_as(C.c_void_p),
                                              nf.ctypes.data_as(C.c_void_p))


def lbm_knudsen_solve_batch(fluids, pore_diams, tau_ref=1.0, d_ref_nm=60.0, voxel_nm=1.5,
                            c_in=1.0, c_out=0.0, T=323.0, M=0.016043, max_steps=1_000_000,
                            fixed_steps=0, check_every=100, tol=1e-7, want_c=False, c_inits=None,
                            n_fluids=None, variant=LBM_VARIANT_AUTO, group_bytes=0,
                            workspace=None, steady_tol=0.0):
    """D3Q7 Knudsen solves of several lattices in one batch.  c_inits: None or a list of
    float32 fields (entries may be None); group_bytes as in lbm_flow_solve_batch.  Returns
    (status, list of result dicts, list of concentration fields or None, schedule dict)."""
    for m, d in zip(fluids, pore_diams):
        _vol(m, torch.uint8, "fluid")
        _vol(d, torch.float64, "pore_diam")
        if d.shape != m.shape:
            raise ValueError("pore_diam and fluid shapes differ")
    if c_inits is not None:
        for c0, m in zip(c_inits, fluids):
            if c0 is not None and (_vol(c0, torch.float32, "c_init").shape != m.shape):
                raise ValueError("c_init and fluid shapes differ")
    if n_fluids is None:
        n_fluids = [lbm_count(m) for m in fluids]
    count = len(fluids)
    n = np.array([[m.shape[2], m.shape[1], m.shape[0]] for m in fluids], np.int32)
    nf = np.ascontiguousarray(n_fluids, np.int64)
    if workspace is None:
        workspace = Workspace(lbm_knudsen_batch_workspace([m.shape for m in fluids], nf),
                              fluids[0].device)
    p = lbm_knudsen_params(tau_ref, d_ref_nm, voxel_nm, c_in, c_out, T, M, max_steps, fixed_steps,
                           check_every, 0, tol, int(variant), 0, float(steady_tol))
    res = (lbm_knudsen_result * count)()
    cs = [torch.empty(m.shape, dtype=torch.float32, device=m.device) for m in fluids] \
        if want_c else None
    V = C.c_void_p * count
    masks = V(*[m.data_ptr() for m in fluids])
    diams = V(*[d.data_ptr() for d in pore_diams])
    c_ptrs = V(*[c.data_ptr() for c in cs]) if want_c else None
    i_ptrs = V(*[0 if c0 is None else c0.data_ptr() for c0 in c_inits]) if c_inits else None
    sched = lbm_batch_sched(int(group_bytes))
    st = _check(load().lbm_knudsen_solve_batch(count, n.ctypes.data_as(C.c_void_p), masks, diams,
                                               nf.ctypes.data_as(C.c_void_p), C.byref(p),
                                               C.byref(sched), res, c_ptrs, i_ptrs, workspace.ptr,
                                               workspace.nbytes, _stream()),
                "lbm_knudsen_solve_batch")
    return st, [_as_dict(r) for r in res], cs, _as_dict(sched)


def lbm_knudsen_step(workspace, steps):
    _check(load().lbm_knudsen_step(workspace.ptr, workspace.nbytes, int(steps), _stream()),
           "lbm_knudsen_step")


def lbm_knudsen_sample(workspace, vox):
    """Post-collision g_i (float64 [count, q], q = 7 or 19 by the lattice of the solve
    that left the state), tau_g as used, fluid flags at `vox`."""
    vox = np.ascontiguousarray(vox, np.int64)
    q = 19 if getattr(workspace, "lattice", LBM_LATTICE_D3Q7) == LBM_LATTICE_D3Q19 else 7
    g = np.zeros((len(vox), 19), np.float64)  # room for either lattice
    tau = np.zeros(len(vox), np.float64)
    flag = np.zeros(len(vox), np.uint8)
    _check(load().lbm_knudsen_sample(workspace.ptr, workspace.nbytes,
                                     vox.ctypes.data_as(C.c_void_p), len(vox),
                                     g.ctypes.data_as(C.c_void_p), tau.ctypes.data_as(C.c_void_p),
                                     flag.ctypes.data_as(C.c_void_p), _stream()),
           "lbm_knudsen_sample")
    return g.reshape(-1)[:len(vox) * q].reshape(len(vox), q), tau, flag


# ------------------------------------------------------------------ properties
def lbm_props(label_stats=None, flow=None, knudsen=None, d_mean_nm=45.0, P=17236893.0, T=323.0,
              mu=1.73e-5, M=0.016043):
    def mk(cls, d):
        if d is None:
            return None
        s = cls()
        for name, _ in cls._fields_:
            v = d.get(name, 0)
            if hasattr(getattr(s, name), "__len__"):
                getattr(s, name)[:] = v
            else:
                setattr(s, name, v)
        return C.byref(s)

    p = lbm_props_params(d_mean_nm, P, T, mu, M)
    out = lbm_props_out()
    fr = flow.result if isinstance(flow, Solve) else flow
    kr = knudsen.result if isinstance(knudsen, Solve) else knudsen
    _check(load().lbm_props(mk(lbm_label_stats, label_stats), mk(lbm_flow_result, fr),
                            mk(lbm_knudsen_result, kr), C.byref(p), C.byref(out)), "lbm_props")
    return _as_dict(out)
