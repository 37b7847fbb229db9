"""Seeded synthetic workloads and hand-made test geometries.

This module holds no step of the method: it only states the parameter sets of the
workloads and draws simple masks (slits, ducts, tubes, random voxel masks) and random
states with numpy.  Both the HIP path's tests and the oracle's tests take their inputs
from here.

Volumes are C-ordered numpy arrays of shape (nz, ny, nx): linear index x + nx*(y + ny*z).
"""
import numpy as np

# --------------------------------------------------------------------------- workloads
# Sphere diameters are in voxels, drawn N(d_mean, d_std) (the paper draws uniform
# diameters in nm, Section 2; these workloads state the normal law in voxels).
# p_overlap is not given by the paper; 0.5 is used throughout.
SMALL_32 = dict(
    name="recon32_eps0.35_d8",
    recon=dict(n=(32, 32, 32), porosity=0.35, d_mean=8.0, d_std=2.0, d_min=1.0,
               overlap_tol=0.5, p_overlap=0.5, seed=1, psd="chord13"),
    voxel_nm=1.5,
    flow=dict(tau=0.8, force=(1e-6, 0.0, 0.0), fixed_steps=2000, check_every=100, tol=1e-7),
    knudsen=dict(tau_ref=1.0, d_ref_nm=60.0, c_in=1.0, c_out=0.0, T=323.0,
                 fixed_steps=2000, check_every=100, tol=1e-7),
)

METHANE_128 = dict(
    name="recon128_eps0.40_d12_mis_ch4_400K",
    recon=dict(n=(128, 128, 128), porosity=0.40, d_mean=12.0, d_std=3.0, d_min=1.0,
               overlap_tol=0.3, p_overlap=0.5, seed=2, psd="mis"),
    voxel_nm=2.0,
    flow=dict(tau=0.8, force=(1e-6, 0.0, 0.0), fixed_steps=0, max_steps=400_000,
              check_every=100, tol=1e-7),
    knudsen=dict(tau_ref=1.0, d_ref_nm=60.0, c_in=1.0, c_out=0.0, T=400.0,
                 fixed_steps=0, max_steps=4_000_000, check_every=100, tol=1e-7),
)

LARGE_512 = dict(
    name="recon512_eps0.25_d16",
    recon=dict(n=(512, 512, 512), porosity=0.25, d_mean=16.0, d_std=4.0, d_min=1.0,
               overlap_tol=0.7, p_overlap=0.5, seed=3, psd="mis"),
    voxel_nm=1.5,
    flow=dict(tau=0.8, force=(1e-6, 0.0, 0.0), fixed_steps=0, max_steps=400_000,
              check_every=100, tol=1e-7),
    crop=((192, 320), (192, 320), (192, 320)),
)

WORKLOADS = {w["name"]: w for w in (SMALL_32, METHANE_128, LARGE_512)}


def batch_params(count=150, seed=4):
    """Parameter draws of the batch of uneven reconstructions: edge in {64, 96, 128, 160},
    porosity U[0.2, 0.5], mean diameter U[6, 20] voxels (std = mean/4), overlap tolerance
    U[0, 1], seeds 1000 + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        edge = int(rng.choice([64, 96, 128, 160]))
        dm = float(rng.uniform(6.0, 20.0))
        out.append(dict(n=(edge, edge, edge), porosity=float(rng.uniform(0.2, 0.5)), d_mean=dm,
                        d_std=dm / 4.0, d_min=1.0, overlap_tol=float(rng.uniform(0.0, 1.0)),
                        p_overlap=0.5, seed=1000 + i, psd="mis"))
    return out


# The batch of uneven reconstructions (parameter draws of batch_params), 2 nm voxels,
# flow and Knudsen settings as in the 128^3 methane workload, binary32 state.
BATCH = dict(
    name="batch150_edges64-160_eps0.2-0.5", count=150, voxel_nm=2.0,
    flow=dict(tau=0.8, force=(1e-6, 0.0, 0.0), max_steps=400_000, check_every=100, tol=1e-7),
    knudsen=dict(tau_ref=1.0, d_ref_nm=60.0, c_in=1.0, c_out=0.0, T=400.0, check_every=100,
                 max_steps=4_000_000, tol=1e-7),
)


# The learned warm start: 96^3 reconstructions drawn with the batch's parameter laws
# (porosity U[0.2, 0.5], mean diameter U[6, 20] voxels with std = mean/4, overlap
# tolerance U[0, 1]); training seeds 5000-5399, held-out seeds 6000-6049.  Flow and
# Knudsen settings as in the 128^3 methane workload (2 nm voxels, CH4 at 400 K).
WARMSTART = dict(
    edge=96, train_seeds=range(5000, 5400), test_seeds=range(6000, 6050), voxel_nm=2.0,
    flow=dict(tau=0.8, force=(1e-6, 0.0, 0.0), check_every=100, max_steps=400_000),
    knudsen=dict(tau_ref=1.0, d_ref_nm=60.0, c_in=1.0, c_out=0.0, T=400.0, check_every=100,
                 max_steps=4_000_000),
)


def warmstart_params(seed, edge=96):
    """Reconstruction parameters of warm-start sample `seed`."""
    rng = np.random.default_rng(seed)
    dm = float(rng.uniform(6.0, 20.0))
    return dict(n=(edge, edge, edge), porosity=float(rng.uniform(0.2, 0.5)), d_mean=dm,
                d_std=dm / 4.0, d_min=1.0, overlap_tol=float(rng.uniform(0.0, 1.0)),
                p_overlap=0.5, seed=int(seed), psd="mis")


# --------------------------------------------------------------------------- geometries
def slit(nx, ny, nz, h, axis=1):
    """Fluid slab of width h centred across `axis` (1 = y, 2 = z), solid elsewhere."""
    m = np.zeros((nz, ny, nx), np.uint8)
    n = (nx, ny, nz)[axis]
    lo = (n - h) // 2
    sl = [slice(None)] * 3
    sl[2 - axis] = slice(lo, lo + h)
    m[tuple(sl)] = 1
    return m


def square_duct(nx, side, pad=1):
    """Fluid square duct along x of the given side with `pad` solid layers around it."""
    n = side + 2 * pad
    m = np.zeros((n, n, nx), np.uint8)
    m[pad:pad + side, pad:pad + side, :] = 1
    return m


def tube(nx, radius, pad=1):
    """Voxelised circular tube along x: voxel centres within `radius` of the axis."""
    n = int(2 * np.ceil(radius)) + 2 * pad
    c = n / 2.0
    yy, zz = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="xy")
    disk = ((yy - c) ** 2 + (zz - c) ** 2 <= radius * radius).astype(np.uint8)  # [z][y]
    return np.repeat(disk[:, :, None], nx, axis=2)


def sphere_in_cube(n):
    """Solid sphere of diameter n inscribed in an n^3 cube (voxel centres within n/2 of
    the centre are solid); the rest is pore."""
    c = n / 2.0
    z, y, x = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    return ((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2 > c * c).astype(np.uint8)


def random_mask(shape, p, seed):
    """Independent Bernoulli(p) pore voxels; shape is (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    return (rng.random(shape) < p).astype(np.uint8)


def blob_mask(shape, p, seed, smooth=1):
    """Random mask with some spatial correlation: Bernoulli field averaged over a
    (2*smooth+1)^3 box (periodic) and thresholded to pore fraction ~p."""
    rng = np.random.default_rng(seed)
    a = rng.random(shape)
    acc = np.zeros_like(a)
    for dz in range(-smooth, smooth + 1):
        for dy in range(-smooth, smooth + 1):
            for dx in range(-smooth, smooth + 1):
                acc += np.roll(a, (dz, dy, dx), axis=(0, 1, 2))
    thr = np.quantile(acc, 1.0 - p)
    return (acc > thr).astype(np.uint8)


def random_state(n_nodes, q, scale, seed):
    """Seeded random population offsets (node-major [n_nodes, q]) of size `scale`."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((n_nodes, q))


def _fmix64(k):
    """MurmurHash3's 64-bit finaliser (uint64 numpy arrays, wrapping arithmetic)."""
    k = k ^ (k >> np.uint64(33))
    k = k * np.uint64(0xFF51AFD7ED558CCD)
    k = k ^ (k >> np.uint64(33))
    k = k * np.uint64(0xC4CEB9FE1A85EC53)
    return k ^ (k >> np.uint64(33))


def hash_uniform(seed, idx):
    """Counter-based uniforms in [0, 1) for integer indices `idx`: any subset of a large
    field can be drawn without drawing the rest (float64, 53 bits)."""
    idx = np.asarray(idx, np.uint64)
    with np.errstate(over="ignore"):
        k = _fmix64(idx * np.uint64(0x9E3779B97F4A7C15) + _fmix64(np.uint64(seed) + np.uint64(1)))
    return (k >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def hash_field(shape, seed, lo, hi, comps=1, lin=None):
    """Seeded field of values uniform in [lo, hi): planar [comps, nz, ny, nx] float32
    (comps > 1) or [nz, ny, nx].  With `lin` (linear voxel indices) only those voxels are
    drawn, shape [comps, len(lin)]."""
    nvox = int(np.prod(shape))
    out = []
    for c in range(comps):
        idx = np.arange(nvox, dtype=np.uint64) if lin is None else np.asarray(lin, np.uint64)
        u = hash_uniform(seed * 8 + c, idx + np.uint64(c) * np.uint64(nvox))
        v = (lo + (hi - lo) * u).astype(np.float32)
        out.append(v.reshape(shape) if lin is None else v)
    return np.stack(out) if comps > 1 else out[0]
