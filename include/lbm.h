/*
 * lbm.h -- C ABI of the MI355X lattice Boltzmann transport library (liblbm.so).
 *
 * The library computes, on one gfx950 GPU, the method of Chen, Kang, Zhang & Tao,
 * "Lattice Boltzmann prediction of transport properties in reconstructed
 * nanostructures of organic matters in shales" (arXiv:1410.1921): given the
 * parameters of a random-overlapping-sphere reconstruction of an organic-matter
 * nanostructure (Section 2) it gives its porosity, connectivity and pore-size map
 * (Section 4.1), its intrinsic permeability from a D3Q19 flow solve (Sections 3.1,
 * 3.3, 3.4, Eq. 13) and its effective Knudsen diffusivity and tortuosity from a
 * D3Q7 mass-transport solve with a local relaxation time (Sections 3.2-3.4,
 * Eqs. 10-12, 14, 16), and the derived properties of Section 4 (Eqs. 11, 15, 17,
 * 26, 29).
 *
 * Conventions
 *  - Volumes are [nz][ny][nx] with x fastest: voxel v = x + nx*(y + ny*z).
 *  - Pointers named *_h are HOST memory; every other array pointer is DEVICE memory
 *    allocated by the caller.  The library allocates no device memory: each call
 *    that needs scratch takes a caller-owned device `workspace` of `ws_bytes`
 *    bytes, sized by lbm_workspace_size().  Host scratch (reconstruction) is
 *    allocated and freed inside the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All
 *    device work is ordered on it.  Calls that return scalars to the host
 *    synchronise the stream before returning.
 *  - Calls on different streams with different workspaces and outputs may run
 *    concurrently; the library keeps no global state besides the per-thread error
 *    string.
 *  - Negative status values are errors (outputs unspecified); LBM_W_NOT_CONVERGED
 *    is a warning with every output filled at the step limit.  lbm_last_error()
 *    describes the most recent failure on the calling thread.
 *  - Device kernels are written for gfx950 only; a call on another device fails
 *    with LBM_E_DEVICE.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_W_NOT_CONVERGED 1
#define LBM_E_INVAL (-1)       /* bad argument: null pointer, size, parameter range */
#define LBM_E_NOMEM (-2)       /* workspace (or host memory) too small */
#define LBM_E_DEVICE (-3)      /* HIP runtime error or unsupported device */
#define LBM_E_RECON_STALL (-4) /* reconstruction hit max_trials below the porosity */
#define LBM_E_DIVERGED (-5)    /* NaN/Inf in a convergence reduction */

/* pore-size map of Section 4.1 or the maximum-inscribed-sphere map */
#define LBM_PSD_CHORD13 0
#define LBM_PSD_MIS 1

/* workspace kinds for lbm_workspace_size() */
#define LBM_WS_LABEL 0
#define LBM_WS_PORE_DIAM 1
#define LBM_WS_FLOW 2      /* flow solve, binary32 storage */
#define LBM_WS_KNUDSEN 3
#define LBM_WS_FLOW_FP16 4 /* flow solve, binary16 storage */
#define LBM_WS_FLOW_FP64 5 /* flow solve, binary64 storage */
#define LBM_WS_KNUDSEN_D3Q19 6 /* mass-transport solve on the D3Q19 lattice */

/* mass-transport lattice (the `lattice` field of lbm_knudsen_params) */
#define LBM_LATTICE_D3Q7 0  /* rest weight 1/4, face weights 1/8, c_s^2 = 1/4 */
#define LBM_LATTICE_D3Q19 1 /* the paper's: a_i = 1/3, 1/18, 1/36, c_s^2 = 1/3 */

/* population storage of the flow solve */
#define LBM_STORE_FP32 0 /* binary32 offsets f_i - w_i (1 + r(x)), r a reference density
                            (rho - 1) per 32-voxel half row segment, linear in x: the
                            least-squares line through rho - 1 of its nodes at the last
                            convergence check; collision in binary32 */
#define LBM_STORE_FP16 1 /* binary16 of S (f_i - w_i (1 + r(x))), S = 2^k with S max|F| in
                            [1, 2) (1 when F = 0); collision in binary32 */
#define LBM_STORE_FP64 2 /* binary64 offsets f_i - w_i, collision in binary64 */

/* x boundaries of the flow solve */
#define LBM_BOUNDARY_PERIODIC 0 /* periodic in x (driven by the body force) */
#define LBM_BOUNDARY_PRESSURE 1 /* pressure boundaries by non-equilibrium extrapolation
                                   (Section 3.3): ghost planes at x = -1 and x = nx; the
                                   ghost beside boundary node b holds f_eq(rho_bc, u_b) +
                                   f(b) - f_eq(rho_b, u_b) (Eq. 3's f_eq, rho_b, u_b the
                                   moments of b, u_b = (j - F/2)/rho_b), a ghost beside a
                                   solid b is solid (bounce back); binary32 or binary64
                                   storage; k = nu <rho u_x> / (F_x + (rho_in - rho_out) /
                                   (3 (nx + 1))) */

/* collision operator of the flow solve */
#define LBM_COLLIDE_BGK 0 /* single relaxation time 1/tau (Eq. 1) */
#define LBM_COLLIDE_MRT 1 /* the paper's MRT (Eqs. 4-7, Appendix A): moments under its Q, rates
                             0 (conserved), 1/tau (m1, m2, m9-m15) and
                             s_q = 8 (2 tau - 1)/(8 tau - 1) (m4, m6, m8, m16-m18), equilibrium
                             moments A1-A9 with rho0 = 1; the body force as Guo's source in
                             moment space scaled by (1 - s_k/2) */
#define LBM_COLLIDE_TRT 2 /* the same collision in velocity space: Eq. 7 relaxes the even
                             moments at 1/tau and the odd ones at s_q, so each pair of
                             opposite velocities splits into an even part (rate 1/tau) and an
                             odd part (rate s_q) around the incompressible equilibrium; equal to
                             LBM_COLLIDE_MRT up to rounding, at the cost of BGK */

/* sweep kernel variant (the `variant` field of the solve parameters): 0 lets the library
 * choose from the working-set size; otherwise LBM_VARIANT_EXPLICIT plus any of
 *   LBM_VARIANT_REMAP   workgroups ordered so that each XCD walks one contiguous region
 *   LBM_VARIANT_NTSTORE non-temporal (streaming) population stores
 * All variants compute identical results; they differ only in speed.  Any other bit
 * (2 included) is rejected with LBM_E_INVAL.  A batched solve without
 * LBM_VARIANT_EXPLICIT chooses the variant of each of its groups from the group's size.
 * Population offsets (direction x stride + node) are 32-bit while q x stride fits in
 * 32 bits (stride: the fluid-node count rounded up to 64; q = 19 for the flow and the
 * D3Q19 mass transport, 7 for D3Q7), which keeps the sweeps' register count down, and
 * 64-bit beyond, so that a 1024^3 domain of any porosity is solved; LBM_VARIANT_OFF64
 * asks for the 64-bit kernels on any size (single-lattice solves, with or without
 * LBM_VARIANT_EXPLICIT; identical results). */
#define LBM_VARIANT_AUTO 0
#define LBM_VARIANT_EXPLICIT 1
#define LBM_VARIANT_REMAP 4
#define LBM_VARIANT_NTSTORE 8
#define LBM_VARIANT_NOGRAPH 16 /* batched solves only: launch each step from the host
                                  instead of replaying a captured check interval */
#define LBM_VARIANT_OFF64 32 /* single-lattice solves only: 64-bit population offsets */

/* ------------------------------------------------------------------------------
 * Reconstruction (Section 2, Steps 1-3): pore spheres with random centres and
 * diameters are placed one by one; a trial must overlap an existing sphere with
 * probability p_overlap, and every lens it forms may hold at most overlap_tol of
 * either sphere's volume; placement stops at the first accepted sphere that brings
 * the pore-voxel count to ceil(porosity * N^3).
 *
 * Random numbers: SplitMix64 seeded with `seed`; uniforms are the top 53 bits.
 * Draw order per trial: overlap coin (skipped for the first sphere), centre x, y,
 * z (floor(u * 1024 * n) in 1/1024-voxel units), then the diameter ~ N(d_mean,
 * d_std) voxels by the Marsaglia polar method (first normal of a pair), redrawn
 * while below d_min, stored as round(d * 1024).  The geometry is not periodic;
 * voxel (i,j,k) is pore iff 4*sum((1024 i + 512 - c)^2) <= d^2 in integers.  The
 * forced-overlap branch needs overlap_tol > 0.  The result is bit-identical for
 * equal parameters on any x86-64 host with the same C library.
 *
 * pore      : device uint8[N^3] out, 1 = pore.
 * spheres_h : host int64[sphere_cap][4] out (cx, cy, cz, d in 1/1024 voxel), nullable;
 *             rows beyond sphere_cap are dropped (stats still count them).
 * stats_h   : host out, required.
 * Errors: LBM_E_INVAL (n < 1, porosity outside (0,1), overlap_tol or p_overlap
 * outside [0,1], d_mean <= 0, d_std < 0), LBM_E_RECON_STALL, LBM_E_DEVICE.
 * ---------------------------------------------------------------------------- */
typedef struct {
    int32_t n[3];         /* nx, ny, nz */
    double porosity;      /* target pore fraction, (0,1) */
    double d_mean, d_std; /* diameter law, voxels */
    double d_min;         /* smallest accepted diameter, voxels */
    double overlap_tol;   /* xi in [0,1] */
    double p_overlap;     /* p0 in [0,1] */
    uint64_t seed;
    int64_t max_trials;   /* <= 0: 10^8 */
} lbm_recon_params;

typedef struct {
    int64_t n_spheres, n_trials, n_pore;
    double porosity;
} lbm_recon_stats;

lbm_status lbm_reconstruct(const lbm_recon_params *p, uint8_t *pore, int64_t *spheres_h,
                           int64_t sphere_cap, lbm_recon_stats *stats_h, void *stream);

/* ------------------------------------------------------------------------------
 * Connected-phase labelling (Section 4.1): pore voxels joined through their 18
 * neighbours (6 faces, 12 edges), periodic in y and z, open in x.  Each component's
 * label is the smallest linear index it contains; a component is "transport" when
 * it touches both x = 0 and x = nx-1; connectivity = n_transport / n_pore.
 *
 * pore      : device uint8[N^3] in.
 * label     : device int32[N^3] out (-1 at solid voxels), required.
 * transport : device uint8[N^3] out, nullable.
 * workspace : LBM_WS_LABEL bytes.
 * ---------------------------------------------------------------------------- */
typedef struct {
    int64_t n_pore, n_transport, n_components;
    double porosity, connectivity;
} lbm_label_stats;

lbm_status lbm_label(const int32_t n[3], const uint8_t *pore, int32_t *label, uint8_t *transport,
                     lbm_label_stats *stats_h, void *workspace, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------------
 * lbm_label without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same labelling, counts and results as lbm_label, with its scratch (counters and the
 * two per-voxel face-flag arrays) in a static device array of 32 MiB + 256 B that each
 * device holds from the first call until the process ends.  It calls no hipMalloc,
 * hipFree or allocating library routine, and clears its scratch with kernels.
 * Volumes above LBM_LABEL_NOALLOC_MAX_VOXELS (256^3) fail with LBM_E_NOMEM.  Every call
 * on one device shares that device's scratch: calls that overlap on one device (other
 * streams, other host threads) race and must be serialised by the caller.
 * ---------------------------------------------------------------------------- */
#define LBM_LABEL_NOALLOC_MAX_VOXELS (16777216LL)
lbm_status lbm_label_noalloc(const int32_t n[3], const uint8_t *pore, int32_t *label,
                             uint8_t *transport, lbm_label_stats *stats_h, void *stream);

/* ------------------------------------------------------------------------------
 * Local pore diameter in voxels (double, 0 at solid voxels).
 * LBM_PSD_CHORD13 (Section 4.1): per pore voxel, the mean of its pore chords along
 *   13 directions (3 axes, 6 face diagonals, 4 body diagonals), each chord the run
 *   of consecutive pore voxels through it, stopped at the domain faces, times the
 *   direction's length: ((A + sqrt2*B) + sqrt3*C)/13 with A, B, C the integer
 *   per-class voxel sums.
 * LBM_PSD_MIS: d(p) = 2 sqrt(max{E(c) : c pore, |p-c|^2 < E(c)}) - 1 with E the
 *   exact squared distance from a voxel centre to the nearest solid voxel centre
 *   (no wrap); LBM_E_INVAL when the domain has no solid voxel.
 * Both maps are bit-identical to their plain definitions (no FMA contraction).
 *
 * pore      : device uint8[N^3] in.   diam : device double[N^3] out.
 * workspace : LBM_WS_PORE_DIAM bytes.
 * ---------------------------------------------------------------------------- */
lbm_status lbm_pore_diameter(const int32_t n[3], const uint8_t *pore, int32_t method,
                             double *diam, void *workspace, size_t ws_bytes, void *stream);

/* Number of non-zero voxels of a device uint8[N^3] mask (to size workspaces).
 * workspace: at least 256 bytes of device memory. */
lbm_status lbm_count(const int32_t n[3], const uint8_t *mask, int64_t *count_h, void *workspace,
                     size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------------
 * Flow solve (Section 3.1 with BGK, Eqs. 1-3, 8-9; half-way bounce-back at solid
 * links, Section 3.3; periodic in y and z, and in x unless `boundary` asks for the
 * pressure boundaries of Section 3.3, see LBM_BOUNDARY_PRESSURE).  The flow is driven by
 * the constant body-force density `force` added by Guo's scheme: u = (j + F/2)/rho and the
 * source (1 - 1/(2 tau)) w_i [3 (e_i - u) + 9 (e_i.u) e_i].F.  Starts from rho = 1
 * and u = u_init (or 0).  Every check_every steps (and at the last step) the
 * residual ||u(t) - u(t - n_c)|| / (n_c ||u(t)||) over fluid nodes is formed in
 * FP64; with fixed_steps > 0 exactly that many steps run, otherwise the solve stops
 * at the first check with residual < tol (and, with steady_tol > 0, an estimated distance
 * to steady state at or below steady_tol; Section 3.4 takes k at steady state, and the
 * residual alone bounds only the change per step) or at max_steps (LBM_W_NOT_CONVERGED).
 * Darcy (Eq. 13): k = nu <rho u_x> / F_x with nu = (tau - 1/2)/3 and the average
 * over the whole box; k_m2 = k voxel^2 (Eq. 15).
 *
 * D3Q19 velocities: 0 rest; 1..6 (+-1,0,0), (0,+-1,0), (0,0,+-1); 7..10 (+1,+1,0),
 * (-1,+1,0), (+1,-1,0), (-1,-1,0); 11..14 (+1,0,+1), (-1,0,+1), (+1,0,-1), (-1,0,-1);
 * 15..18 (0,+1,+1), (0,-1,+1), (0,+1,-1), (0,-1,-1) (the column order of the
 * paper's transformation matrix).
 *
 * fluid     : device uint8[N^3] in, 1 = fluid node (pass the pore mask, or the
 *             transport mask to drop dead pores).
 * u_out     : device float[3][N^3] out (planar, 0 at solids), nullable; with
 *             with_rho = 1 float[4][N^3], the fourth plane rho - 1.
 * u_init    : device float[3][N^3] in, nullable (warm start: the populations start at
 *             the equilibrium of u); with with_rho = 1 float[4][N^3], the fourth plane
 *             rho - 1 (else rho = 1).
 * workspace : LBM_WS_FLOW (_FP16, _FP64 for those storages) bytes for the fluid
 *             count; it also keeps the state for lbm_flow_step / lbm_flow_sample /
 *             resume (a resume must use the storage, collision and boundary of the
 *             solve that left it; one refused with LBM_E_INVAL leaves that state
 *             usable).
 * With binary16 storage a check interval without any change is reported as a stall
 * (LBM_W_NOT_CONVERGED, converged = 0): the rounded iteration has reached a fixed point
 * short of steady state.
 * The convergence residual, the velocity snapshot it compares against and u_out are
 * formed from the collision arithmetic and kept in binary32 (sums in binary64) for
 * every storage.
 * Errors: LBM_E_INVAL (tau <= 1/2, a non-finite force, voxel size <= 0 or non-finite,
 * check_every < 1, no fluid node, N > 1024, unknown storage, collision, boundary or
 * variant bits; pressure boundaries with binary16 storage, non-positive densities or no
 * driving), LBM_E_NOMEM, LBM_E_DIVERGED (NaN/Inf in a check, e.g. from a u_init that
 * holds one), LBM_E_DEVICE.
 * ---------------------------------------------------------------------------- */
typedef struct {
    double tau;
    double force[3];      /* body-force density, lattice units */
    int64_t max_steps;
    int64_t fixed_steps;  /* > 0: run exactly this many steps */
    int32_t check_every;  /* n_c */
    int32_t storage;      /* LBM_STORE_* */
    double tol;
    double voxel_nm;      /* lattice spacing, for k in m^2 and mD */
    int32_t resume;       /* 1: continue from the state in the workspace */
    int32_t variant;      /* LBM_VARIANT_* (0: automatic) */
    int32_t with_rho;     /* 1: u_init / u_out carry rho - 1 as a fourth plane */
    int32_t collision;    /* LBM_COLLIDE_BGK, LBM_COLLIDE_MRT or LBM_COLLIDE_TRT */
    int32_t boundary;     /* LBM_BOUNDARY_PERIODIC (0) or LBM_BOUNDARY_PRESSURE */
    int32_t reserved;
    double rho_in, rho_out; /* densities of the pressure boundaries (p = rho / 3) */
    double steady_tol;    /* > 0: a check also needs the estimated distance to steady state
                             (steady_dist of the result) at or below this; 0: residual only */
} lbm_flow_params;

typedef struct {
    int64_t steps, n_fluid;
    int32_t converged, reserved;
    double k_lattice, k_m2, k_mD;
    double residual;
    double mean_rho_u[3];
    double mass_dev;      /* sum over fluid of rho - 1 */
    double sweep_ms;      /* GPU time of the stream-collide kernels (HIP events) */
    double mlups;         /* fluid-node updates per microsecond of sweep_ms */
    double gbps;          /* algorithmic bytes per second of sweep_ms: 152 per update
                             (binary32), 304 (binary64), 76 (binary16) */
    double steady_dist;   /* estimated ||u - u_steady|| / ||u|| at the last check: r n_c rho /
                             (1 - rho), rho the mean decay ratio of the residual r over the
                             last (up to) 5 check intervals; +inf while r does not decay */
} lbm_flow_result;

lbm_status lbm_flow_solve(const int32_t n[3], const uint8_t *fluid, const lbm_flow_params *p,
                          lbm_flow_result *r_h, float *u_out, const float *u_init,
                          void *workspace, size_t ws_bytes, void *stream);

/* Advance the state held in `workspace` (left by lbm_flow_solve) by `steps` plain
 * stream-collide steps with the same parameters; no checks, no host sync. */
lbm_status lbm_flow_step(void *workspace, size_t ws_bytes, int64_t steps, void *stream);

/* Read the post-collision populations of `count` voxels from the state in
 * `workspace`: f_h[count][19] receives f_i - w_i (double: the stored value, divided by S
 * for binary16 storage, plus w_i r(x) at the node for binary32 and binary16),
 * fluid_h[count] whether the voxel is a fluid node (rows of solid voxels are 0).
 * count <= 65536. */
lbm_status lbm_flow_sample(void *workspace, size_t ws_bytes, const int64_t *vox_h, int64_t count,
                           double *f_h, uint8_t *fluid_h, void *stream);

/* ------------------------------------------------------------------------------
 * Batched flow solves: `count` independent lattices (Section 3.1, as lbm_flow_solve,
 * with one parameter set for all of them), advanced together so that small lattices
 * fill the device.  Each lattice's fluid list starts on a 256-node block of one
 * concatenated list.  The lattices still iterating are split, in order, into groups of
 * at most a byte budget of state (168 bytes per fluid node); each check interval runs
 * the groups one after the other, each for the whole interval, so that a group whose
 * state fits the 256 MB Infinity Cache keeps it there.  A group's interval is one
 * captured HIP graph (re-captured when the groups change) unless variant has
 * LBM_VARIANT_NOGRAPH; its kernel variant follows from its size unless variant has
 * LBM_VARIANT_EXPLICIT.  A lattice stops at its first check with residual < tol (its
 * result is then frozen) and the groups are formed again.  The populations, residuals,
 * steps and k of each lattice are those lbm_flow_solve gives it alone (the sums of a
 * check may differ in the last bits through their order), whatever the schedule.
 *
 * n_h      : host int32[count][3] lattice sizes (nx, ny, nz), each <= 1024.
 * fluid    : host array of count device pointers, each uint8[nz][ny][nx] (1 = fluid).
 * nf_h     : host int64[count] fluid-node counts (each >= 1; checked against the masks).
 * p        : one parameter set; storage must be LBM_STORE_FP32, resume and with_rho 0,
 *            force[0] != 0 (k is reported along x).
 * sched    : nullable, in/out (see lbm_batch_sched); null = autotuned budget.
 * r_h      : host lbm_flow_result[count] out; sweep_ms, mlups and gbps are those of
 *            the whole batch (autotuning included) in every entry.
 * u_out    : host array of count device pointers (or null; entries may be null), each
 *            float[3][nz][ny][nx] out: the lattice's velocity at its last check.
 * workspace: lbm_flow_batch_workspace(count, n_h, nf_h) bytes of device memory.
 * The work runs on an internal stream ordered after `stream` and before later work
 * on it; the call returns when the solve is finished.
 * Errors: LBM_E_INVAL (as lbm_flow_solve; a mask whose count is not nf_h, binary16 or
 * binary64 storage, resume, with_rho), LBM_E_NOMEM (workspace too small),
 * LBM_E_DIVERGED, LBM_W_NOT_CONVERGED (some lattice reached max_steps), LBM_E_DEVICE.
 * ---------------------------------------------------------------------------- */
typedef struct {
    int64_t group_bytes;      /* in: 0 autotune (the first check intervals run one
                                 candidate each: the whole batch as one group, then
                                 budgets of 128, 192, 256 and 384 MB; the fastest per
                                 node update runs the rest), < 0 one group, > 0 this
                                 budget */
    int64_t group_bytes_run;  /* out: the budget run (-1: one group) */
    int32_t groups;           /* out: groups once the budget is fixed */
    int32_t variant;          /* out: the variant bits run (0: chosen per group) */
    double tune_ms;           /* out: GPU time of the tuning intervals (their steps count) */
} lbm_batch_sched;

size_t lbm_flow_batch_workspace(int32_t count, const int32_t *n_h, const int64_t *nf_h);

lbm_status lbm_flow_solve_batch(int32_t count, const int32_t *n_h, const uint8_t *const *fluid,
                                const int64_t *nf_h, const lbm_flow_params *p,
                                lbm_batch_sched *sched, lbm_flow_result *r_h,
                                float *const *u_out, void *workspace, size_t ws_bytes,
                                void *stream);

/* ------------------------------------------------------------------------------
 * Knudsen mass-transport solve (Section 3.2, Eq. 10) on the D3Q7 lattice (rest weight
 * 1/4, face weights 1/8, c_s^2 = 1/4) or the paper's D3Q19 lattice (a_i = 1/3, 1/18,
 * 1/36, c_s^2 = 1/3, velocities as in the flow solve), g_eq = w_i C.  Local relaxation
 * time from the local pore diameter (Eq. 12): tau_g = (d_p/d_ref)(tau_ref - 1/2) +
 * 1/2 with d_ref = d_ref_nm / voxel_nm.  Boundaries (Section 3.3): bounce-back at
 * solid links, periodic in y and z, equilibrium ghost planes w_i C_in at x = -1 and
 * w_i C_out at x = nx (every population arriving from beyond an x face, diagonal ones
 * included, takes the ghost's value).  Starts from C = c_init (or 0); checks as in the
 * flow solve
 * with C as the field; with steady_tol > 0 a check with residual < tol also needs the
 * spread (max - min)/|mean| of the link-plane fluxes at or below steady_tol (the mean
 * taken as at least 1e-6 of the flux of an open box at tau_ref, so that a medium with no
 * path between the faces, whose steady fluxes all vanish, can converge too).
 * Eq. 14 on the lattice: D_eff = Phi_out / (ny nz) *
 * (nx + 1)/(C_in - C_out), Phi_out the net flux into the outlet ghost plane of the
 * last step's post-collision state.  Reported: D_eff / D_K,ref with D_K,ref =
 * c_s^2 (tau_ref - 1/2) in lattice units; D_eff in m^2/s via Eq. 11 at d_ref, T,
 * M (Eq. 15); tortuosity eps D_K,ref / D_eff (Eq. 16) with eps = n_fluid / N^3;
 * and the spread of the link-plane fluxes.
 *
 * fluid        : device uint8[N^3] in.
 * pore_diam    : device double[N^3] in (voxels; read at fluid voxels, each > 0).
 * c_field      : device float[N^3] out (0 at solids), nullable.
 * c_init       : device float[N^3] in, nullable.
 * plane_flux_h : host double[nx + 1] out, nullable: Phi(x - 1/2), x = 0..nx, over
 *                links with both ends fluid (ghost planes count as fluid; on D3Q19
 *                the five links with e_x = +1 per node).
 * workspace    : LBM_WS_KNUDSEN (LBM_WS_KNUDSEN_D3Q19 for that lattice) bytes.
 * Errors: LBM_E_INVAL (tau_g <= 1/2 or NaN anywhere, C_in == C_out, a non-finite C_in,
 * C_out, tau_ref, d_ref_nm or voxel_nm, unknown lattice, a resume with another lattice,
 * ...; a refused resume leaves the stored state usable), LBM_E_NOMEM, LBM_E_DIVERGED
 * (NaN/Inf in a check, e.g. from a c_init that holds one), LBM_E_DEVICE.
 * ---------------------------------------------------------------------------- */
typedef struct {
    double tau_ref;       /* tau_g at d_ref (the paper: 1.0) */
    double d_ref_nm;      /* reference pore diameter (the paper: 60 nm) */
    double voxel_nm;
    double c_in, c_out;
    double T_K, M_kg_mol; /* gas temperature and molar mass for D_K,ref (Eq. 11) */
    int64_t max_steps;
    int64_t fixed_steps;
    int32_t check_every;
    int32_t resume;
    double tol;
    int32_t variant;      /* LBM_VARIANT_* (0: automatic) */
    int32_t lattice;      /* LBM_LATTICE_D3Q7 (0) or LBM_LATTICE_D3Q19 */
    double steady_tol;    /* > 0: a check with residual < tol also needs the spread of the
                             link-plane fluxes at or below this (at steady state every plane
                             carries the same flux); 0: residual only */
} lbm_knudsen_params;

typedef struct {
    int64_t steps, n_fluid;
    int32_t converged, reserved;
    double Deff_lattice, Deff_over_DKref, Deff_m2s, DK_ref_m2s;
    double tortuosity, tortuosity_local; /* eps D_ref/D_eff and eps <D_L>/D_eff */
    double phi_in, phi_out, flux_spread; /* spread = (max - min)/mean of plane fluxes */
    double residual, sum_c;
    double sweep_ms, mlups, gbps;        /* gbps with 60 (D3Q7) or 156 (D3Q19) algorithmic
                                            bytes per update */
    double steady_dist;                  /* as in lbm_flow_result, for C */
    double Deff_planes;                  /* Eq. 14 with the mean of the nx + 1 link-plane
                                            fluxes in place of the outlet's: equal to
                                            Deff_lattice at steady state, nearer to it
                                            before (each slow mode's flux profile along x
                                            averages out) */
} lbm_knudsen_result;

lbm_status lbm_knudsen_solve(const int32_t n[3], const uint8_t *fluid, const double *pore_diam,
                             const lbm_knudsen_params *p, lbm_knudsen_result *r_h, float *c_field,
                             const float *c_init, double *plane_flux_h, void *workspace,
                             size_t ws_bytes, void *stream);

lbm_status lbm_knudsen_step(void *workspace, size_t ws_bytes, int64_t steps, void *stream);

/* g_h[count][q] (q = 7, or 19 for a D3Q19 state) receives the post-collision g_i (the
 * stored deviation plus w_i C_ref of its frame); tau_h[count] the node's tau_g as used
 * (binary32 widened), fluid_h as in lbm_flow_sample.  count <= 65536. */
lbm_status lbm_knudsen_sample(void *workspace, size_t ws_bytes, const int64_t *vox_h,
                              int64_t count, double *g_h, double *tau_h, uint8_t *fluid_h,
                              void *stream);

/* ------------------------------------------------------------------------------
 * Batched Knudsen solves: `count` independent lattices (Section 3.2, as
 * lbm_knudsen_solve, one parameter set for all), scheduled as the batched flow solves
 * are (block-aligned concatenated lists, groups of at most a byte budget of state at 68
 * bytes per fluid node run one after the other for whole check intervals, captured
 * intervals unless LBM_VARIANT_NOGRAPH, per-lattice retirement at checks).  Each
 * lattice keeps its own reference frames; the populations, steps and D_eff of a
 * lattice are those lbm_knudsen_solve gives it alone (check sums up to their
 * summation order), whatever the schedule.
 *
 * n_h       : host int32[count][3] lattice sizes, each <= 1024.
 * fluid     : host array of count device pointers, uint8[nz][ny][nx] each.
 * pore_diam : host array of count device pointers, double[nz][ny][nx] each (voxels).
 * nf_h      : host int64[count] fluid-node counts (each >= 1; checked).
 * p         : one parameter set; resume must be 0, lattice LBM_LATTICE_D3Q7.
 * sched     : nullable, in/out (lbm_batch_sched); null = autotuned budget.
 * r_h       : host lbm_knudsen_result[count] out (sweep_ms, mlups, gbps of the batch).
 * c_field   : host array of count device pointers or null (entries may be null),
 *             float[nz][ny][nx] out: C at the lattice's last check.
 * c_init    : host array of count device pointers or null (entries may be null),
 *             float[nz][ny][nx] in: initial C (warm start).
 * workspace : lbm_knudsen_batch_workspace(count, n_h, nf_h) bytes.
 * The work runs on an internal stream ordered after `stream` and before later work on
 * it; the call returns when the solve is finished.
 * Errors: as lbm_knudsen_solve; LBM_E_INVAL also for resume or a count mismatch.
 * ---------------------------------------------------------------------------- */
size_t lbm_knudsen_batch_workspace(int32_t count, const int32_t *n_h, const int64_t *nf_h);

lbm_status lbm_knudsen_solve_batch(int32_t count, const int32_t *n_h, const uint8_t *const *fluid,
                                   const double *const *pore_diam, const int64_t *nf_h,
                                   const lbm_knudsen_params *p, lbm_batch_sched *sched,
                                   lbm_knudsen_result *r_h, float *const *c_field,
                                   const float *const *c_init, void *workspace, size_t ws_bytes,
                                   void *stream);

/* ------------------------------------------------------------------------------
 * Derived properties (host only, pure).  Eq. 15 unit conversions; D_K of Eq. 11 at
 * the mean pore diameter; Kozeny-Carman k = d^2/180 eps^3/(1-eps)^2 (Eq. 17) with
 * d = d_mean_nm; Bruggeman exponent alpha = ln(D_eff/D_K,ref)/ln(eps) (Section
 * 4.2); mean free path (Eq. 29); f_c = 1 + D_eff mu/(k P) and k_a = k f_c (Eq. 26).
 * Any input pointer may be NULL; the outputs that need it are then NaN.
 * ---------------------------------------------------------------------------- */
typedef struct {
    double d_mean_nm;  /* mean pore-sphere diameter for Eq. 17 */
    double P_Pa, T_K, mu_Pa_s, M_kg_mol;
} lbm_props_params;

typedef struct {
    double porosity, connectivity;
    double k_m2, k_mD, k_KC_m2;
    double Deff_m2s, DK_ref_m2s, tortuosity, bruggeman_alpha;
    double mean_free_path_m, fc_dgm, k_apparent_m2;
} lbm_props_out;

lbm_status lbm_props(const lbm_label_stats *g, const lbm_flow_result *f,
                     const lbm_knudsen_result *d, const lbm_props_params *p, lbm_props_out *out);

/* Workspace bytes for a call of the given kind on an N^3 volume with n_fluid fluid
 * nodes (n_fluid < 0: assume every voxel). */
lbm_status lbm_workspace_size(int32_t kind, const int32_t n[3], int64_t n_fluid, size_t *bytes_h);

const char *lbm_last_error(void);
const char *lbm_version(void);

/* Measurement aid: copies `bytes` (a multiple of 16) from device buffer src to device
 * buffer dst with a plain streaming kernel (16-byte loads and stores, grid-stride).  Its
 * time is the attainable HBM bandwidth the sweeps are compared with, and its byte
 * counters calibrate FETCH_SIZE / WRITE_SIZE.  The buffers must not overlap. */
lbm_status lbm_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

/* sizeof() of the parameter and result structs, for bindings to check their mirrors:
 * 0 recon_params, 1 recon_stats, 2 label_stats, 3 flow_params, 4 flow_result,
 * 5 knudsen_params, 6 knudsen_result, 7 props_params, 8 props_out; 0 otherwise. */
size_t lbm_sizeof(int32_t which);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
