// D3Q7 Knudsen mass-transport solve: fused pull-stream + BGK collision with the local
// relaxation time of each node (Section 3.2, Eqs. 10-12 on D3Q7), bounce-back at solid
// links, periodic in y and z, equilibrium ghost planes at x = -1 and x = nx (Section
// 3.3), and the outlet-plane flux of Eq. 14.
//
// Storage: s[i][node] = g_i - w_i C_ref(x) in binary32, where C_ref(x) is a reference
// profile along x: the mean concentration of plane x, refreshed at every convergence
// check (ghost planes: C_ref(-1) = C_in, C_ref(nx) = C_out).  The collision is carried
// out on these deviations, so rounding acts on numbers far smaller than g itself: both
// the transient front and the steady state keep binary32 errors near 1e-7 relative,
// where storing g directly freezes the iteration (per-step changes below half an ulp)
// up to ~1e-3 away from its steady state on long channels.  The reference costs no
// bandwidth: it depends on x alone (a table of nx + 2 values).  1/tau_g per node in
// binary32.  Per fluid-node update: 7 loads + 7 stores of 4 bytes + 4 bytes of 1/tau_g.
#include <cmath>
#include <cstring>
#include <vector>

#include "lbm_internal.h"

namespace lbm {

// D3Q7: rest, then +x, -x, +y, -y, +z, -z.
#define LBM_D3Q7_TABLES [[maybe_unused]] constexpr int OPP[7] = {0, 2, 1, 4, 3, 6, 5};

constexpr uint64_t kKnMagic = 0x4c424d4b4e554431ull;  // "LBMKNUD1"
constexpr int kKnSums = 5;  // |dC|^2, C^2, Phi_out, Phi_in, C
constexpr int kKnSampleMax = 65536;
constexpr float kW0 = 0.25f, kW1 = 0.125f;

struct KnHeader {
    uint64_t magic;
    int32_t nx, ny, nz, cur;
    int64_t n_fluid, steps_done;
    double c_in, c_out;
};

struct KnWs {
    KnHeader *hdr;
    unsigned long long *counter;
    double *res;
    double *plane;
    int32_t *bcount, *idmap;
    int64_t *samp_vox;
    double *samp_out;
    uint8_t *samp_flag;
    uint32_t *coords;
    float *g[2];
    float *omega;
    float *csnap;
    double *partials;
    double *ref, *ref_new;  // reference profile C_ref(x), index x + 1 for x = -1..nx
    float *shm, *shp;       // w_1 (C_ref(x -+ 1) - C_ref(x)), index x + 1
    int64_t stride;
    size_t bytes;
};

static int64_t kn_blocks(int64_t nf) { return (nf + 255) / 256; }

static KnWs carve_kn(void *base, const Grid &g, int64_t nf) {
    KnWs w;
    Carver c(base);
    w.hdr = c.take<KnHeader>(1);
    w.counter = c.take<unsigned long long>(4);
    w.res = c.take<double>(32);
    w.plane = c.take<double>(kMaxEdge + 1);
    w.bcount = c.take<int32_t>(g.nbricks() + 1);
    w.idmap = c.take<int32_t>(g.nbricks() * kBrickVox);
    w.samp_vox = c.take<int64_t>(kKnSampleMax);
    w.samp_out = c.take<double>((size_t)kKnSampleMax * 8);
    w.samp_flag = c.take<uint8_t>(kKnSampleMax);
    int64_t nfp = nf < 1 ? 1 : nf;
    w.stride = (nfp + 63) / 64 * 64;
    w.coords = c.take<uint32_t>(nfp);
    w.g[0] = c.take<float>((size_t)7 * w.stride);
    w.g[1] = c.take<float>((size_t)7 * w.stride);
    w.omega = c.take<float>(w.stride);
    w.csnap = c.take<float>(w.stride);
    w.partials = c.take<double>((size_t)xcd_launch(kn_blocks(nfp)) * kKnSums);
    w.ref = c.take<double>(kMaxEdge + 2);
    w.ref_new = c.take<double>(kMaxEdge + 2);
    w.shm = c.take<float>(kMaxEdge + 2);
    w.shp = c.take<float>(kMaxEdge + 2);
    w.bytes = c.off;
    return w;
}

size_t knudsen_ws_bytes_n(const int32_t n[3], int64_t nf) {
    Grid g = make_grid(n);
    return carve_kn(nullptr, g, nf < 0 ? g.nvox() : nf).bytes;
}

struct Sweep7 {
    Grid g;
    int64_t nf, stride, launched;
    const uint32_t *__restrict__ coords;
    const int32_t *__restrict__ idmap;
    const float *__restrict__ omega;
    const float *__restrict__ src;
    float *__restrict__ dst;
    const float *__restrict__ shm;  // change of reference along a +x link into x
    const float *__restrict__ shp;  // change of reference along a -x link into x
    // check variant
    const double *__restrict__ ref;
    float *__restrict__ csnap;
    float *__restrict__ c_out;
    double *__restrict__ partials;
};

template <bool CHECK>
__global__ __launch_bounds__(256) void k_sweep7(Sweep7 a) {
    LBM_D3Q7_TABLES
    const int64_t lb = xcd_block(blockIdx.x, a.launched);
    const int64_t n = lb * 256 + threadIdx.x;
    double acc[kKnSums] = {0, 0, 0, 0, 0};
    if (n < a.nf) {
        const uint32_t c = a.coords[n];
        const int x = c & 1023, y = (c >> 10) & 1023, z = c >> 20;
        const Grid &g = a.g;
        const int xm = x - 1, xp = x + 1;  // ghost planes beyond the x faces
        const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
        const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
        // neighbour slots in direction order 1..6 (source x - e_i); beyond an x face the
        // slot of the node itself stands in, its id is replaced by -2 (ghost plane)
        int slot[7];
        slot[1] = (int)g.slot(xm >= 0 ? xm : x, y, z);
        slot[2] = (int)g.slot(xp < g.nx ? xp : x, y, z);
        slot[3] = (int)g.slot(x, ym, z);
        slot[4] = (int)g.slot(x, yp, z);
        slot[5] = (int)g.slot(x, y, zm);
        slot[6] = (int)g.slot(x, y, zp);
        // phase 1: ids, 1/tau_g and the link shifts, all in flight together
        int ids[7];
#pragma unroll
        for (int i = 1; i < 7; i++) ids[i] = a.idmap[slot[i]];
        const float om = a.omega[n];
        const float sm = a.shm[x + 1], sp = a.shp[x + 1];
        if (xm < 0) ids[1] = -2;
        if (xp >= g.nx) ids[2] = -2;
        // phase 2: the populations (id -1: solid, bounce back; -2: ghost plane)
        uint32_t off[7];
        off[0] = (uint32_t)n;
#pragma unroll
        for (int i = 1; i < 7; i++)
            off[i] = ids[i] >= 0 ? (uint32_t)(i * a.stride + ids[i]) : (uint32_t)(OPP[i] * a.stride + n);
        float ai[7];
#pragma unroll
        for (int i = 0; i < 7; i++) ai[i] = a.src[off[i]];
        // incoming deviations from this node's reference w_i C_ref(x): a population
        // streamed along +-x from a fluid neighbour (or a ghost plane, whose deviation is
        // 0) changes reference plane; bounced and y/z populations keep theirs
        if (ids[1] == -2) ai[1] = 0.f;
        if (ids[2] == -2) ai[2] = 0.f;
        if (ids[1] != -1) ai[1] += sm;
        if (ids[2] != -1) ai[2] += sp;
        float cdev = 0.f;  // C - C_ref(x)
#pragma unroll
        for (int i = 0; i < 7; i++) cdev += ai[i];
        float so[7];
#pragma unroll
        for (int i = 0; i < 7; i++) {
            const float w = i == 0 ? kW0 : kW1;
            so[i] = ai[i] - om * (ai[i] - w * cdev);
            a.dst[(int64_t)i * a.stride + n] = so[i];
        }
        if (CHECK) {
            const double conc = a.ref[x + 1] + (double)cdev;
            const double d = conc - (double)a.csnap[n];
            acc[0] = d * d;
            acc[1] = conc * conc;
            // net +x flux into the outlet ghost plane and out of the inlet one, as
            // streamed (in the node's reference frame)
            if (xp >= g.nx) acc[2] = (double)so[1] - (double)sp;
            if (xm < 0) acc[3] = (double)sm - (double)so[2];
            acc[4] = conc;
            a.csnap[n] = (float)conc;
            if (a.c_out) a.c_out[g.lin(x, y, z)] = (float)conc;
        }
    }
    if (CHECK) {
        __shared__ double lds[4 * kKnSums];
        double out[kKnSums];
        block_sum<kKnSums>(acc, lds, out);
        if (threadIdx.x == 0 && lb * 256 < a.nf)
#pragma unroll
            for (int k = 0; k < kKnSums; k++) a.partials[lb * kKnSums + k] = out[k];
    }
}

// 1/tau_g per node from the pore diameter (Eq. 12); counts nodes with tau_g <= 1/2 and
// forms the partial sums of tau_g - 1/2 (for the local tortuosity).
__global__ __launch_bounds__(256) void k_kn_init(Grid g, int64_t nf, int64_t stride,
                                                 const uint32_t *__restrict__ coords,
                                                 const double *__restrict__ diam, double d_ref,
                                                 double tau_ref, const float *__restrict__ c_init,
                                                 float *__restrict__ gbuf,
                                                 float *__restrict__ omega,
                                                 float *__restrict__ csnap, int init_pop,
                                                 unsigned long long *bad,
                                                 double *__restrict__ partials) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double acc[1] = {0.0};
    if (n < nf) {
        const uint32_t c = coords[n];
        const int64_t v = g.lin(c & 1023, (c >> 10) & 1023, c >> 20);
        const double tau = diam[v] / d_ref * (tau_ref - 0.5) + 0.5;
        if (!(tau > 0.5)) atomicAdd(bad, 1ull);
        omega[n] = (float)(1.0 / tau);
        acc[0] = tau - 0.5;
        if (init_pop) {
            // equilibrium w_i C_init against a zero reference; the solve re-centres it
            // on the plane means before the first step
            const float c0 = c_init ? c_init[v] : 0.f;
            gbuf[n] = kW0 * c0;
            for (int i = 1; i < 7; i++) gbuf[(int64_t)i * stride + n] = kW1 * c0;
            csnap[n] = c0;
        }
    }
    __shared__ double lds[4];
    double out[1];
    block_sum<1>(acc, lds, out);
    if (threadIdx.x == 0) partials[blockIdx.x] = out[0];
}

// Net +x flux through the link plane x = px - 1/2 (px = 0..nx), one block per plane,
// over links with both ends fluid (ghost planes count as fluid).
__global__ __launch_bounds__(256) void k_plane_flux(Grid g, int64_t stride,
                                                    const int32_t *__restrict__ idmap,
                                                    const float *__restrict__ gcur,
                                                    const float *__restrict__ shm,
                                                    double *__restrict__ plane) {
    const int px = blockIdx.x;
    const int left = px - 1, right = px;
    double acc[1] = {0.0};
    for (int64_t k = threadIdx.x; k < (int64_t)g.ny * g.nz; k += 256) {
        const int y = (int)(k % g.ny), z = (int)(k / g.ny);
        const int il = left >= 0 ? idmap[g.slot(left, y, z)] : -2;
        const int ir = right < g.nx ? idmap[g.slot(right, y, z)] : -2;
        if (il == -1 || ir == -1) continue;
        // g_{+x}(left) - g_{-x}(right) in the frame of `right`: s_{+x}(left) + shm(right) -
        // s_{-x}(right); the ghost planes hold zero deviation
        const double fwd = left >= 0 ? (double)gcur[stride + il] : 0.0;
        const double bwd = right < g.nx ? (double)gcur[2 * stride + ir] : 0.0;
        acc[0] += (fwd + (double)shm[right + 1]) - bwd;
    }
    __shared__ double lds[4];
    double out[1];
    block_sum<1>(acc, lds, out);
    if (threadIdx.x == 0) plane[px] = out[0];
}

__global__ void k_kn_sample(Grid g, int64_t count, int64_t stride, const int64_t *__restrict__ vox,
                            const int32_t *__restrict__ idmap, const float *__restrict__ gcur,
                            const float *__restrict__ omega, const double *__restrict__ cref,
                            double *__restrict__ out, uint8_t *__restrict__ flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const int64_t v = vox[s];
    const int x = (int)(v % g.nx), y = (int)((v / g.nx) % g.ny), z = (int)(v / ((int64_t)g.nx * g.ny));
    const int id = idmap[g.slot(x, y, z)];
    flag[s] = id >= 0;
    const double ref = cref[x + 1];
    for (int i = 0; i < 7; i++)
        out[s * 8 + i] = id >= 0 ? (double)gcur[(int64_t)i * stride + id] + (i ? 0.125 : 0.25) * ref
                                 : 0.0;
    out[s * 8 + 7] = id >= 0 ? 1.0 / (double)omega[id] : 0.0;
}

// The reference profile follows the solution: at each check the plane means of C become
// the new C_ref (planes without fluid keep theirs), the stored state is moved onto it,
// and the link shift tables are rebuilt.  All three steps are deterministic.
__global__ __launch_bounds__(256) void k_plane_mean(Grid g, const int32_t *__restrict__ idmap,
                                                    const float *__restrict__ csnap,
                                                    const double *__restrict__ ref,
                                                    double *__restrict__ ref_new) {
    const int x = blockIdx.x;
    double acc[2] = {0.0, 0.0};
    for (int64_t k = threadIdx.x; k < (int64_t)g.ny * g.nz; k += 256) {
        const int id = idmap[g.slot(x, (int)(k % g.ny), (int)(k / g.ny))];
        if (id >= 0) {
            acc[0] += (double)csnap[id];
            acc[1] += 1.0;
        }
    }
    __shared__ double lds[8];
    double out[2];
    block_sum<2>(acc, lds, out);
    if (threadIdx.x == 0) ref_new[x + 1] = out[1] > 0.0 ? out[0] / out[1] : ref[x + 1];
}

__global__ __launch_bounds__(256) void k_recenter(int64_t nf, int64_t stride,
                                                  const uint32_t *__restrict__ coords,
                                                  const double *__restrict__ ref,
                                                  const double *__restrict__ ref_new,
                                                  float *__restrict__ s) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nf) return;
    const int x = coords[n] & 1023;
    const double d = ref[x + 1] - ref_new[x + 1];
    s[n] += (float)(0.25 * d);
    const float d1 = (float)(0.125 * d);
    for (int i = 1; i < 7; i++) s[(int64_t)i * stride + n] += d1;
}

__global__ __launch_bounds__(1024) void k_ref_commit(int nx, double c_in, double c_out,
                                                     double *__restrict__ ref,
                                                     const double *__restrict__ ref_new,
                                                     float *__restrict__ shm,
                                                     float *__restrict__ shp) {
    for (int k = threadIdx.x; k < nx + 2; k += 1024)
        ref[k] = k == 0 ? c_in : (k == nx + 1 ? c_out : ref_new[k]);
    __syncthreads();
    for (int k = threadIdx.x; k < nx + 2; k += 1024) {
        shm[k] = k >= 1 ? (float)(0.125 * (ref[k - 1] - ref[k])) : 0.f;
        shp[k] = k <= nx ? (float)(0.125 * (ref[k + 1] - ref[k])) : 0.f;
    }
}

static lbm_status kn_recenter(const KnWs &w, const Grid &g, int64_t nf, const KnHeader &h,
                              int cur, hipStream_t s) {
    k_plane_mean<<<(unsigned)g.nx, 256, 0, s>>>(g, w.idmap, w.csnap, w.ref, w.ref_new);
    LBM_CHECK_LAUNCH();
    k_recenter<<<(unsigned)kn_blocks(nf), 256, 0, s>>>(nf, w.stride, w.coords, w.ref, w.ref_new,
                                                       w.g[cur]);
    LBM_CHECK_LAUNCH();
    k_ref_commit<<<1, 1024, 0, s>>>(g.nx, h.c_in, h.c_out, w.ref, w.ref_new, w.shm, w.shp);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

static lbm_status kn_launch(const KnWs &w, const Grid &g, int64_t nf, const KnHeader &h, int &cur,
                            int64_t steps, bool check_last, float *c_field, hipStream_t s) {
    Sweep7 a;
    a.g = g;
    a.nf = nf;
    a.stride = w.stride;
    a.launched = xcd_launch(kn_blocks(nf));
    a.coords = w.coords;
    a.idmap = w.idmap;
    a.omega = w.omega;
    a.shm = w.shm;
    a.shp = w.shp;
    a.ref = w.ref;
    a.csnap = w.csnap;
    a.c_out = c_field;
    a.partials = w.partials;
    for (int64_t t = 0; t < steps; t++) {
        a.src = w.g[cur];
        a.dst = w.g[cur ^ 1];
        if (check_last && t == steps - 1)
            k_sweep7<true><<<(unsigned)a.launched, 256, 0, s>>>(a);
        else
            k_sweep7<false><<<(unsigned)a.launched, 256, 0, s>>>(a);
        LBM_CHECK_LAUNCH();
        cur ^= 1;
    }
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_knudsen_solve(const int32_t n[3], const uint8_t *fluid,
                                        const double *pore_diam, const lbm_knudsen_params *p,
                                        lbm_knudsen_result *r, float *c_field, const float *c_init,
                                        double *plane_flux_h, void *workspace, size_t ws_bytes,
                                        void *stream) {
    LBM_REQUIRE(n, LBM_E_INVAL, "null size");
    LBM_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && n[0] <= kMaxEdge && n[1] <= kMaxEdge &&
                    n[2] <= kMaxEdge,
                LBM_E_INVAL, "sizes must lie in [1, %d]", kMaxEdge);
    LBM_REQUIRE(fluid && pore_diam && p && r && workspace, LBM_E_INVAL,
                "lbm_knudsen_solve: null argument");
    LBM_REQUIRE(p->check_every >= 1, LBM_E_INVAL, "check_every must be >= 1");
    LBM_REQUIRE(p->fixed_steps > 0 || p->max_steps > 0, LBM_E_INVAL, "no step limit given");
    LBM_REQUIRE(p->c_in != p->c_out, LBM_E_INVAL, "C_in equals C_out: no driving difference");
    LBM_REQUIRE(p->tau_ref > 0.5 && p->d_ref_nm > 0 && p->voxel_nm > 0, LBM_E_INVAL,
                "tau_ref must exceed 1/2 and d_ref, voxel size be positive");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g = make_grid(n);

    KnWs w0 = carve_kn(workspace, g, 1);
    LBM_REQUIRE(ws_bytes >= (size_t)((char *)w0.coords - (char *)workspace), LBM_E_NOMEM,
                "workspace of %zu bytes is below the grid part", ws_bytes);
    int64_t nf = 0;
    st = layout_count(g, fluid, w0.bcount, &nf, s);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(nf > 0, LBM_E_INVAL, "the fluid mask is empty");
    KnWs w = carve_kn(workspace, g, nf);
    LBM_REQUIRE(7 * w.stride <= (int64_t)UINT32_MAX, LBM_E_INVAL,
                "%lld fluid nodes exceed the 32-bit population offsets", (long long)nf);
    LBM_REQUIRE(ws_bytes >= w.bytes, LBM_E_NOMEM,
                "workspace of %zu bytes; %zu needed for %lld fluid nodes", ws_bytes, w.bytes,
                (long long)nf);
    KnHeader h;
    int64_t t0 = 0;
    int cur = 0;
    if (p->resume) {
        LBM_TRY_HIP(hipMemcpyAsync(&h, w.hdr, sizeof(h), hipMemcpyDeviceToHost, s));
        LBM_TRY_HIP(hipStreamSynchronize(s));
        LBM_REQUIRE(h.magic == kKnMagic && h.nx == n[0] && h.ny == n[1] && h.nz == n[2] &&
                        h.n_fluid == nf,
                    LBM_E_INVAL, "resume: the workspace holds no state for this geometry");
        t0 = h.steps_done;
        cur = h.cur;
    }
    st = layout_fill(g, fluid, w.bcount, w.idmap, w.coords, s);
    if (st != LBM_OK) return st;
    h.magic = kKnMagic;
    h.nx = n[0]; h.ny = n[1]; h.nz = n[2];
    h.n_fluid = nf;
    h.c_in = p->c_in;
    h.c_out = p->c_out;
    const double d_ref = p->d_ref_nm / p->voxel_nm;
    LBM_TRY_HIP(hipMemsetAsync(w.counter, 0, sizeof(unsigned long long), s));
    if (!p->resume) LBM_TRY_HIP(hipMemsetAsync(w.ref, 0, sizeof(double) * (kMaxEdge + 2), s));
    k_kn_init<<<(unsigned)kn_blocks(nf), 256, 0, s>>>(g, nf, w.stride, w.coords, pore_diam, d_ref,
                                                      p->tau_ref, c_init, w.g[cur], w.omega,
                                                      w.csnap, p->resume ? 0 : 1, w.counter,
                                                      w.partials);
    LBM_CHECK_LAUNCH();
    if (!p->resume) {
        st = kn_recenter(w, g, nf, h, cur, s);
        if (st != LBM_OK) return st;
    }
    st = reduce_partials(w.partials, kn_blocks(nf), 1, w.res + 8, s);
    if (st != LBM_OK) return st;
    unsigned long long bad = 0;
    double sum_tau = 0.0;
    LBM_TRY_HIP(hipMemcpyAsync(&bad, w.counter, sizeof(bad), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipMemcpyAsync(&sum_tau, w.res + 8, sizeof(double), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    LBM_REQUIRE(bad == 0, LBM_E_INVAL, "%llu fluid nodes have tau_g <= 1/2 (pore diameter <= 0)", bad);
    if (c_field) LBM_TRY_HIP(hipMemsetAsync(c_field, 0, sizeof(float) * g.nvox(), s));

    hipEvent_t e0, e1;
    LBM_TRY_HIP(hipEventCreate(&e0));
    LBM_TRY_HIP(hipEventCreate(&e1));
    const int64_t limit = p->fixed_steps > 0 ? p->fixed_steps : p->max_steps;
    const int nc = p->check_every;
    double sums[kKnSums] = {0, 0, 0, 0, 0};
    double resid = INFINITY, sweep_ms = 0.0;
    bool converged = false, diverged = false;
    int64_t t = 0;
    lbm_status out = LBM_OK;
    while (t < limit) {
        const int64_t abs_t = t0 + t;
        int64_t chunk = nc - (abs_t % nc);
        if (chunk > limit - t) chunk = limit - t;
        LBM_TRY_HIP(hipEventRecord(e0, s));
        out = kn_launch(w, g, nf, h, cur, chunk, true, c_field, s);
        if (out != LBM_OK) break;
        LBM_TRY_HIP(hipEventRecord(e1, s));
        out = reduce_partials(w.partials, kn_blocks(nf), kKnSums, w.res, s);
        if (out != LBM_OK) break;
        out = kn_recenter(w, g, nf, h, cur, s);
        if (out != LBM_OK) break;
        LBM_TRY_HIP(hipMemcpyAsync(sums, w.res, sizeof(sums), hipMemcpyDeviceToHost, s));
        LBM_TRY_HIP(hipStreamSynchronize(s));
        float ms = 0.f;
        LBM_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
        sweep_ms += ms;
        t += chunk;
        if (!std::isfinite(sums[0]) || !std::isfinite(sums[1]) || !std::isfinite(sums[2])) {
            diverged = true;
            break;
        }
        if ((t0 + t) % nc == 0) {
            resid = std::sqrt(sums[0]) / ((double)nc * std::sqrt(sums[1]));
            if (p->fixed_steps <= 0 && resid < p->tol) {
                converged = true;
                break;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (out != LBM_OK) return out;
    h.cur = cur;
    h.steps_done = t0 + t;
    LBM_TRY_HIP(hipMemcpyAsync(w.hdr, &h, sizeof(h), hipMemcpyHostToDevice, s));
    // link-plane fluxes of the final state
    k_plane_flux<<<(unsigned)(g.nx + 1), 256, 0, s>>>(g, w.stride, w.idmap, w.g[cur], w.shm,
                                                      w.plane);
    LBM_CHECK_LAUNCH();
    double planes[kMaxEdge + 1];
    LBM_TRY_HIP(hipMemcpyAsync(planes, w.plane, sizeof(double) * (g.nx + 1), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    if (plane_flux_h) std::memcpy(plane_flux_h, planes, sizeof(double) * (g.nx + 1));

    std::memset(r, 0, sizeof(*r));
    r->steps = t;
    r->n_fluid = nf;
    r->converged = converged;
    r->residual = resid;
    r->phi_out = sums[2];
    r->phi_in = sums[3];
    r->sum_c = sums[4];
    const double dc = p->c_in - p->c_out;
    r->Deff_lattice = sums[2] / ((double)g.ny * g.nz) * (double)(g.nx + 1) / dc;
    const double cs2 = 0.25;
    const double d_lref = cs2 * (p->tau_ref - 0.5);
    r->Deff_over_DKref = r->Deff_lattice / d_lref;
    const double R = 8.314462618, PI = 3.141592653589793;
    r->DK_ref_m2s = p->d_ref_nm * 1e-9 / 3.0 * std::sqrt(8.0 * R * p->T_K / (PI * p->M_kg_mol));
    r->Deff_m2s = r->Deff_over_DKref * r->DK_ref_m2s;
    const double eps = (double)nf / (double)g.nvox();
    r->tortuosity = eps * d_lref / r->Deff_lattice;
    r->tortuosity_local = eps * (cs2 * sum_tau / (double)nf) / r->Deff_lattice;
    double mn = planes[0], mx = planes[0], mean = 0.0;
    for (int k = 0; k <= g.nx; k++) {
        mn = planes[k] < mn ? planes[k] : mn;
        mx = planes[k] > mx ? planes[k] : mx;
        mean += planes[k];
    }
    mean /= (double)(g.nx + 1);
    r->flux_spread = mean != 0.0 ? (mx - mn) / std::fabs(mean) : INFINITY;
    r->sweep_ms = sweep_ms;
    const double updates = (double)nf * (double)t;
    r->mlups = sweep_ms > 0 ? updates / (sweep_ms * 1e3) : 0.0;
    r->gbps = sweep_ms > 0 ? updates * 60.0 / (sweep_ms * 1e-3) / 1e9 : 0.0;
    if (diverged) {
        set_error("Knudsen solve diverged (NaN/Inf) by step %lld", (long long)(t0 + t));
        return LBM_E_DIVERGED;
    }
    if (p->fixed_steps > 0 || converged) return LBM_OK;
    set_error("Knudsen solve not converged after %lld steps (residual %.3e)", (long long)t, resid);
    return LBM_W_NOT_CONVERGED;
}

static lbm_status read_kn_state(void *workspace, size_t ws_bytes, hipStream_t s, KnHeader &h,
                                Grid &g, KnWs &w) {
    LBM_REQUIRE(workspace && ws_bytes >= sizeof(KnHeader), LBM_E_INVAL, "null workspace");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    LBM_TRY_HIP(hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    LBM_REQUIRE(h.magic == kKnMagic, LBM_E_INVAL, "the workspace holds no Knudsen state");
    const int32_t n[3] = {h.nx, h.ny, h.nz};
    g = make_grid(n);
    w = carve_kn(workspace, g, h.n_fluid);
    LBM_REQUIRE(ws_bytes >= w.bytes, LBM_E_NOMEM, "workspace smaller than its state");
    return LBM_OK;
}

extern "C" lbm_status lbm_knudsen_step(void *workspace, size_t ws_bytes, int64_t steps, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    KnHeader h;
    Grid g;
    KnWs w;
    lbm_status st = read_kn_state(workspace, ws_bytes, s, h, g, w);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(steps >= 0, LBM_E_INVAL, "negative step count");
    int cur = h.cur;
    st = kn_launch(w, g, h.n_fluid, h, cur, steps, false, nullptr, s);
    if (st != LBM_OK) return st;
    h.cur = cur;
    h.steps_done += steps;
    LBM_TRY_HIP(hipMemcpyAsync(w.hdr, &h, sizeof(h), hipMemcpyHostToDevice, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return LBM_OK;
}

extern "C" lbm_status lbm_knudsen_sample(void *workspace, size_t ws_bytes, const int64_t *vox_h,
                                         int64_t count, double *g_h, double *tau_h,
                                         uint8_t *fluid_h, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    LBM_REQUIRE(vox_h && g_h && tau_h && fluid_h, LBM_E_INVAL, "lbm_knudsen_sample: null argument");
    LBM_REQUIRE(count >= 0 && count <= kKnSampleMax, LBM_E_INVAL, "count must lie in [0, %d]",
                kKnSampleMax);
    KnHeader h;
    Grid g;
    KnWs w;
    lbm_status st = read_kn_state(workspace, ws_bytes, s, h, g, w);
    if (st != LBM_OK) return st;
    if (count == 0) return LBM_OK;
    for (int64_t i = 0; i < count; i++)
        LBM_REQUIRE(vox_h[i] >= 0 && vox_h[i] < g.nvox(), LBM_E_INVAL, "voxel %lld out of range",
                    (long long)vox_h[i]);
    LBM_TRY_HIP(hipMemcpyAsync(w.samp_vox, vox_h, sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
    k_kn_sample<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(g, count, w.stride, w.samp_vox,
                                                               w.idmap, w.g[h.cur], w.omega,
                                                               w.ref,
                                                               w.samp_out, w.samp_flag);
    LBM_CHECK_LAUNCH();
    std::vector<double> tmp((size_t)count * 8);
    LBM_TRY_HIP(hipMemcpyAsync(tmp.data(), w.samp_out, sizeof(double) * 8 * count, hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipMemcpyAsync(fluid_h, w.samp_flag, count, hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < count; i++) {
        for (int k = 0; k < 7; k++) g_h[i * 7 + k] = tmp[i * 8 + k];
        tau_h[i] = tmp[i * 8 + 7];
    }
    return LBM_OK;
}
