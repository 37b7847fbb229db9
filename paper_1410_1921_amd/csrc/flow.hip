// D3Q19 flow solve: fused pull-stream + BGK collision + Guo body force with half-way
// bounce-back, on the sparse fluid-node list (Section 3.1, Eqs. 1-3, 8-9; Section 3.3;
// Darcy's law, Eq. 13).
//
// Storage: structure of arrays f[i][node] of f_i - w_i in binary32 ("shifted"
// populations: the flow signal lives in deviations of order 1e-6 from w_i, which
// binary32 keeps to ~1e-13 absolute once the constant w_i is removed).  Two buffers,
// ping-pong.  Per fluid-node update the method moves 19 loads + 19 stores of 4 bytes.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "lbm_internal.h"

namespace lbm {

// D3Q19 velocities in the column order of the paper's transformation matrix.
#define LBM_D3Q19_TABLES                                                                      \
    [[maybe_unused]] constexpr int EX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1,              \
                                             1, -1, 1, -1, 0, 0, 0, 0};                       \
    [[maybe_unused]] constexpr int EY[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1,              \
                                             0, 0, 0, 0, 1, -1, 1, -1};                       \
    [[maybe_unused]] constexpr int EZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0,                \
                                             1, 1, -1, -1, 1, 1, -1, -1};                     \
    [[maybe_unused]] constexpr int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8,                  \
                                              7, 14, 13, 12, 11, 18, 17, 16, 15};

constexpr uint64_t kFlowMagic = 0x4c424d464c4f5731ull;  // "LBMFLOW1"
constexpr int kFlowSums = 6;      // |du|^2, |u|^2, rho u (3), rho - 1
constexpr int kSampleMax = 65536;

struct FlowHeader {
    uint64_t magic;
    int32_t nx, ny, nz, cur;
    int64_t n_fluid, steps_done;
    double tau, force[3];
    int32_t variant, reserved;
};

struct FlowWs {
    FlowHeader *hdr;
    unsigned long long *counter;
    double *res;
    int32_t *total;
    RankWord *rank;
    int64_t *samp_vox;
    double *samp_out;
    uint8_t *samp_flag;
    uint32_t *coords;
    float *f[2];
    float *usnap;
    double *partials;
    int64_t stride;  // distance between population arrays (elements)
    size_t bytes;
};

static int64_t blocks_for(int64_t nf) { return (nf + 255) / 256; }

static FlowWs carve_flow(void *base, const Grid &g, int64_t nf) {
    FlowWs w;
    Carver c(base);
    w.hdr = c.take<FlowHeader>(1);
    w.counter = c.take<unsigned long long>(4);
    w.res = c.take<double>(32);
    w.total = c.take<int32_t>(1);
    w.rank = c.take<RankWord>(g.nsegs());
    w.samp_vox = c.take<int64_t>(kSampleMax);
    w.samp_out = c.take<double>((size_t)kSampleMax * 19);
    w.samp_flag = c.take<uint8_t>(kSampleMax);
    int64_t nfp = nf < 1 ? 1 : nf;
    w.stride = (nfp + 63) / 64 * 64;
    w.coords = c.take<uint32_t>(nfp);
    w.f[0] = c.take<float>((size_t)19 * w.stride);
    w.f[1] = c.take<float>((size_t)19 * w.stride);
    w.usnap = c.take<float>((size_t)3 * w.stride);
    w.partials = c.take<double>((size_t)xcd_launch(blocks_for(nfp)) * kFlowSums);
    w.bytes = c.off;
    return w;
}

size_t flow_ws_bytes(const Grid &g, int64_t nf) { return carve_flow(nullptr, g, nf).bytes; }

struct Sweep19 {
    Grid g;
    int64_t nf, stride, launched;
    const uint32_t *__restrict__ coords;
    const RankWord *__restrict__ rank;
    const float *__restrict__ src;
    float *__restrict__ dst;
    float omega, fpre, Fx, Fy, Fz;
    int remap;                         // XCD-contiguous workgroup order
    // check variant
    float *__restrict__ usnap;
    float *__restrict__ u_out;
    double *__restrict__ partials;
    int update_snap;
};

// Kernel variants (chosen per solve from the working-set size, or forced):
//   REMAP: XCD-contiguous workgroup order, so neighbouring rows share an L2;
//   NT: populations are written with streaming (non-temporal) stores; right when the
//     arrays far exceed the 256 MB Infinity Cache, wrong when they fit in it.

// The update of fluid node n at (x, y, z) whose 18 pull sources are resolved: ids[i] is
// the node at x - e_i, or -1 when that voxel is solid (half-way bounce-back).
template <bool CHECK, bool NT>
__device__ inline void node19(const Sweep19 &a, int64_t n, int x, int y, int z,
                              const int (&ids)[19], double (&acc)[kFlowSums]) {
    LBM_D3Q19_TABLES
    constexpr float W0 = 1.0f / 3.0f, W1 = 1.0f / 18.0f, W2 = 1.0f / 36.0f;
    uint32_t off[19];
    off[0] = (uint32_t)n;
#pragma unroll
    for (int i = 1; i < 19; i++)
        off[i] = ids[i] >= 0 ? (uint32_t)(i * a.stride + ids[i]) : (uint32_t)(OPP[i] * a.stride + n);
    float f[19];
#pragma unroll
    for (int i = 0; i < 19; i++) f[i] = a.src[off[i]];

    float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < 19; i++) {
        drho += f[i];
        if (EX[i]) jx += EX[i] > 0 ? f[i] : -f[i];
        if (EY[i]) jy += EY[i] > 0 ? f[i] : -f[i];
        if (EZ[i]) jz += EZ[i] > 0 ? f[i] : -f[i];
    }
    const float rho = 1.0f + drho;
    const float inv = 1.0f / rho;
    const float mx = jx + 0.5f * a.Fx, my = jy + 0.5f * a.Fy, mz = jz + 0.5f * a.Fz;
    const float ux = mx * inv, uy = my * inv, uz = mz * inv;
    const float uu15 = 1.5f * (ux * ux + uy * uy + uz * uz);
    const float uF = ux * a.Fx + uy * a.Fy + uz * a.Fz;
#pragma unroll
    for (int i = 0; i < 19; i++) {
        const float w = i == 0 ? W0 : (i < 7 ? W1 : W2);
        const float eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        const float eF = EX[i] * a.Fx + EY[i] * a.Fy + EZ[i] * a.Fz;
        const float feq = w * (drho + rho * (3.0f * eu + 4.5f * eu * eu - uu15));
        const float src = a.fpre * w * (3.0f * (eF - uF) + 9.0f * eu * eF);
        const float out = f[i] - a.omega * (f[i] - feq) + src;
        if (NT)
            __builtin_nontemporal_store(out, &a.dst[(int64_t)i * a.stride + n]);
        else
            a.dst[(int64_t)i * a.stride + n] = out;
    }
    if (CHECK) {
        const double dux = (double)ux - (double)a.usnap[n];
        const double duy = (double)uy - (double)a.usnap[a.stride + n];
        const double duz = (double)uz - (double)a.usnap[2 * a.stride + n];
        acc[0] += dux * dux + duy * duy + duz * duz;
        acc[1] += (double)ux * ux + (double)uy * uy + (double)uz * uz;
        acc[2] += (double)jx + 0.5 * (double)a.Fx;
        acc[3] += (double)jy + 0.5 * (double)a.Fy;
        acc[4] += (double)jz + 0.5 * (double)a.Fz;
        acc[5] += drho;
        if (a.update_snap) {
            a.usnap[n] = ux;
            a.usnap[a.stride + n] = uy;
            a.usnap[2 * a.stride + n] = uz;
        }
        if (a.u_out) {
            const int64_t v = a.g.lin(x, y, z), nv = a.g.nvox();
            a.u_out[v] = ux;
            a.u_out[nv + v] = uy;
            a.u_out[2 * nv + v] = uz;
        }
    }
}

template <int NV>
__device__ inline void write_partials(double (&acc)[NV], int64_t row, bool valid, double *part) {
    __shared__ double lds[4 * NV];
    double out[NV];
    block_sum<NV>(acc, lds, out);
    if (threadIdx.x == 0 && valid)
#pragma unroll
        for (int k = 0; k < NV; k++) part[row * NV + k] = out[k];
}

// One stream-collide step, one fluid node per thread, neighbour ids gathered from the
// global id map.  CHECK also forms the FP64 partial sums of the convergence check and
// writes the velocity snapshot / field.
template <bool CHECK, bool NT>
__global__ __launch_bounds__(256) void k_sweep19(Sweep19 a) {
    LBM_D3Q19_TABLES
    const int64_t lb = a.remap ? xcd_block(blockIdx.x, a.launched) : (int64_t)blockIdx.x;
    const int64_t n = lb * 256 + threadIdx.x;
    double acc[kFlowSums] = {0, 0, 0, 0, 0, 0};
    if (n < a.nf) {
        const uint32_t c = a.coords[n];
        const int x = c & 1023, y = (c >> 10) & 1023, z = c >> 20;
        const Grid &g = a.g;
        // per-axis pieces of the rank word and bit of x-1, x, x+1 (periodic), etc.
        int xs[3], ys[3], zs[3];
        xs[0] = x == 0 ? g.nx - 1 : x - 1; xs[1] = x; xs[2] = x == g.nx - 1 ? 0 : x + 1;
        ys[0] = y == 0 ? g.ny - 1 : y - 1; ys[1] = y; ys[2] = y == g.ny - 1 ? 0 : y + 1;
        zs[0] = z == 0 ? g.nz - 1 : z - 1; zs[1] = z; zs[2] = z == g.nz - 1 ? 0 : z + 1;
        int wx[3], wy[3], wz[3], bx[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            wx[k] = xs[k] >> kSegLog;
            wy[k] = ys[k] * g.nseg;
            wz[k] = zs[k] * (g.ny * g.nseg);
            bx[k] = xs[k] & (kSeg - 1);
        }
        // the 18 rank words are loaded as one batch, then the 19 populations as another
        RankWord rw[19];
#pragma unroll
        for (int i = 1; i < 19; i++) rw[i] = a.rank[wx[1 - EX[i]] + wy[1 - EY[i]] + wz[1 - EZ[i]]];
        int ids[19];
        ids[0] = 0;
#pragma unroll
        for (int i = 1; i < 19; i++) ids[i] = rank_lookup(rw[i], bx[1 - EX[i]]);
        node19<CHECK, NT>(a, n, x, y, z, ids, acc);
    }
    if (CHECK) write_partials<kFlowSums>(acc, lb, lb * 256 < a.nf, a.partials);
}

// f - w_i at the equilibrium of rho = 1 and u_init (zero without it); the snapshot
// starts at u_init.
__global__ __launch_bounds__(256) void k_flow_init(Grid g, int64_t nf, int64_t stride,
                                                   const uint32_t *__restrict__ coords,
                                                   const float *__restrict__ u_init,
                                                   float *__restrict__ f,
                                                   float *__restrict__ usnap) {
    LBM_D3Q19_TABLES
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nf) return;
    float ux = 0.f, uy = 0.f, uz = 0.f;
    if (u_init) {
        const uint32_t c = coords[n];
        const int64_t v = g.lin(c & 1023, (c >> 10) & 1023, c >> 20), nv = g.nvox();
        ux = u_init[v]; uy = u_init[nv + v]; uz = u_init[2 * nv + v];
    }
    const float uu15 = 1.5f * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int i = 0; i < 19; i++) {
        const float w = i == 0 ? 1.0f / 3.0f : (i < 7 ? 1.0f / 18.0f : 1.0f / 36.0f);
        const float eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        f[(int64_t)i * stride + n] = w * (3.0f * eu + 4.5f * eu * eu - uu15);
    }
    usnap[n] = ux; usnap[stride + n] = uy; usnap[2 * stride + n] = uz;
}

__global__ void k_flow_sample(Grid g, int64_t count, int64_t stride,
                              const int64_t *__restrict__ vox, const RankWord *__restrict__ rank,
                              const float *__restrict__ f, double *__restrict__ out,
                              uint8_t *__restrict__ flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const int64_t v = vox[s];
    const int x = (int)(v % g.nx), y = (int)((v / g.nx) % g.ny), z = (int)(v / ((int64_t)g.nx * g.ny));
    const int id = node_at(rank, g, x, y, z);
    flag[s] = id >= 0;
    for (int i = 0; i < 19; i++) out[s * 19 + i] = id >= 0 ? (double)f[(int64_t)i * stride + id] : 0.0;
}

// Kernel variant: explicit bits, or chosen from the working set: when the two
// population arrays exceed ~3/4 of the 256 MB Infinity Cache the sweep streams from HBM
// (plain workgroup order, non-temporal stores), otherwise it keeps the state in the cache
// (XCD-contiguous order, ordinary stores).
struct Variant19 {
    bool remap, nt;
};

static Variant19 pick_variant(int32_t v, int64_t stride) {
    Variant19 m;
    if (v & LBM_VARIANT_EXPLICIT) {
        m.remap = v & LBM_VARIANT_REMAP;
        m.nt = v & LBM_VARIANT_NTSTORE;
        return m;
    }
    const bool stream = 2.0 * 19 * 4 * (double)stride > 192e6;
    m.remap = !stream;
    m.nt = stream;
    return m;
}

template <bool CHECK>
static void launch19(const Sweep19 &a, const Variant19 &m, hipStream_t s) {
    const unsigned grid = (unsigned)a.launched;
    if (m.nt) k_sweep19<CHECK, true><<<grid, 256, 0, s>>>(a);
    else k_sweep19<CHECK, false><<<grid, 256, 0, s>>>(a);
}

static lbm_status launch_sweeps(const FlowWs &w, const Grid &g, int64_t nf, const FlowHeader &h,
                                const Variant19 &m, int &cur, int64_t steps, bool check_last,
                                float *u_out, hipStream_t s) {
    Sweep19 a;
    a.g = g;
    a.nf = nf;
    a.stride = w.stride;
    a.launched = xcd_launch(blocks_for(nf));
    a.coords = w.coords;
    a.rank = w.rank;
    a.omega = (float)(1.0 / h.tau);
    a.fpre = (float)(1.0 - 0.5 / h.tau);
    a.Fx = (float)h.force[0];
    a.Fy = (float)h.force[1];
    a.Fz = (float)h.force[2];
    a.remap = m.remap;
    a.usnap = w.usnap;
    a.u_out = u_out;
    a.partials = w.partials;
    a.update_snap = 1;
    for (int64_t t = 0; t < steps; t++) {
        a.src = w.f[cur];
        a.dst = w.f[cur ^ 1];
        if (check_last && t == steps - 1)
            launch19<true>(a, m, s);
        else
            launch19<false>(a, m, s);
        LBM_CHECK_LAUNCH();
        cur ^= 1;
    }
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

static lbm_status validate_n(const int32_t n[3]) {
    LBM_REQUIRE(n, LBM_E_INVAL, "null size");
    LBM_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && n[0] <= kMaxEdge && n[1] <= kMaxEdge &&
                    n[2] <= kMaxEdge,
                LBM_E_INVAL, "sizes must lie in [1, %d], got %d x %d x %d", kMaxEdge, n[0], n[1], n[2]);
    return LBM_OK;
}

namespace lbm {
size_t flow_ws_bytes_n(const int32_t n[3], int64_t nf) {
    Grid g = make_grid(n);
    return flow_ws_bytes(g, nf < 0 ? g.nvox() : nf);
}
}  // namespace lbm

extern "C" lbm_status lbm_flow_solve(const int32_t n[3], const uint8_t *fluid,
                                     const lbm_flow_params *p, lbm_flow_result *r,
                                     float *u_out, const float *u_init, void *workspace,
                                     size_t ws_bytes, void *stream) {
    lbm_status st = validate_n(n);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(fluid && p && r && workspace, LBM_E_INVAL, "lbm_flow_solve: null argument");
    LBM_REQUIRE(p->tau > 0.5 && std::isfinite(p->tau), LBM_E_INVAL, "tau must exceed 1/2");
    LBM_REQUIRE(p->check_every >= 1, LBM_E_INVAL, "check_every must be >= 1");
    LBM_REQUIRE(p->fixed_steps > 0 || p->max_steps > 0, LBM_E_INVAL, "no step limit given");
    LBM_REQUIRE(p->storage == LBM_STORE_FP32, LBM_E_INVAL, "unknown storage %d", p->storage);
    LBM_REQUIRE((p->variant & ~kVariantBits) == 0, LBM_E_INVAL, "unknown variant bits 0x%x",
                p->variant);
    st = check_device();
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g = make_grid(n);

    // the grid-sized part of the workspace comes first: count the fluid nodes there
    FlowWs w0 = carve_flow(workspace, g, 1);
    LBM_REQUIRE(ws_bytes >= (size_t)((char *)w0.coords - (char *)workspace), LBM_E_NOMEM,
                "workspace of %zu bytes is below the grid part", ws_bytes);
    int64_t nf = 0;
    st = layout_count(g, fluid, w0.rank, w0.total, &nf, s);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(nf > 0, LBM_E_INVAL, "the fluid mask is empty");
    FlowWs w = carve_flow(workspace, g, nf);
    LBM_REQUIRE(19 * w.stride <= (int64_t)UINT32_MAX, LBM_E_INVAL,
                "%lld fluid nodes exceed the 32-bit population offsets", (long long)nf);
    LBM_REQUIRE(ws_bytes >= w.bytes, LBM_E_NOMEM,
                "workspace of %zu bytes; %zu needed for %lld fluid nodes", ws_bytes, w.bytes,
                (long long)nf);

    FlowHeader h;
    int64_t t0 = 0;
    int cur = 0;
    if (p->resume) {
        LBM_TRY_HIP(hipMemcpyAsync(&h, w.hdr, sizeof(h), hipMemcpyDeviceToHost, s));
        LBM_TRY_HIP(hipStreamSynchronize(s));
        LBM_REQUIRE(h.magic == kFlowMagic && h.nx == n[0] && h.ny == n[1] && h.nz == n[2] &&
                        h.n_fluid == nf,
                    LBM_E_INVAL, "resume: the workspace holds no state for this geometry");
        t0 = h.steps_done;
        cur = h.cur;
    }
    st = layout_fill(g, w.rank, w.coords, s);
    if (st != LBM_OK) return st;
    h.magic = kFlowMagic;
    h.nx = n[0]; h.ny = n[1]; h.nz = n[2];
    h.n_fluid = nf;
    h.tau = p->tau;
    h.variant = p->variant;
    h.reserved = 0;
    const Variant19 mode = pick_variant(p->variant, w.stride);
    for (int a = 0; a < 3; a++) h.force[a] = p->force[a];
    if (!p->resume) {
        k_flow_init<<<(unsigned)blocks_for(nf), 256, 0, s>>>(g, nf, w.stride, w.coords, u_init,
                                                             w.f[0], w.usnap);
        LBM_CHECK_LAUNCH();
    }
    if (u_out) LBM_TRY_HIP(hipMemsetAsync(u_out, 0, sizeof(float) * 3 * g.nvox(), s));

    hipEvent_t e0, e1;
    LBM_TRY_HIP(hipEventCreate(&e0));
    LBM_TRY_HIP(hipEventCreate(&e1));
    const int64_t limit = p->fixed_steps > 0 ? p->fixed_steps : p->max_steps;
    const int nc = p->check_every;
    double sums[kFlowSums] = {0, 0, 0, 0, 0, 0};
    double resid = INFINITY, sweep_ms = 0.0;
    bool converged = false, diverged = false;
    int64_t t = 0;
    lbm_status out = LBM_OK;
    while (t < limit) {
        // run to the next check (a multiple of n_c counted from the first step) or the limit
        const int64_t abs_t = t0 + t;
        int64_t chunk = nc - (abs_t % nc);
        if (chunk > limit - t) chunk = limit - t;
        LBM_TRY_HIP(hipEventRecord(e0, s));
        out = launch_sweeps(w, g, nf, h, mode, cur, chunk, true, u_out, s);
        if (out != LBM_OK) break;
        LBM_TRY_HIP(hipEventRecord(e1, s));
        out = reduce_partials(w.partials, blocks_for(nf), kFlowSums, w.res, s);
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
    LBM_TRY_HIP(hipStreamSynchronize(s));

    const double nvox = (double)g.nvox();
    const double nu = (p->tau - 0.5) / 3.0;
    std::memset(r, 0, sizeof(*r));
    r->steps = t;
    r->n_fluid = nf;
    r->converged = converged;
    r->residual = resid;
    for (int a = 0; a < 3; a++) r->mean_rho_u[a] = sums[2 + a] / nvox;
    r->mass_dev = sums[5];
    r->k_lattice = nu * r->mean_rho_u[0] / p->force[0];
    const double dx = p->voxel_nm * 1e-9;
    r->k_m2 = r->k_lattice * dx * dx;
    r->k_mD = r->k_m2 / 9.869233e-16;
    r->sweep_ms = sweep_ms;
    const double updates = (double)nf * (double)t;
    r->mlups = sweep_ms > 0 ? updates / (sweep_ms * 1e3) : 0.0;
    r->gbps = sweep_ms > 0 ? updates * 152.0 / (sweep_ms * 1e-3) / 1e9 : 0.0;
    if (diverged) {
        set_error("flow solve diverged (NaN/Inf) by step %lld", (long long)(t0 + t));
        return LBM_E_DIVERGED;
    }
    if (p->fixed_steps > 0 || converged) return LBM_OK;
    set_error("flow solve not converged after %lld steps (residual %.3e)", (long long)t, resid);
    return LBM_W_NOT_CONVERGED;
}

static lbm_status read_flow_state(void *workspace, size_t ws_bytes, hipStream_t s, FlowHeader &h,
                                  Grid &g, FlowWs &w) {
    LBM_REQUIRE(workspace && ws_bytes >= sizeof(FlowHeader), LBM_E_INVAL, "null workspace");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    LBM_TRY_HIP(hipMemcpyAsync(&h, workspace, sizeof(h), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    LBM_REQUIRE(h.magic == kFlowMagic, LBM_E_INVAL, "the workspace holds no flow state");
    const int32_t n[3] = {h.nx, h.ny, h.nz};
    g = make_grid(n);
    w = carve_flow(workspace, g, h.n_fluid);
    LBM_REQUIRE(ws_bytes >= w.bytes, LBM_E_NOMEM, "workspace smaller than its state");
    return LBM_OK;
}

extern "C" lbm_status lbm_flow_step(void *workspace, size_t ws_bytes, int64_t steps, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    FlowHeader h;
    Grid g;
    FlowWs w;
    lbm_status st = read_flow_state(workspace, ws_bytes, s, h, g, w);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(steps >= 0, LBM_E_INVAL, "negative step count");
    int cur = h.cur;
    st = launch_sweeps(w, g, h.n_fluid, h, pick_variant(h.variant, w.stride), cur, steps, false,
                       nullptr, s);
    if (st != LBM_OK) return st;
    h.cur = cur;
    h.steps_done += steps;
    LBM_TRY_HIP(hipMemcpyAsync(w.hdr, &h, sizeof(h), hipMemcpyHostToDevice, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return LBM_OK;
}

extern "C" lbm_status lbm_flow_sample(void *workspace, size_t ws_bytes, const int64_t *vox_h,
                                      int64_t count, double *f_h, uint8_t *fluid_h, void *stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    LBM_REQUIRE(vox_h && f_h && fluid_h, LBM_E_INVAL, "lbm_flow_sample: null argument");
    LBM_REQUIRE(count >= 0 && count <= kSampleMax, LBM_E_INVAL, "count must lie in [0, %d]",
                kSampleMax);
    FlowHeader h;
    Grid g;
    FlowWs w;
    lbm_status st = read_flow_state(workspace, ws_bytes, s, h, g, w);
    if (st != LBM_OK) return st;
    if (count == 0) return LBM_OK;
    for (int64_t i = 0; i < count; i++)
        LBM_REQUIRE(vox_h[i] >= 0 && vox_h[i] < g.nvox(), LBM_E_INVAL, "voxel %lld out of range",
                    (long long)vox_h[i]);
    LBM_TRY_HIP(hipMemcpyAsync(w.samp_vox, vox_h, sizeof(int64_t) * count, hipMemcpyHostToDevice, s));
    k_flow_sample<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(g, count, w.stride, w.samp_vox,
                                                                 w.rank, w.f[h.cur], w.samp_out,
                                                                 w.samp_flag);
    LBM_CHECK_LAUNCH();
    LBM_TRY_HIP(hipMemcpyAsync(f_h, w.samp_out, sizeof(double) * 19 * count, hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipMemcpyAsync(fluid_h, w.samp_flag, count, hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return LBM_OK;
}
