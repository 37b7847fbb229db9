// D3Q7 Knudsen mass-transport solve: fused pull-stream + BGK collision with the local
// relaxation time of each node (Section 3.2, Eqs. 10-12 on D3Q7), bounce-back at solid
// links, periodic in y and z, equilibrium ghost planes at x = -1 and x = nx (Section
// 3.3), and the outlet-plane flux of Eq. 14.
//
// Storage: s_i(node) = g_i - w_i C_ref(x) in binary32, at element popq(q, i, node)
// below, where C_ref(x) is a reference profile along x (the "frame" of the state): the
// mean concentration of plane x at the latest convergence check (ghost planes:
// C_ref(-1) = C_in, C_ref(nx) = C_out).  The collision is carried out on these
// deviations, so rounding acts on numbers far smaller than g itself: both the
// transient front and the steady state keep binary32 errors
// near 1e-7 relative, where storing g directly freezes the iteration (per-step changes
// below half an ulp) up to ~1e-3 away from its steady state on long channels.
// A new frame costs no extra pass: the first sweep after a check reads the state in the
// old frame and writes it in the new one, through a per-x table of reference shifts.
// 1/tau_g per node in binary32.  Per fluid-node update: 7 loads + 7 stores of 4 bytes +
// 4 bytes of 1/tau_g.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lbm_internal.h"

namespace lbm {

// D3Q7: rest, then +x, -x, +y, -y, +z, -z.
#define LBM_D3Q7_TABLES [[maybe_unused]] constexpr int OPP[7] = {0, 2, 1, 4, 3, 6, 5};

constexpr uint64_t kKnMagic = 0x4c424d4b4e554435ull;  // "LBMKNUD5"
constexpr int kKnSums = 5;  // |dC|^2, C^2, Phi_out, Phi_in, C
constexpr int kKnSampleMax = 65536;
constexpr float kW0 = 0.25f, kW1 = 0.125f;
// The paper's D3Q19 diffusion weights a_i (Section 3.2), binary32.
__host__ __device__ inline float a19(int i) {
    return i == 0 ? 1.f / 3.f : (i < 7 ? 1.f / 18.f : 1.f / 36.f);
}
constexpr int kPlaneParts = 16;  // workgroups per plane in the plane-mean pass

struct KnHeader {
    uint64_t magic;
    int32_t nx, ny, nz, cur;
    int64_t n_fluid, steps_done;
    double c_in, c_out;
    int32_t frame;    // reference profile the stored state is relative to
    int32_t variant;  // LBM_VARIANT_* of the solve
    int32_t lattice;  // LBM_LATTICE_*
    int32_t pad;
    double tau_ref, d_ref;  // Eq. 12 parameters the relaxation times were formed with
};

// Populations per node and the weights of a lattice: D3Q7 (rest 1/4, faces 1/8) or the
// paper's D3Q19 (1/3, 1/18, 1/36).
static int kn_q(int32_t lattice) { return lattice == LBM_LATTICE_D3Q19 ? 19 : 7; }
// Scale of the frame shift tables: D3Q7 stores w_1 times the reference differences (all
// its moving weights are 1/8), D3Q19 the differences themselves (the sweep multiplies by
// a_i).
static double kn_shift_scale(int32_t lattice) { return lattice == LBM_LATTICE_D3Q19 ? 1.0 : 0.125; }

// Reference shifts for a sweep from frame `in` to frame `out`, per x (index x + 1), times
// the lattice's shift scale:
// t0 = ref_in(x) - ref_out(x)      populations with e_x = 0 and bounced ones
// tm = ref_in(x - 1) - ref_out(x)  populations with e_x = +1, streamed from x - 1
// tp = ref_in(x + 1) - ref_out(x)  populations with e_x = -1, streamed from x + 1
struct Shift {
    float t0, tm, tp, pad;
};

struct KnWs {
    KnHeader *hdr;
    unsigned long long *counter;
    double *res;
    double *plane;
    int32_t *total;
    RankWord *rank;
    int64_t *samp_vox;
    double *samp_out;
    uint8_t *samp_flag;
    uint32_t *coords;
    float *g[2];
    float *omega;
    float *csnap;
    double *partials;
    double *ref[2];    // the two reference profiles, index x + 1 for x = -1..nx
    Shift *steady[2];  // shifts within each frame (t0 = 0)
    Shift *trans;      // shifts from the current frame to the other one
    double *part;      // plane-mean partial sums [nx][kPlaneParts][2]
    double *fpart;     // link-plane flux partial sums [nx + 1][kPlaneParts]
    int64_t stride;
    size_t bytes;
};

static int64_t kn_blocks(int64_t nf) { return (nf + 255) / 256; }

// Population i of fluid node m on a lattice of q velocities: blocks of 256 nodes, each
// with its q arrays of 256 side by side, so that the populations a wave pulls lie in few
// pages (the same layout as the flow lattice; 2.5 % faster than one array of the whole
// lattice per direction for D3Q7 at 128^3, 11 % at 512^3).
__host__ __device__ inline int64_t popq(int q, int i, int64_t m) {
    return ((m >> 8) * q + i) * 256 + (m & 255);
}

static KnWs carve_kn(void *base, const Grid &g, int64_t nf, int q) {
    KnWs w;
    Carver c(base);
    w.hdr = c.take<KnHeader>(1);
    w.counter = c.take<unsigned long long>(4);
    w.res = c.take<double>(32);
    w.plane = c.take<double>(kMaxEdge + 1);
    w.total = c.take<int32_t>(1);
    w.rank = c.take<RankWord>(g.nsegs());
    w.samp_vox = c.take<int64_t>(kKnSampleMax);
    w.samp_out = c.take<double>((size_t)kKnSampleMax * 20);
    w.samp_flag = c.take<uint8_t>(kKnSampleMax);
    for (int f = 0; f < 2; f++) w.ref[f] = c.take<double>(kMaxEdge + 2);
    for (int f = 0; f < 2; f++) w.steady[f] = c.take<Shift>(kMaxEdge + 2);
    w.trans = c.take<Shift>(kMaxEdge + 2);
    w.part = c.take<double>((size_t)kMaxEdge * kPlaneParts * 2);
    w.fpart = c.take<double>((size_t)(kMaxEdge + 1) * kPlaneParts);
    int64_t nfp = nf < 1 ? 1 : nf;
    w.stride = (nfp + 255) / 256 * 256;  // whole blocks of 256 nodes (popq)
    w.coords = c.take<uint32_t>(nfp);
    w.g[0] = c.take<float>((size_t)q * w.stride);
    w.g[1] = c.take<float>((size_t)q * w.stride);
    w.omega = c.take<float>(w.stride);
    w.csnap = c.take<float>(w.stride);
    w.partials = c.take<double>((size_t)xcd_launch(kn_blocks(nfp)) * kKnSums);
    w.bytes = c.off;
    return w;
}

size_t knudsen_ws_bytes_n(const int32_t n[3], int64_t nf, int q) {
    Grid g = make_grid(n);
    return carve_kn(nullptr, g, nf < 0 ? g.nvox() : nf, q).bytes;
}

struct Sweep7 {
    Grid g;
    int64_t nf, stride, launched;
    int64_t launched_live;             // batched solves: blocks of the launch with work
    const uint32_t *__restrict__ coords;
    const RankWord *__restrict__ rank;
    const float *__restrict__ omega;
    const float *__restrict__ src;
    float *__restrict__ dst;
    const Shift *__restrict__ shift;
    int64_t chunk;                     // XCD remap run length in blocks (0: none)
    // check variant
    const double *__restrict__ ref_out;
    float *__restrict__ csnap;
    float *__restrict__ c_out;
    double *__restrict__ partials;
};

// The update of fluid node n at (x, y, z) with its 6 pull sources resolved: ids[i] is the
// node at x - e_i, -1 when that voxel is solid (bounce back), -2 beyond an x face (ghost
// plane).
template <bool CHECK, bool NT, class Off>
__device__ inline void node7(const Sweep7 &a, int64_t n, int x, int y, int z, const int (&ids)[7],
                             double (&acc)[kKnSums]) {
    LBM_D3Q7_TABLES
    const float om = a.omega[n];
    const Shift sh = a.shift[x + 1];
    // element offsets popq(q, i, node): 32-bit while q * stride fits, 64-bit beyond
    Off off[7];
    off[0] = (Off)popq(7, 0, n);
#pragma unroll
    for (int i = 1; i < 7; i++)
        off[i] = ids[i] >= 0 ? (Off)popq(7, i, ids[i]) : (Off)popq(7, OPP[i], n);
    float ai[7];
#pragma unroll
    for (int i = 0; i < 7; i++) ai[i] = a.src[off[i]];
    // incoming deviations, moved onto this node's output reference w_i C_ref(x): a
    // population streamed along +-x from a fluid neighbour (or a ghost plane, whose
    // deviation is 0) also changes plane
    if (ids[1] == -2) ai[1] = 0.f;
    if (ids[2] == -2) ai[2] = 0.f;
    ai[0] += 2.f * sh.t0;
    ai[1] += ids[1] == -1 ? sh.t0 : sh.tm;
    ai[2] += ids[2] == -1 ? sh.t0 : sh.tp;
#pragma unroll
    for (int i = 3; i < 7; i++) ai[i] += sh.t0;
    float cdev = 0.f;  // C - C_ref(x)
#pragma unroll
    for (int i = 0; i < 7; i++) cdev += ai[i];
    float so[7];
#pragma unroll
    for (int i = 0; i < 7; i++) {
        const float w = i == 0 ? kW0 : kW1;
        so[i] = ai[i] - om * (ai[i] - w * cdev);
        if (NT)
            __builtin_nontemporal_store(so[i], &a.dst[popq(7, i, n)]);
        else
            a.dst[popq(7, i, n)] = so[i];
    }
    if (CHECK) {
        const double conc = a.ref_out[x + 1] + (double)cdev;
        const double d = conc - (double)a.csnap[n];
        acc[0] += d * d;
        acc[1] += conc * conc;
        // net +x flux into the outlet ghost plane and out of the inlet one, as streamed
        // (both sides in the node's output frame)
        if (ids[2] == -2) acc[2] += (double)so[1] - (double)sh.tp;
        if (ids[1] == -2) acc[3] += (double)sh.tm - (double)so[2];
        acc[4] += conc;
        a.csnap[n] = (float)conc;
        if (a.c_out) a.c_out[a.g.lin(x, y, z)] = (float)conc;
    }
}

template <int NV>
__device__ inline void write_partials7(double (&acc)[NV], int64_t row, bool valid, double *part) {
    __shared__ double lds[4 * NV];
    double out[NV];
    block_sum<NV>(acc, lds, out);
    if (threadIdx.x == 0 && valid)
#pragma unroll
        for (int k = 0; k < NV; k++) part[row * NV + k] = out[k];
}

// The update of fluid node n: its 6 pull sources.  A row's fluid nodes are consecutive
// in the list, in x order, so the node at x - 1 (x + 1), when fluid, is n - 1 (n + 1):
// the entry's coordinates tell, loaded from the cache lines of n's own; the four sources
// in the neighbouring rows come from the rank map.
template <bool CHECK, bool NT, class Off>
__device__ inline void sweep7_node(const Sweep7 &a, int64_t n, double (&acc)[kKnSums]) {
    const uint32_t c = a.coords[n];
    const uint32_t cm = n > 0 ? a.coords[n - 1] : 0xffffffffu;
    const uint32_t cp = n + 1 < a.nf ? a.coords[n + 1] : 0xffffffffu;
    const int x = c & 1023, y = (c >> 10) & 1023, z = c >> 20;
    const Grid &g = a.g;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    // rows of the sources 3..6 (source x - e_i)
    const int nys[7] = {y, y, y, ym, yp, y, y};
    const int nzs[7] = {z, z, z, z, z, zm, zp};
    RankWord rw[7];
#pragma unroll
    for (int i = 3; i < 7; i++) rw[i] = a.rank[g.seg(x, nys[i], nzs[i])];
    int ids[7];
    ids[0] = 0;
    // beyond an x face the source is the ghost plane (-2)
    ids[1] = x == 0 ? -2 : (cm == pack_xyz(x - 1, y, z) ? (int)(n - 1) : -1);
    ids[2] = x == g.nx - 1 ? -2 : (cp == pack_xyz(x + 1, y, z) ? (int)(n + 1) : -1);
#pragma unroll
    for (int i = 3; i < 7; i++) ids[i] = rank_lookup(rw[i], x & (kSeg - 1));
    node7<CHECK, NT, Off>(a, n, x, y, z, ids, acc);
}

// One step, one fluid node per thread.
template <bool CHECK, bool NT, class Off>
__global__ __launch_bounds__(256) void k_sweep7(Sweep7 a) {
    const int64_t lb = a.chunk ? xcd_block(blockIdx.x, a.chunk) : (int64_t)blockIdx.x;
    const int64_t n = lb * 256 + threadIdx.x;
    double acc[kKnSums] = {0, 0, 0, 0, 0};
    if (n < a.nf) sweep7_node<CHECK, NT, Off>(a, n, acc);
    if (CHECK) write_partials7<kKnSums>(acc, lb, lb * 256 < a.nf, a.partials);
}

// ---------------------------------------------------------------- D3Q19 diffusion
// The same update on the paper's D3Q19 lattice (Section 3.2): 18 pull sources through the
// rank map, bounce-back at solid links, the ghost planes beyond the x faces for the five
// populations with e_x = +1 (at x = 0) or -1 (at x = nx - 1), shifts a_i (t0, tm, tp)
// from the unscaled tables, BGK with 1/tau_g towards a_i C (the rest population closing
// the balance of C).
template <bool CHECK, bool NT, class Off>
__device__ inline void sweep19d_node(const Sweep7 &a, int64_t n, double (&acc)[kKnSums]) {
    LBM_D3Q19_TABLES
    const uint32_t c = a.coords[n];
    // the sources x -+ 1 in the node's own row are the list's neighbouring entries (see
    // sweep7_node); the other 16 come from the rank map
    const uint32_t cm = n > 0 ? a.coords[n - 1] : 0xffffffffu;
    const uint32_t cp = n + 1 < a.nf ? a.coords[n + 1] : 0xffffffffu;
    const int x = c & 1023, y = (c >> 10) & 1023, z = c >> 20;
    const Grid &g = a.g;
    const bool gm = x == 0, gp = x == g.nx - 1;  // x - 1, x + 1 beyond a face
    int xs[3], ys[3], zs[3];
    xs[0] = gm ? x : x - 1; xs[1] = x; xs[2] = gp ? x : x + 1;  // the node stands in
    ys[0] = y == 0 ? g.ny - 1 : y - 1; ys[1] = y; ys[2] = y == g.ny - 1 ? 0 : y + 1;
    zs[0] = z == 0 ? g.nz - 1 : z - 1; zs[1] = z; zs[2] = z == g.nz - 1 ? 0 : z + 1;
    RankWord rw[19];
#pragma unroll
    for (int i = 3; i < 19; i++)
        rw[i] = a.rank[g.seg(xs[1 - EX[i]], ys[1 - EY[i]], zs[1 - EZ[i]])];
    int ids[19];
    ids[0] = 0;
    static_assert(EY[1] == 0 && EZ[1] == 0 && EX[1] == 1 && EY[2] == 0 && EZ[2] == 0 && EX[2] == -1,
                  "directions 1, 2 are +x, -x");
    ids[1] = cm == pack_xyz(x - 1, y, z) && !gm ? (int)(n - 1) : -1;
    ids[2] = cp == pack_xyz(x + 1, y, z) && !gp ? (int)(n + 1) : -1;
#pragma unroll
    for (int i = 3; i < 19; i++) ids[i] = rank_lookup(rw[i], xs[1 - EX[i]] & (kSeg - 1));
#pragma unroll
    for (int i = 1; i < 19; i++)
        if ((EX[i] == 1 && gm) || (EX[i] == -1 && gp)) ids[i] = -2;
    const float om = a.omega[n];
    const Shift sh = a.shift[x + 1];
    // element offsets popq(q, i, node): 32-bit while q * stride fits, 64-bit beyond
    Off off[19];
    off[0] = (Off)popq(19, 0, n);
#pragma unroll
    for (int i = 1; i < 19; i++)
        off[i] = ids[i] >= 0 ? (Off)popq(19, i, ids[i]) : (Off)popq(19, OPP[i], n);
    float ai[19];
#pragma unroll
    for (int i = 0; i < 19; i++) ai[i] = a.src[off[i]];
    // onto this node's output reference a_i C_ref(x); a ghost plane holds deviation 0
#pragma unroll
    for (int i = 0; i < 19; i++) {
        if (ids[i] == -2) ai[i] = 0.f;
        const float d = (EX[i] == 0 || ids[i] == -1) ? sh.t0 : (EX[i] == 1 ? sh.tm : sh.tp);
        ai[i] += a19(i) * d;
    }
    float cdev = 0.f;  // C - C_ref(x)
#pragma unroll
    for (int i = 0; i < 19; i++) cdev += ai[i];
    // the moving populations relax towards a_i C; the rest one takes what remains of C,
    // so the collision conserves C exactly although the binary32 a_i sum to 1 + 2.4e-8
    float so[19], moved = 0.f;
#pragma unroll
    for (int i = 1; i < 19; i++) {
        so[i] = ai[i] - om * (ai[i] - a19(i) * cdev);
        moved += so[i];
    }
    so[0] = cdev - moved;
#pragma unroll
    for (int i = 0; i < 19; i++) {
        if (NT)
            __builtin_nontemporal_store(so[i], &a.dst[popq(19, i, n)]);
        else
            a.dst[popq(19, i, n)] = so[i];
    }
    if (CHECK) {
        const double conc = a.ref_out[x + 1] + (double)cdev;
        const double dd = conc - (double)a.csnap[n];
        acc[0] += dd * dd;
        acc[1] += conc * conc;
        // net +x flux into the outlet ghost plane and out of the inlet one: the five
        // populations leaving towards the plane less the five it sends (weight 1/6)
        if (gp) {
            double out = 0.0;
#pragma unroll
            for (int i = 1; i < 19; i++)
                if (EX[i] == 1) out += (double)so[i];
            acc[2] += out - (double)sh.tp / 6.0;
        }
        if (gm) {
            double back = 0.0;
#pragma unroll
            for (int i = 1; i < 19; i++)
                if (EX[i] == -1) back += (double)so[i];
            acc[3] += (double)sh.tm / 6.0 - back;
        }
        acc[4] += conc;
        a.csnap[n] = (float)conc;
        if (a.c_out) a.c_out[a.g.lin(x, y, z)] = (float)conc;
    }
}

template <bool CHECK, bool NT, class Off>
__global__ __launch_bounds__(256) void k_sweep19d(Sweep7 a) {
    const int64_t lb = a.chunk ? xcd_block(blockIdx.x, a.chunk) : (int64_t)blockIdx.x;
    const int64_t n = lb * 256 + threadIdx.x;
    double acc[kKnSums] = {0, 0, 0, 0, 0};
    if (n < a.nf) sweep19d_node<CHECK, NT, Off>(a, n, acc);
    if (CHECK) write_partials7<kKnSums>(acc, lb, lb * 256 < a.nf, a.partials);
}

// ---------------------------------------------------------------- batched solves
// As in the batched flow solve: concatenated block-aligned fluid lists, rank maps with
// global node ids, block b of a launch runs physical block blocks[b].  Each lattice has
// its own per-x frame tables (nx + 2 entries from sh0) and nx plane-mean rows (from pl0).
struct KnLat {
    Grid g;
    int64_t n_end;  // one past the lattice's last node (global id)
    int64_t rk0;    // first rank word
    int64_t b0, b1; // physical blocks
    int64_t sh0;    // first entry of the per-x tables
    int64_t pl0;    // first plane row of the plane-mean partials
    float *c_out;   // concentration field written at checks (nullable)
};

// Launched block b of a batched sweep runs the work descs[b] describes (one record, one
// scalar load).  As in the batched flow solve, lattice l owns blocks [b0, b1): local node
// ids [0, nf) at offset n0 = 256 b0, arrays contiguous there with stride 256 (b1 - b0)
// (populations at 7 n0).
struct KnBlk {
    Grid g;
    int32_t pb;      // physical block (partial-sum row)
    int32_t b0, b1;  // the lattice's blocks
    int32_t nf;      // its fluid nodes
    int64_t rk0;     // first rank word (local ids)
    int64_t sh0;     // first entry of the per-x tables
    float *c_out;    // concentration field written at checks (nullable)
};
static_assert(sizeof(KnBlk) == 64, "one record per launched block");

template <bool CHECK, bool NT>
__global__ __launch_bounds__(256) void k_sweep7b(Sweep7 a, const KnBlk *__restrict__ descs) {
    const int64_t lb = a.chunk ? xcd_block(blockIdx.x, a.chunk) : (int64_t)blockIdx.x;
    double acc[kKnSums] = {0, 0, 0, 0, 0};
    const bool live = lb < a.launched_live;
    int64_t pb = 0;
    if (live) {
        const KnBlk D = descs[lb];
        pb = D.pb;
        const int64_t n0 = (int64_t)D.b0 * 256;
        Sweep7 b = a;
        b.g = D.g;
        b.nf = D.nf;
        b.stride = (int64_t)(D.b1 - D.b0) * 256;
        b.coords = a.coords + n0;
        b.rank = a.rank + D.rk0;
        b.omega = a.omega + n0;
        b.src = a.src + 7 * n0;
        b.dst = a.dst + 7 * n0;
        b.csnap = a.csnap + n0;
        b.shift = a.shift + D.sh0;
        b.ref_out = a.ref_out + D.sh0;
        b.c_out = D.c_out;
        const int64_t n = (pb - D.b0) * 256 + threadIdx.x;
        if (n < D.nf) sweep7_node<CHECK, NT, uint32_t>(b, n, acc);
    }
    if (CHECK) write_partials7<kKnSums>(acc, pb, live, a.partials);
}

// 1/tau_g per node from the pore diameter (Eq. 12); counts nodes with tau_g <= 1/2 and
// forms the partial sums of tau_g - 1/2 (for the local tortuosity).  With init_pop the
// populations start at the equilibrium w_i C_init in frame 0 (C_ref = 0 inside).
__global__ __launch_bounds__(256) void k_kn_init(Grid g, int64_t nf, int64_t stride,
                                                 const uint32_t *__restrict__ coords,
                                                 const double *__restrict__ diam, double d_ref,
                                                 double tau_ref, const float *__restrict__ c_init,
                                                 float *__restrict__ gbuf,
                                                 float *__restrict__ omega,
                                                 float *__restrict__ csnap, int init_pop,
                                                 unsigned long long *bad,
                                                 double *__restrict__ partials, int q) {
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
            const float c0 = c_init ? c_init[v] : 0.f;
            if (q == 7) {
                gbuf[popq(7, 0, n)] = kW0 * c0;
                for (int i = 1; i < 7; i++) gbuf[popq(7, i, n)] = kW1 * c0;
            } else {
                for (int i = 0; i < 19; i++) gbuf[popq(19, i, n)] = a19(i) * c0;
            }
            csnap[n] = c0;
        }
    }
    __shared__ double lds[4];
    double out[1];
    block_sum<1>(acc, lds, out);
    if (threadIdx.x == 0) partials[blockIdx.x] = out[0];
}

// Frame 0: C_ref = 0 inside, C_in / C_out on the ghost planes, and its steady shifts.
__global__ __launch_bounds__(1024) void k_frame0(int nx, double c_in, double c_out,
                                                 double *__restrict__ ref,
                                                 Shift *__restrict__ steady, double ws) {
    for (int k = threadIdx.x; k < nx + 2; k += 1024)
        ref[k] = k == 0 ? c_in : (k == nx + 1 ? c_out : 0.0);
    __syncthreads();
    for (int k = threadIdx.x; k < nx + 2; k += 1024) {
        Shift s;
        s.t0 = 0.f;
        s.tm = k >= 1 ? (float)(ws * (ref[k - 1] - ref[k])) : 0.f;
        s.tp = k <= nx ? (float)(ws * (ref[k + 1] - ref[k])) : 0.f;
        s.pad = 0.f;
        steady[k] = s;
    }
}

// Plane sums of the checked concentration, kPlaneParts workgroups per plane: workgroup
// p of plane x writes its (sum, count) to row[0], row[1].
__device__ inline void plane_mean_part(const Grid &g, const RankWord *__restrict__ rank,
                                       const float *__restrict__ csnap, int x, int p,
                                       double *__restrict__ row) {
    double acc[2] = {0.0, 0.0};
    const int64_t m = (int64_t)g.ny * g.nz;
    for (int64_t k = (int64_t)p * 256 + threadIdx.x; k < m; k += kPlaneParts * 256) {
        const int id = node_at(rank, g, x, (int)(k % g.ny), (int)(k / g.ny));
        if (id >= 0) {
            acc[0] += (double)csnap[id];
            acc[1] += 1.0;
        }
    }
    __shared__ double lds[8];
    double out[2];
    block_sum<2>(acc, lds, out);
    if (threadIdx.x == 0) {
        row[0] = out[0];
        row[1] = out[1];
    }
}

__global__ __launch_bounds__(256) void k_plane_mean(Grid g, const RankWord *__restrict__ rank,
                                                    const float *__restrict__ csnap,
                                                    double *__restrict__ part) {
    const int p = blockIdx.x, x = blockIdx.y;
    plane_mean_part(g, rank, csnap, x, p, part + 2 * (x * kPlaneParts + p));
}

// Batched: planes[q] = (lattice, x) of the q-th plane of the active lattices, workgroup
// q * kPlaneParts + p.
__global__ __launch_bounds__(256) void k_plane_mean_b(const int32_t *__restrict__ planes,
                                                      const KnLat *__restrict__ lats,
                                                      const RankWord *__restrict__ rank,
                                                      const float *__restrict__ csnap,
                                                      double *__restrict__ part) {
    const int64_t q = blockIdx.x / kPlaneParts;
    const int p = (int)(blockIdx.x % kPlaneParts);
    const int x = planes[2 * q + 1];
    const KnLat L = lats[planes[2 * q]];
    plane_mean_part(L.g, rank + L.rk0, csnap + L.b0 * 256, x, p,
                    part + 2 * ((L.pl0 + x) * kPlaneParts + p));
}

// The next frame: plane means (planes without fluid keep the current value), its steady
// shifts, and the shifts from the current frame into it.  Sums in fixed order.
__device__ inline void frame_next(int nx, double c_in, double c_out,
                                  const double *__restrict__ part,
                                  const double *__restrict__ ref_cur, double *__restrict__ ref_next,
                                  Shift *__restrict__ steady_next, Shift *__restrict__ trans,
                                  double ws) {
    for (int k = threadIdx.x; k < nx + 2; k += 1024) {
        double v;
        if (k == 0) {
            v = c_in;
        } else if (k == nx + 1) {
            v = c_out;
        } else {
            double s = 0.0, c = 0.0;
            for (int q = 0; q < kPlaneParts; q++) {
                s += part[2 * ((k - 1) * kPlaneParts + q)];
                c += part[2 * ((k - 1) * kPlaneParts + q) + 1];
            }
            v = c > 0.0 ? s / c : ref_cur[k];
        }
        ref_next[k] = v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nx + 2; k += 1024) {
        Shift s, t;
        s.t0 = 0.f;
        s.tm = k >= 1 ? (float)(ws * (ref_next[k - 1] - ref_next[k])) : 0.f;
        s.tp = k <= nx ? (float)(ws * (ref_next[k + 1] - ref_next[k])) : 0.f;
        s.pad = 0.f;
        t.t0 = (float)(ws * (ref_cur[k] - ref_next[k]));
        t.tm = k >= 1 ? (float)(ws * (ref_cur[k - 1] - ref_next[k])) : 0.f;
        t.tp = k <= nx ? (float)(ws * (ref_cur[k + 1] - ref_next[k])) : 0.f;
        t.pad = 0.f;
        steady_next[k] = s;
        trans[k] = t;
    }
}

__global__ __launch_bounds__(1024) void k_frame_next(int nx, double c_in, double c_out,
                                                     const double *__restrict__ part,
                                                     const double *__restrict__ ref_cur,
                                                     double *__restrict__ ref_next,
                                                     Shift *__restrict__ steady_next,
                                                     Shift *__restrict__ trans, double ws) {
    frame_next(nx, c_in, c_out, part, ref_cur, ref_next, steady_next, trans, ws);
}

// Batched: workgroup l forms the next frame of lattice lat_ids[l].
__global__ __launch_bounds__(1024) void k_frame_next_b(const int32_t *__restrict__ lat_ids,
                                                       const KnLat *__restrict__ lats,
                                                       double c_in, double c_out,
                                                       const double *__restrict__ part,
                                                       const double *__restrict__ ref_cur,
                                                       double *__restrict__ ref_next,
                                                       Shift *__restrict__ steady_next,
                                                       Shift *__restrict__ trans) {
    const KnLat L = lats[lat_ids[blockIdx.x]];
    frame_next(L.g.nx, c_in, c_out, part + 2 * L.pl0 * kPlaneParts, ref_cur + L.sh0,
               ref_next + L.sh0, steady_next + L.sh0, trans + L.sh0, 0.125);
}

// Net +x flux through the link plane x = px - 1/2 (px = 0..nx) over links with both ends
// fluid (ghost planes count as fluid), kPlaneParts workgroups per plane (blockIdx.y = px),
// each summing every kPlaneParts-th run of 256 rows into part[px][blockIdx.x].
// g_{+x}(left) - g_{-x}(right) in the frame of `right` is s_{+x}(left) + tm(right) -
// s_{-x}(right); the ghost planes hold zero deviation.
__global__ __launch_bounds__(256) void k_plane_flux(Grid g, const RankWord *__restrict__ rank,
                                                    const float *__restrict__ gcur,
                                                    const Shift *__restrict__ steady,
                                                    double *__restrict__ part) {
    const int px = blockIdx.y;
    const int left = px - 1, right = px;
    double acc[1] = {0.0};
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < (int64_t)g.ny * g.nz;
         k += 256 * kPlaneParts) {
        const int y = (int)(k % g.ny), z = (int)(k / g.ny);
        const int il = left >= 0 ? node_at(rank, g, left, y, z) : -2;
        const int ir = right < g.nx ? node_at(rank, g, right, y, z) : -2;
        if (il == -1 || ir == -1) continue;
        const double fwd = left >= 0 ? (double)gcur[popq(7, 1, il)] : 0.0;
        const double bwd = right < g.nx ? (double)gcur[popq(7, 2, ir)] : 0.0;
        acc[0] += (fwd + (double)steady[right + 1].tm) - bwd;
    }
    __shared__ double lds[4];
    double out[1];
    block_sum<1>(acc, lds, out);
    if (threadIdx.x == 0) part[px * kPlaneParts + blockIdx.x] = out[0];
}

// The same on D3Q19: over the five directions with e_x = +1, the links from
// (px - 1, y - e_y, z - e_z) to (px, y, z) with both ends fluid; the shift tables are
// unscaled, so the frame difference is a_i tm.
__global__ __launch_bounds__(256) void k_plane_flux19(Grid g, const RankWord *__restrict__ rank,
                                                      const float *__restrict__ gcur,
                                                      const Shift *__restrict__ steady,
                                                      double *__restrict__ part) {
    LBM_D3Q19_TABLES
    const int px = blockIdx.y;
    const int left = px - 1, right = px;
    const double tm = (double)steady[right + 1].tm;
    double acc[1] = {0.0};
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < (int64_t)g.ny * g.nz;
         k += 256 * kPlaneParts) {
        const int y = (int)(k % g.ny), z = (int)(k / g.ny);
        const int ir = right < g.nx ? node_at(rank, g, right, y, z) : -2;
        if (ir == -1) continue;
        for (int i = 1; i < 19; i++) {
            if (EX[i] != 1) continue;
            const int ly = (y - EY[i] + g.ny) % g.ny, lz = (z - EZ[i] + g.nz) % g.nz;
            const int il = left >= 0 ? node_at(rank, g, left, ly, lz) : -2;
            if (il == -1) continue;
            const double fwd = il >= 0 ? (double)gcur[popq(19, i, il)] : 0.0;
            const double bwd = ir >= 0 ? (double)gcur[popq(19, OPP[i], ir)] : 0.0;
            acc[0] += (fwd - bwd) + (double)a19(i) * tm;
        }
    }
    __shared__ double lds[4];
    double out[1];
    block_sum<1>(acc, lds, out);
    if (threadIdx.x == 0) part[px * kPlaneParts + blockIdx.x] = out[0];
}

// plane[px] = the sum of the kPlaneParts partials of link plane px, in a fixed order.
__global__ __launch_bounds__(256) void k_plane_flux_sum(int planes, const double *__restrict__ part,
                                                        double *__restrict__ plane) {
    const int px = blockIdx.x * 256 + threadIdx.x;
    if (px >= planes) return;
    double s = 0.0;
    for (int p = 0; p < kPlaneParts; p++) s += part[px * kPlaneParts + p];
    plane[px] = s;
}

// The nx + 1 link-plane fluxes of the state gcur (in the frame whose steady shifts are
// `steady`) into plane[0..nx]; part holds (nx + 1) kPlaneParts doubles.
static lbm_status kn_plane_fluxes(const Grid &g, const RankWord *rank, const float *gcur,
                                  const Shift *steady, double *part, double *plane, int32_t lattice,
                                  hipStream_t s) {
    const dim3 grid(kPlaneParts, (unsigned)(g.nx + 1));
    if (lattice == LBM_LATTICE_D3Q19)
        k_plane_flux19<<<grid, 256, 0, s>>>(g, rank, gcur, steady, part);
    else
        k_plane_flux<<<grid, 256, 0, s>>>(g, rank, gcur, steady, part);
    LBM_CHECK_LAUNCH();
    k_plane_flux_sum<<<(unsigned)((g.nx + 1 + 255) / 256), 256, 0, s>>>(g.nx + 1, part, plane);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

// Denominator floor of the flux spread: 1e-6 of the flux an open box (every voxel fluid,
// tau_g = tau_ref) carries between the ghost planes.
static double kn_spread_floor(const Grid &g, const lbm_knudsen_params *p, int32_t lattice) {
    const double cs2 = lattice == LBM_LATTICE_D3Q19 ? 1.0 / 3.0 : 0.25;
    return 1e-6 * cs2 * (p->tau_ref - 0.5) * (double)g.ny * g.nz *
           std::fabs(p->c_in - p->c_out) / (double)(g.nx + 1);
}

__global__ void k_kn_sample(Grid g, int64_t count, const int64_t *__restrict__ vox,
                            const RankWord *__restrict__ rank, const float *__restrict__ gcur,
                            const float *__restrict__ omega, const double *__restrict__ cref,
                            double *__restrict__ out, uint8_t *__restrict__ flag, int q) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const int64_t v = vox[s];
    const int x = (int)(v % g.nx), y = (int)((v / g.nx) % g.ny), z = (int)(v / ((int64_t)g.nx * g.ny));
    const int id = node_at(rank, g, x, y, z);
    flag[s] = id >= 0;
    const double ref = cref[x + 1];
    for (int i = 0; i < q; i++) {
        const double w = q == 7 ? (i ? 0.125 : 0.25) : (double)a19(i);
        out[s * (q + 1) + i] = id >= 0 ? (double)gcur[popq(q, i, id)] + w * ref : 0.0;
    }
    out[s * (q + 1) + q] = id >= 0 ? 1.0 / (double)omega[id] : 0.0;
}

// Plane means of the checked concentration become the next frame (kept pending until
// the next sweep moves the state into it).
static lbm_status kn_next_frame(const KnWs &w, const Grid &g, const KnHeader &h, hipStream_t s) {
    k_plane_mean<<<dim3(kPlaneParts, g.nx), 256, 0, s>>>(g, w.rank, w.csnap, w.part);
    LBM_CHECK_LAUNCH();
    const int f = h.frame;
    k_frame_next<<<1, 1024, 0, s>>>(g.nx, h.c_in, h.c_out, w.part, w.ref[f], w.ref[f ^ 1],
                                    w.steady[f ^ 1], w.trans, kn_shift_scale(h.lattice));
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

// Kernel variant: explicit bits, or chosen from the working set (see the flow solve):
// streaming (plain order, non-temporal stores) once the two population arrays, 1/tau_g,
// the snapshot and the coordinates exceed the 256 MB Infinity Cache, cache-resident
// (XCD-contiguous order) below.
struct Variant7 {
    bool remap, nt;
    bool wide;  // 64-bit population offsets
};

static Variant7 pick_variant7(int32_t v, int64_t stride, int q = 7) {
    Variant7 m;
    m.wide = (v & LBM_VARIANT_OFF64) || q * stride > (int64_t)UINT32_MAX;
    if (v & LBM_VARIANT_EXPLICIT) {
        m.remap = v & LBM_VARIANT_REMAP;
        m.nt = v & LBM_VARIANT_NTSTORE;
        return m;
    }
    const bool stream = (2.0 * q * 4 + 12.0) * (double)stride > kCacheBytes;
    m.remap = !stream;
    m.nt = stream;
    return m;
}

template <bool CHECK, class Off>
static void launch7o(const Sweep7 &a, const Variant7 &m, int32_t lattice, hipStream_t s) {
    const unsigned grid = (unsigned)a.launched;
    if (lattice == LBM_LATTICE_D3Q19) {
        if (m.nt) k_sweep19d<CHECK, true, Off><<<grid, 256, 0, s>>>(a);
        else k_sweep19d<CHECK, false, Off><<<grid, 256, 0, s>>>(a);
    } else {
        if (m.nt) k_sweep7<CHECK, true, Off><<<grid, 256, 0, s>>>(a);
        else k_sweep7<CHECK, false, Off><<<grid, 256, 0, s>>>(a);
    }
}

template <bool CHECK>
static void launch7(const Sweep7 &a, const Variant7 &m, int32_t lattice, hipStream_t s) {
    if (m.wide || kn_q(lattice) * a.stride > (int64_t)UINT32_MAX) launch7o<CHECK, int64_t>(a, m, lattice, s);
    else launch7o<CHECK, uint32_t>(a, m, lattice, s);
}

// `steps` sweeps; the first one moves the state into the pending frame if there is one.
static lbm_status kn_launch(const KnWs &w, const Grid &g, int64_t nf, KnHeader &h,
                            const Variant7 &m, int &cur, bool &pending, int64_t steps,
                            bool check_last, float *c_field, hipStream_t s) {
    Sweep7 a;
    a.g = g;
    a.nf = nf;
    a.stride = w.stride;
    a.chunk = m.remap ? (kn_blocks(nf) + kXcd - 1) / kXcd : 0;
    a.launched = a.chunk ? xcd_launch(kn_blocks(nf), a.chunk) : kn_blocks(nf);
    a.coords = w.coords;
    a.rank = w.rank;
    a.omega = w.omega;
    a.csnap = w.csnap;
    a.c_out = c_field;
    a.partials = w.partials;
    for (int64_t t = 0; t < steps; t++) {
        if (pending) {
            a.shift = w.trans;
            h.frame ^= 1;
            pending = false;
        } else {
            a.shift = w.steady[h.frame];
        }
        a.ref_out = w.ref[h.frame];
        a.src = w.g[cur];
        a.dst = w.g[cur ^ 1];
        if (check_last && t == steps - 1)
            launch7<true>(a, m, h.lattice, s);
        else
            launch7<false>(a, m, h.lattice, s);
        LBM_CHECK_LAUNCH();
        cur ^= 1;
    }
    return LBM_OK;
}

// The reported quantities of a Knudsen solve from its last check sums (Phi_out, Phi_in,
// sum C), the sum of tau_g - 1/2 and the link-plane fluxes (Eqs. 11, 14-16).
static void kn_result(lbm_knudsen_result *r, const lbm_knudsen_params *p, const Grid &g,
                      int64_t nf, int64_t t, bool converged, double resid, const double *sums,
                      double sum_tau, const double *planes, double sweep_ms, double updates,
                      int32_t lattice) {
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
    const double cs2 = lattice == LBM_LATTICE_D3Q19 ? 1.0 / 3.0 : 0.25;
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
    r->Deff_planes = mean / ((double)g.ny * g.nz) * (double)(g.nx + 1) / dc;
    r->sweep_ms = sweep_ms;
    r->mlups = sweep_ms > 0 ? updates / (sweep_ms * 1e3) : 0.0;
    const double bytes = lattice == LBM_LATTICE_D3Q19 ? 156.0 : 60.0;  // 2 x q x 4 + 1/tau_g
    r->gbps = sweep_ms > 0 ? updates * bytes / (sweep_ms * 1e-3) / 1e9 : 0.0;
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
    LBM_REQUIRE(p->steady_tol >= 0.0 && std::isfinite(p->steady_tol), LBM_E_INVAL,
                "steady_tol must be finite and >= 0");
    LBM_REQUIRE(std::isfinite(p->c_in) && std::isfinite(p->c_out), LBM_E_INVAL,
                "C_in and C_out must be finite");
    LBM_REQUIRE(p->c_in != p->c_out, LBM_E_INVAL, "C_in equals C_out: no driving difference");
    LBM_REQUIRE(p->tau_ref > 0.5 && p->d_ref_nm > 0 && p->voxel_nm > 0 &&
                    std::isfinite(p->tau_ref) && std::isfinite(p->d_ref_nm) &&
                    std::isfinite(p->voxel_nm),
                LBM_E_INVAL, "tau_ref must exceed 1/2 and d_ref, voxel size be positive (all finite)");
    LBM_REQUIRE((p->variant & ~kSolveVariantBits) == 0, LBM_E_INVAL, "unknown variant bits 0x%x",
                p->variant);
    LBM_REQUIRE(p->lattice == LBM_LATTICE_D3Q7 || p->lattice == LBM_LATTICE_D3Q19, LBM_E_INVAL,
                "unknown lattice %d", p->lattice);
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g = make_grid(n);
    const int q = kn_q(p->lattice);

    KnWs w0 = carve_kn(workspace, g, 1, q);
    LBM_REQUIRE(ws_bytes >= (size_t)((char *)w0.coords - (char *)workspace), LBM_E_NOMEM,
                "workspace of %zu bytes is below the grid part", ws_bytes);
    int64_t nf = 0;
    KnHeader h;
    int64_t t0 = 0;
    int cur = 0;
    if (p->resume) {
        // checked against a plain count of the mask before the rank map is rebuilt, so
        // that a refused resume leaves the stored state usable
        LBM_TRY_HIP(hipMemcpyAsync(&h, w0.hdr, sizeof(h), hipMemcpyDeviceToHost, s));
        st = count_nonzero(g, fluid, w0.counter, &nf, s);
        if (st != LBM_OK) return st;
        LBM_REQUIRE(h.magic == kKnMagic && h.nx == n[0] && h.ny == n[1] && h.nz == n[2] &&
                        h.n_fluid == nf && h.c_in == p->c_in && h.c_out == p->c_out &&
                        h.lattice == p->lattice,
                    LBM_E_INVAL, "resume: the workspace holds no state for this problem");
        // the relaxation times are formed again from pore_diam: only under the same Eq. 12
        LBM_REQUIRE(h.tau_ref == p->tau_ref && h.d_ref == p->d_ref_nm / p->voxel_nm, LBM_E_INVAL,
                    "resume: tau_ref or d_ref / voxel size differ from the state's");
        t0 = h.steps_done;
        cur = h.cur;
    } else {
        h.frame = 0;
    }
    st = layout_count(g, fluid, w0.rank, w0.total, &nf, s);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(nf > 0, LBM_E_INVAL, "the fluid mask is empty");
    KnWs w = carve_kn(workspace, g, nf, q);
    LBM_REQUIRE(ws_bytes >= w.bytes, LBM_E_NOMEM,
                "workspace of %zu bytes; %zu needed for %lld fluid nodes", ws_bytes, w.bytes,
                (long long)nf);
    h.variant = p->variant;
    h.lattice = p->lattice;
    h.pad = 0;
    const Variant7 mode = pick_variant7(p->variant, w.stride, q);
    st = layout_fill(g, w.rank, w.coords, s);
    if (st != LBM_OK) return st;
    h.magic = kKnMagic;
    h.nx = n[0]; h.ny = n[1]; h.nz = n[2];
    h.n_fluid = nf;
    h.c_in = p->c_in;
    h.c_out = p->c_out;
    const double d_ref = p->d_ref_nm / p->voxel_nm;
    h.tau_ref = p->tau_ref;
    h.d_ref = d_ref;
    LBM_TRY_HIP(hipMemsetAsync(w.counter, 0, sizeof(unsigned long long), s));
    k_kn_init<<<(unsigned)kn_blocks(nf), 256, 0, s>>>(g, nf, w.stride, w.coords, pore_diam, d_ref,
                                                      p->tau_ref, c_init, w.g[cur], w.omega,
                                                      w.csnap, p->resume ? 0 : 1, w.counter,
                                                      w.partials, q);
    LBM_CHECK_LAUNCH();
    bool pending = false;
    if (!p->resume) {
        // frame 0 holds the initial state; its plane means become the first pending frame
        k_frame0<<<1, 1024, 0, s>>>(g.nx, h.c_in, h.c_out, w.ref[0], w.steady[0],
                                    kn_shift_scale(h.lattice));
        LBM_CHECK_LAUNCH();
        st = kn_next_frame(w, g, h, s);
        if (st != LBM_OK) return st;
        pending = true;
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

    // The check sums land in pinned host memory, copied right after their reduction, so
    // the frame update that follows runs while the host reads them and queues the next
    // interval (the same kernels in the same order as without the copy moved forward).
    // (Buffer and events are released on every return.)
    struct Pinned {
        double *p = nullptr;
        hipEvent_t got = nullptr, e0 = nullptr, e1 = nullptr;
        ~Pinned() {
            if (e1) (void)hipEventDestroy(e1);
            if (e0) (void)hipEventDestroy(e0);
            if (got) (void)hipEventDestroy(got);
            if (p) (void)hipHostFree(p);
        }
    } pin;
    LBM_TRY_HIP(hipHostMalloc((void **)&pin.p, sizeof(double) * kKnSums, hipHostMallocDefault));
    LBM_TRY_HIP(hipEventCreateWithFlags(&pin.got, hipEventDisableTiming));
    LBM_TRY_HIP(hipEventCreate(&pin.e0));
    LBM_TRY_HIP(hipEventCreate(&pin.e1));
    const hipEvent_t e0 = pin.e0, e1 = pin.e1;
    const int64_t limit = p->fixed_steps > 0 ? p->fixed_steps : p->max_steps;
    const int nc = p->check_every;
    double sums[kKnSums] = {0, 0, 0, 0, 0};
    double resid = INFINITY, sweep_ms = 0.0;
    SteadyEst est;
    const double spread_floor = kn_spread_floor(g, p, h.lattice);
    bool converged = false, diverged = false;
    int64_t t = 0;
    lbm_status out = LBM_OK;
    while (t < limit) {
        const int64_t abs_t = t0 + t;
        int64_t chunk = nc - (abs_t % nc);
        if (chunk > limit - t) chunk = limit - t;
        LBM_TRY_HIP(hipEventRecord(e0, s));
        out = kn_launch(w, g, nf, h, mode, cur, pending, chunk, true, c_field, s);
        if (out != LBM_OK) break;
        LBM_TRY_HIP(hipEventRecord(e1, s));
        out = reduce_partials(w.partials, kn_blocks(nf), kKnSums, w.res, s);
        if (out != LBM_OK) break;
        LBM_TRY_HIP(hipMemcpyAsync(pin.p, w.res, sizeof(sums), hipMemcpyDeviceToHost, s));
        LBM_TRY_HIP(hipEventRecord(pin.got, s));
        out = kn_next_frame(w, g, h, s);
        if (out != LBM_OK) break;
        pending = true;
        LBM_TRY_HIP(hipEventSynchronize(pin.got));
        std::memcpy(sums, pin.p, sizeof(sums));
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
            est.push(resid);
            if (p->fixed_steps <= 0 && resid < p->tol) {
                converged = true;
                if (p->steady_tol > 0.0) {
                    // steady state: the same flux through every link plane (the state is
                    // still in frame h.frame; the pending frame only enters with the next
                    // sweep)
                    out = kn_plane_fluxes(g, w.rank, w.g[cur], w.steady[h.frame], w.fpart,
                                          w.plane, h.lattice, s);
                    if (out != LBM_OK) break;
                    double pl[kMaxEdge + 1];
                    LBM_TRY_HIP(hipMemcpyAsync(pl, w.plane, sizeof(double) * (g.nx + 1),
                                               hipMemcpyDeviceToHost, s));
                    LBM_TRY_HIP(hipStreamSynchronize(s));
                    converged = plane_spread(pl, g.nx + 1, spread_floor) <= p->steady_tol;
                }
                if (converged) break;
            }
        }
    }
    if (out != LBM_OK) return out;
    // a pending frame that no sweep entered is dropped: the state stays in h.frame
    h.cur = cur;
    h.steps_done = t0 + t;
    LBM_TRY_HIP(hipMemcpyAsync(w.hdr, &h, sizeof(h), hipMemcpyHostToDevice, s));
    // link-plane fluxes of the final state
    st = kn_plane_fluxes(g, w.rank, w.g[cur], w.steady[h.frame], w.fpart, w.plane, h.lattice, s);
    if (st != LBM_OK) return st;
    double planes[kMaxEdge + 1];
    LBM_TRY_HIP(hipMemcpyAsync(planes, w.plane, sizeof(double) * (g.nx + 1), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    if (plane_flux_h) std::memcpy(plane_flux_h, planes, sizeof(double) * (g.nx + 1));

    kn_result(r, p, g, nf, t, converged, resid, sums, sum_tau, planes, sweep_ms,
              (double)nf * (double)t, h.lattice);
    r->steady_dist = est.dist(nc);
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
    w = carve_kn(workspace, g, h.n_fluid, kn_q(h.lattice));
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
    bool pending = false;
    st = kn_launch(w, g, h.n_fluid, h, pick_variant7(h.variant, w.stride, kn_q(h.lattice)), cur,
                   pending, steps, false, nullptr, s);
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
    k_kn_sample<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(g, count, w.samp_vox,
                                                               w.rank, w.g[h.cur], w.omega,
                                                               w.ref[h.frame], w.samp_out,
                                                               w.samp_flag, kn_q(h.lattice));
    LBM_CHECK_LAUNCH();
    const int q = kn_q(h.lattice);
    std::vector<double> tmp((size_t)count * (q + 1));
    LBM_TRY_HIP(hipMemcpyAsync(tmp.data(), w.samp_out, sizeof(double) * (q + 1) * count,
                               hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipMemcpyAsync(fluid_h, w.samp_flag, count, hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < count; i++) {
        for (int k = 0; k < q; k++) g_h[i * q + k] = tmp[i * (q + 1) + k];
        tau_h[i] = tmp[i * (q + 1) + q];
    }
    return LBM_OK;
}

// ============================================================== batched Knudsen solves
namespace lbm {

struct KnBatchWs {
    KnLat *lats;
    KnBlk *descs;
    int32_t *lat_ids, *total, *planes;
    unsigned long long *counter;
    double *res, *tau_sum, *plane;
    RankWord *rank;
    uint32_t *coords;
    float *g[2];
    float *omega, *csnap;
    double *partials;
    double *ref[2];
    Shift *steady[2];
    Shift *trans;
    double *part;
    double *fpart;  // link-plane flux partials, kPlaneParts per table row
    int64_t stride, nblk, nrank, ntab, nplane;
    size_t bytes;
};

static KnBatchWs carve_kn_batch(void *base, int count, const int32_t *n_h, const int64_t *nf_h) {
    KnBatchWs w;
    w.nblk = w.nrank = w.ntab = w.nplane = 0;
    for (int l = 0; l < count; l++) {
        const Grid g = make_grid(n_h + 3 * l);
        w.nblk += kn_blocks(nf_h[l] < 1 ? 1 : nf_h[l]);
        w.nrank += g.nsegs();
        w.ntab += g.nx + 2;
        w.nplane += g.nx;
    }
    w.stride = w.nblk * 256;
    Carver c(base);
    w.lats = c.take<KnLat>(count);
    w.descs = c.take<KnBlk>(w.nblk);
    w.lat_ids = c.take<int32_t>(count);
    w.total = c.take<int32_t>(count);
    w.planes = c.take<int32_t>(2 * w.nplane);
    w.counter = c.take<unsigned long long>(1);
    w.res = c.take<double>((size_t)count * kKnSums);
    w.tau_sum = c.take<double>(count);
    w.plane = c.take<double>(w.ntab);  // nx + 1 link planes per lattice fit its nx + 2 rows
    w.rank = c.take<RankWord>(w.nrank);
    w.coords = c.take<uint32_t>(w.stride);
    w.g[0] = c.take<float>((size_t)7 * w.stride);
    w.g[1] = c.take<float>((size_t)7 * w.stride);
    w.omega = c.take<float>(w.stride);
    w.csnap = c.take<float>(w.stride);
    w.partials = c.take<double>((size_t)w.nblk * kKnSums);
    for (int f = 0; f < 2; f++) w.ref[f] = c.take<double>(w.ntab);
    for (int f = 0; f < 2; f++) w.steady[f] = c.take<Shift>(w.ntab);
    w.trans = c.take<Shift>(w.ntab);
    w.part = c.take<double>((size_t)w.nplane * kPlaneParts * 2);
    w.fpart = c.take<double>((size_t)w.ntab * kPlaneParts);
    w.bytes = c.off;
    return w;
}

template <bool CHECK>
static void launch7b(const Sweep7 &a, const Variant7 &m, const KnBlk *descs, hipStream_t s) {
    const unsigned grid = (unsigned)a.launched;
    if (m.nt) k_sweep7b<CHECK, true><<<grid, 256, 0, s>>>(a, descs);
    else k_sweep7b<CHECK, false><<<grid, 256, 0, s>>>(a, descs);
}

// The batch's position in its iteration: population buffer, frame of the stored state,
// and whether the next sweep moves the state into the other frame.
struct KnPos {
    int cur = 0, frame = 0;
    bool pending = false;
};

// The plane means of group g's checked concentration become its lattices' next frames.
static lbm_status kn_batch_frames(const KnBatchWs &w, const BatchGroup &g, int frame,
                                  const lbm_knudsen_params *p, hipStream_t s) {
    k_plane_mean_b<<<(unsigned)(g.n_pl * kPlaneParts), 256, 0, s>>>(
        w.planes + 2 * g.pl_off, w.lats, w.rank, w.csnap, w.part);
    LBM_CHECK_LAUNCH();
    k_frame_next_b<<<(unsigned)g.n_lat, 1024, 0, s>>>(w.lat_ids + g.lat_off, w.lats, p->c_in,
                                                      p->c_out, w.part, w.ref[frame],
                                                      w.ref[frame ^ 1], w.steady[frame ^ 1],
                                                      w.trans);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

// `steps` sweeps of group g from position q; with check_last the last one checks, the
// group's per-lattice sums go to w.res and its next frames are formed.
static lbm_status kn_batch_steps(const KnBatchWs &w, Sweep7 a, const Variant7 &m,
                                 const BatchGroup &g, KnPos &q, int64_t steps, bool check_last,
                                 const lbm_knudsen_params *p, hipStream_t s) {
    const int64_t n_live = g.n_blk;
    a.launched_live = n_live;
    a.chunk = m.remap ? (n_live + kXcd - 1) / kXcd : 0;
    a.launched = a.chunk ? xcd_launch(n_live, a.chunk) : n_live;
    const KnBlk *descs = w.descs + g.blk_off;
    for (int64_t t = 0; t < steps; t++) {
        if (q.pending) {
            a.shift = w.trans;
            q.frame ^= 1;
            q.pending = false;
        } else {
            a.shift = w.steady[q.frame];
        }
        a.ref_out = w.ref[q.frame];
        a.src = w.g[q.cur];
        a.dst = w.g[q.cur ^ 1];
        if (check_last && t == steps - 1) launch7b<true>(a, m, descs, s);
        else launch7b<false>(a, m, descs, s);
        LBM_CHECK_LAUNCH();
        q.cur ^= 1;
    }
    if (check_last) {
        k_lat_reduce<kKnSums><<<(unsigned)g.n_lat, 256, 0, s>>>(w.partials, w.lats,
                                                                w.lat_ids + g.lat_off, w.res);
        LBM_CHECK_LAUNCH();
        lbm_status st = kn_batch_frames(w, g, q.frame, p, s);
        if (st != LBM_OK) return st;
        q.pending = true;
    }
    return LBM_OK;
}

// Binary32 Knudsen state per fluid node: two population buffers, 1/tau_g, snapshot,
// coordinate.
constexpr double kBatchKnNodeBytes = 2 * 7 * 4 + 4 + 4 + 4;

}  // namespace lbm

extern "C" size_t lbm_knudsen_batch_workspace(int32_t count, const int32_t *n_h,
                                              const int64_t *nf_h) {
    if (count < 1 || !n_h || !nf_h) return 0;
    for (int l = 0; l < count; l++)
        if (n_h[3 * l] < 1 || n_h[3 * l + 1] < 1 || n_h[3 * l + 2] < 1 || n_h[3 * l] > kMaxEdge ||
            n_h[3 * l + 1] > kMaxEdge || n_h[3 * l + 2] > kMaxEdge || nf_h[l] < 0)
            return 0;
    return carve_kn_batch(nullptr, count, n_h, nf_h).bytes;
}

extern "C" lbm_status lbm_knudsen_solve_batch(int32_t count, const int32_t *n_h,
                                              const uint8_t *const *fluid,
                                              const double *const *pore_diam, const int64_t *nf_h,
                                              const lbm_knudsen_params *p, lbm_batch_sched *sched,
                                              lbm_knudsen_result *r_h, float *const *c_field,
                                              const float *const *c_init, void *workspace,
                                              size_t ws_bytes, void *stream) {
    LBM_REQUIRE(count >= 1 && n_h && fluid && pore_diam && nf_h && p && r_h && workspace,
                LBM_E_INVAL, "lbm_knudsen_solve_batch: null argument or empty batch");
    for (int l = 0; l < count; l++) {
        const int32_t *n = n_h + 3 * l;
        LBM_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && n[0] <= kMaxEdge && n[1] <= kMaxEdge &&
                        n[2] <= kMaxEdge,
                    LBM_E_INVAL, "lattice %d: sizes must lie in [1, %d]", l, kMaxEdge);
        LBM_REQUIRE(fluid[l] && pore_diam[l] && nf_h[l] >= 1, LBM_E_INVAL,
                    "lattice %d: no fluid mask, pore diameter or node", l);
    }
    LBM_REQUIRE(p->check_every >= 1, LBM_E_INVAL, "check_every must be >= 1");
    LBM_REQUIRE(p->fixed_steps > 0 || p->max_steps > 0, LBM_E_INVAL, "no step limit given");
    LBM_REQUIRE(p->steady_tol >= 0.0 && std::isfinite(p->steady_tol), LBM_E_INVAL,
                "steady_tol must be finite and >= 0");
    LBM_REQUIRE(std::isfinite(p->c_in) && std::isfinite(p->c_out), LBM_E_INVAL,
                "C_in and C_out must be finite");
    LBM_REQUIRE(p->c_in != p->c_out, LBM_E_INVAL, "C_in equals C_out: no driving difference");
    LBM_REQUIRE(p->tau_ref > 0.5 && p->d_ref_nm > 0 && p->voxel_nm > 0 &&
                    std::isfinite(p->tau_ref) && std::isfinite(p->d_ref_nm) &&
                    std::isfinite(p->voxel_nm),
                LBM_E_INVAL, "tau_ref must exceed 1/2 and d_ref, voxel size be positive (all finite)");
    LBM_REQUIRE(!p->resume, LBM_E_INVAL, "batched solves do not resume");
    LBM_REQUIRE(p->lattice == LBM_LATTICE_D3Q7, LBM_E_INVAL,
                "batched solves run the D3Q7 lattice only");
    LBM_REQUIRE((p->variant & ~(kVariantBits | LBM_VARIANT_NOGRAPH)) == 0, LBM_E_INVAL,
                "unknown variant bits 0x%x", p->variant);
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    const KnBatchWs w = carve_kn_batch(workspace, count, n_h, nf_h);
    for (int l = 0; l < count; l++)
        LBM_REQUIRE(7 * kn_blocks(nf_h[l]) * 256 <= (int64_t)UINT32_MAX, LBM_E_INVAL,
                    "lattice %d: %lld nodes exceed the 32-bit population offsets", l,
                    (long long)nf_h[l]);
    LBM_REQUIRE(ws_bytes >= w.bytes, LBM_E_NOMEM, "workspace of %zu bytes; %zu needed", ws_bytes,
                w.bytes);
    hipStream_t caller = static_cast<hipStream_t>(stream);
    BatchRes R;
    st = R.open(caller);
    if (st != LBM_OK) return st;
    hipStream_t s = R.s;

    // layout, lattice table, initial state, relaxation times and frame 0 of every lattice
    const double d_ref = p->d_ref_nm / p->voxel_nm;
    std::vector<KnLat> lats(count);
    std::vector<BatchLat> bl(count);
    std::vector<KnBlk> blk(w.nblk);  // the record of each physical block
    LBM_TRY_HIP(hipMemsetAsync(w.counter, 0, sizeof(unsigned long long), s));
    int64_t n0 = 0, rk0 = 0, b0 = 0, sh0 = 0, pl0 = 0;
    for (int l = 0; l < count; l++) {
        const Grid g = make_grid(n_h + 3 * l);
        int64_t nf = 0;
        st = layout_count(g, fluid[l], w.rank + rk0, w.total + l, &nf, s);
        if (st != LBM_OK) return st;
        LBM_REQUIRE(nf == nf_h[l], LBM_E_INVAL, "lattice %d has %lld fluid nodes, not %lld", l,
                    (long long)nf, (long long)nf_h[l]);
        st = layout_fill(g, w.rank + rk0, w.coords + n0, s);
        if (st != LBM_OK) return st;
        KnLat &L = lats[l];
        L.g = g;
        L.n_end = n0 + nf;
        L.rk0 = rk0;
        L.b0 = b0;
        L.b1 = b0 + kn_blocks(nf);
        L.sh0 = sh0;
        L.pl0 = pl0;
        L.c_out = c_field ? c_field[l] : nullptr;
        if (L.c_out) LBM_TRY_HIP(hipMemsetAsync(L.c_out, 0, sizeof(float) * g.nvox(), s));
        const int64_t span = (L.b1 - L.b0) * 256;
        k_kn_init<<<(unsigned)kn_blocks(nf), 256, 0, s>>>(
            g, nf, span, w.coords + n0, pore_diam[l], d_ref, p->tau_ref,
            c_init ? c_init[l] : nullptr, w.g[0] + 7 * n0, w.omega + n0, w.csnap + n0, 1,
            w.counter, w.partials + b0, 7);
        LBM_CHECK_LAUNCH();
        st = reduce_partials(w.partials + b0, kn_blocks(nf), 1, w.tau_sum + l, s);
        if (st != LBM_OK) return st;
        k_frame0<<<1, 1024, 0, s>>>(g.nx, p->c_in, p->c_out, w.ref[0] + sh0, w.steady[0] + sh0,
                                    0.125);
        LBM_CHECK_LAUNCH();
        bl[l] = BatchLat{L.b0, L.b1, nf, g.nx};
        for (int64_t b = L.b0; b < L.b1; b++)
            blk[b] = KnBlk{g, (int32_t)b, (int32_t)L.b0, (int32_t)L.b1, (int32_t)nf, rk0, sh0,
                           L.c_out};
        n0 = L.b1 * 256;
        rk0 += g.nsegs();
        b0 = L.b1;
        sh0 += g.nx + 2;
        pl0 += g.nx;
    }
    unsigned long long bad = 0;
    std::vector<double> tau_sum(count);
    LBM_TRY_HIP(hipMemcpyAsync(&bad, w.counter, sizeof(bad), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipMemcpyAsync(tau_sum.data(), w.tau_sum, sizeof(double) * count,
                               hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipMemcpyAsync(w.lats, lats.data(), sizeof(KnLat) * count, hipMemcpyHostToDevice, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    LBM_REQUIRE(bad == 0, LBM_E_INVAL, "%llu fluid nodes have tau_g <= 1/2 (pore diameter <= 0)", bad);

    // the active lattices in groups
    std::vector<int32_t> act(count), blocks_h, lat_ids_h, planes_h;
    std::vector<KnBlk> descs_h;
    for (int l = 0; l < count; l++) act[l] = l;
    std::vector<BatchGroup> groups;
    auto regroup = [&](double budget) -> lbm_status {
        groups = form_groups(act, bl, kBatchKnNodeBytes, budget, blocks_h, lat_ids_h, &planes_h);
        descs_h.resize(blocks_h.size());
        for (size_t k = 0; k < blocks_h.size(); k++) descs_h[k] = blk[blocks_h[k]];
        LBM_TRY_HIP(hipMemcpyAsync(w.lat_ids, lat_ids_h.data(), sizeof(int32_t) * lat_ids_h.size(),
                                   hipMemcpyHostToDevice, s));
        LBM_TRY_HIP(hipMemcpyAsync(w.descs, descs_h.data(), sizeof(KnBlk) * descs_h.size(),
                                   hipMemcpyHostToDevice, s));
        LBM_TRY_HIP(hipMemcpyAsync(w.planes, planes_h.data(), sizeof(int32_t) * planes_h.size(),
                                   hipMemcpyHostToDevice, s));
        LBM_TRY_HIP(hipStreamSynchronize(s));  // the host vectors are reused
        R.reset_graphs(groups.size());
        return LBM_OK;
    };
    const int32_t vbits = p->variant & kVariantBits;
    auto group_mode = [&](const BatchGroup &g) { return pick_variant7(vbits, (int64_t)g.nodes); };
    double live_nodes = 0.0;
    for (int l : act) live_nodes += (double)nf_h[l];

    // frame 0 holds the initial state; its plane means become the first pending frame
    st = regroup(-1.0);
    if (st != LBM_OK) return st;
    KnPos q;
    st = kn_batch_frames(w, groups[0], 0, p, s);
    if (st != LBM_OK) return st;
    q.pending = true;

    Sweep7 a{};
    a.stride = w.stride;
    a.coords = w.coords;
    a.rank = w.rank;
    a.omega = w.omega;
    a.csnap = w.csnap;
    a.partials = w.partials;

    const int64_t limit = p->fixed_steps > 0 ? p->fixed_steps : p->max_steps;
    const int nc = p->check_every;
    const bool use_graph = !(p->variant & LBM_VARIANT_NOGRAPH);
    int64_t t = 0;
    double sweep_ms = 0.0, updates = 0.0, tune_ms = 0.0;

    // every group of an interval starts from the same position and ends in the same one
    auto run_groups = [&](int64_t steps, bool check_last) -> lbm_status {
        KnPos end = q;
        for (const BatchGroup &g : groups) {
            end = q;
            lbm_status e = kn_batch_steps(w, a, group_mode(g), g, end, steps, check_last, p, s);
            if (e != LBM_OK) return e;
        }
        q = end;
        return LBM_OK;
    };

    // schedule, as in the batched flow solve: a given budget, or one tuning interval per
    // candidate and the fastest for the rest
    const double cand[kBatchBudgets] = LBM_BATCH_BUDGETS;
    const bool tuning = !sched || sched->group_bytes == 0;
    int tune_k = tuning ? 0 : kBatchBudgets;
    double budget = tuning ? cand[0] : (double)sched->group_bytes, best_rate = INFINITY;
    st = regroup(budget);
    if (st != LBM_OK) return st;
    int32_t groups_run = tuning ? -1 : (int32_t)groups.size();

    std::vector<double> res((size_t)count * kKnSums, 0.0), sums_l((size_t)count * kKnSums, 0.0);
    std::vector<int64_t> steps_l(count, 0);
    std::vector<double> resid_l(count, INFINITY);
    std::vector<SteadyEst> est_l(count);
    std::vector<int> conv_l(count, 0), cur_l(count, 0), frame_l(count, 0);
    std::vector<double> planes(w.ntab);
    bool diverged = false;
    while (t < limit && !act.empty()) {
        const int64_t chunk = std::min<int64_t>(nc - (t % nc), limit - t);
        if (use_graph && chunk == nc && q.pending) {
            // one graph per group and (buffer, frame) at the start of the interval, captured
            // before the timed region
            const int key = q.cur * 2 + q.frame;
            for (size_t gi = 0; gi < groups.size(); gi++) {
                hipGraphExec_t &ex = R.exec[gi * BatchRes::kKeys + key];
                if (ex) continue;
                KnPos qc = q;
                LBM_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                st = kn_batch_steps(w, a, group_mode(groups[gi]), groups[gi], qc, chunk, true, p, s);
                hipGraph_t graph = nullptr;
                hipError_t ec = hipStreamEndCapture(s, &graph);
                if (st != LBM_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return st;
                }
                LBM_TRY_HIP(ec);
                R.graph[gi * BatchRes::kKeys + key] = graph;
                LBM_TRY_HIP(hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0));
            }
            LBM_TRY_HIP(hipEventRecord(R.e0, s));
            for (size_t gi = 0; gi < groups.size(); gi++)
                LBM_TRY_HIP(hipGraphLaunch(R.exec[gi * BatchRes::kKeys + key], s));
            // the position after the interval: one frame change, chunk buffer swaps
            q.frame ^= 1;
            q.cur ^= (int)(chunk & 1);
            q.pending = true;
        } else {
            LBM_TRY_HIP(hipEventRecord(R.e0, s));
            st = run_groups(chunk, true);
            if (st != LBM_OK) return st;
        }
        LBM_TRY_HIP(hipEventRecord(R.e1, s));
        LBM_TRY_HIP(hipMemcpyAsync(res.data(), w.res, sizeof(double) * count * kKnSums,
                                   hipMemcpyDeviceToHost, s));
        LBM_TRY_HIP(hipStreamSynchronize(s));
        float ms = 0.f;
        LBM_TRY_HIP(hipEventElapsedTime(&ms, R.e0, R.e1));
        sweep_ms += ms;
        updates += (double)chunk * live_nodes;
        bool regroup_now = false;
        if (tune_k < kBatchBudgets) {
            tune_ms += ms;
            const double rate = ms / ((double)chunk * live_nodes);
            if (rate < best_rate) {
                best_rate = rate;
                budget = cand[tune_k];
            }
            ++tune_k;
            regroup_now = tune_k < kBatchBudgets || budget != cand[kBatchBudgets - 1];
        }
        t += chunk;
        std::vector<int32_t> keep, below;
        for (int l : act) {
            const double *sm = res.data() + (size_t)l * kKnSums;
            std::copy(sm, sm + kKnSums, sums_l.begin() + (size_t)l * kKnSums);
            steps_l[l] = t;
            cur_l[l] = q.cur;
            frame_l[l] = q.frame;  // the pending frame is not entered by a retired lattice
            if (!std::isfinite(sm[0]) || !std::isfinite(sm[1]) || !std::isfinite(sm[2])) {
                diverged = true;
                continue;
            }
            if (t % nc == 0) {
                resid_l[l] = std::sqrt(sm[0]) / ((double)nc * std::sqrt(sm[1]));
                est_l[l].push(resid_l[l]);
                if (p->fixed_steps <= 0 && resid_l[l] < p->tol) below.push_back(l);
            }
        }
        if (diverged) break;
        if (!below.empty() && p->steady_tol > 0.0) {
            // the steady-state test of the single solve, for the lattices below tol
            for (int l : below) {
                const KnLat &L = lats[l];
                st = kn_plane_fluxes(L.g, w.rank + L.rk0, w.g[q.cur] + 7 * L.b0 * 256,
                                     w.steady[q.frame] + L.sh0, w.fpart + L.sh0 * kPlaneParts,
                                     w.plane + L.sh0, LBM_LATTICE_D3Q7, s);
                if (st != LBM_OK) return st;
            }
            LBM_TRY_HIP(hipMemcpyAsync(planes.data(), w.plane, sizeof(double) * w.ntab,
                                       hipMemcpyDeviceToHost, s));
            LBM_TRY_HIP(hipStreamSynchronize(s));
        }
        for (int l : act) {
            bool done = false;
            if (std::find(below.begin(), below.end(), l) != below.end()) {
                done = p->steady_tol <= 0.0 ||
                       plane_spread(planes.data() + lats[l].sh0, lats[l].g.nx + 1,
                                    kn_spread_floor(lats[l].g, p, LBM_LATTICE_D3Q7)) <=
                           p->steady_tol;
                conv_l[l] = done;
            }
            if (!done) keep.push_back(l);
        }
        if (keep.size() != act.size()) {
            act = keep;
            live_nodes = 0.0;
            for (int l : act) live_nodes += (double)nf_h[l];
            regroup_now = true;
        }
        if (regroup_now && !act.empty()) {
            st = regroup(tune_k < kBatchBudgets ? cand[tune_k] : budget);
            if (st != LBM_OK) return st;
        }
        if (tune_k == kBatchBudgets && groups_run < 0) groups_run = (int32_t)groups.size();
    }
    if (sched) {
        sched->variant = vbits | (p->variant & LBM_VARIANT_NOGRAPH);
        sched->group_bytes_run = (int64_t)budget;
        sched->groups = groups_run < 0 ? (int32_t)groups.size() : groups_run;
        sched->tune_ms = tune_ms;
    }

    // link-plane fluxes of each lattice's final state, then the results
    for (int l = 0; l < count; l++) {
        const KnLat &L = lats[l];
        st = kn_plane_fluxes(L.g, w.rank + L.rk0, w.g[cur_l[l]] + 7 * L.b0 * 256,
                             w.steady[frame_l[l]] + L.sh0, w.fpart + L.sh0 * kPlaneParts,
                             w.plane + L.sh0, LBM_LATTICE_D3Q7, s);
        if (st != LBM_OK) return st;
    }
    LBM_TRY_HIP(hipMemcpyAsync(planes.data(), w.plane, sizeof(double) * w.ntab,
                               hipMemcpyDeviceToHost, s));
    st = R.close(caller);
    if (st != LBM_OK) return st;
    LBM_TRY_HIP(hipStreamSynchronize(s));
    for (int l = 0; l < count; l++) {
        kn_result(r_h + l, p, lats[l].g, nf_h[l], steps_l[l], conv_l[l], resid_l[l],
                  sums_l.data() + (size_t)l * kKnSums, tau_sum[l], planes.data() + lats[l].sh0,
                  sweep_ms, updates, LBM_LATTICE_D3Q7);
        r_h[l].steady_dist = est_l[l].dist(nc);
    }
    if (diverged) {
        set_error("batched Knudsen solve diverged (NaN/Inf) by step %lld", (long long)t);
        return LBM_E_DIVERGED;
    }
    for (int l = 0; l < count; l++)
        if (!conv_l[l] && p->fixed_steps <= 0) {
            set_error("lattice %d not converged after %lld steps", l, (long long)steps_l[l]);
            return LBM_W_NOT_CONVERGED;
        }
    return LBM_OK;
}
