// D3Q19 flow solve: fused pull-stream + BGK collision + Guo body force with half-way
// bounce-back, on the sparse fluid-node list (Section 3.1, Eqs. 1-3, 8-9; Section 3.3;
// Darcy's law, Eq. 13).
//
// Storage: blocks of 256 nodes, each with its 19 arrays of 256 side by side (pop19).  Two
// buffers, ping-pong.  Per fluid-node update the method moves 19 loads + 19 stores of 8,
// 4 or 2 bytes.
//
// binary64 (collision in binary64) stores the offsets f_i - w_i.  binary32 and binary16
// (collision in binary32) store offsets from the equilibrium at rest of a reference
// density per row segment: h_i = S (f_i - w_i (1 + r_s)), with r_s one binary32 value per
// 32-voxel half row segment (r(x) = a + b (x mod 32), fitted to rho - 1 of its nodes) and
// S = 1 for binary32, S = 2^k with S max|F| in [1, 2) for binary16.  In low-permeability
// media the body force is held by pressure (dead ends, tortuous paths), and the density
// part w_i (rho - 1) of f_i - w_i exceeds the velocity part by up to four decades: stored
// relative to w_i alone, binary32 loses ~4e-4 of k on the 128^3 crop of the 512^3
// workload and binary16 loses u entirely.  Where the fluid is still, the pressure is
// hydrostatic under the body force, linear along x, so a linear reference per half
// segment leaves the stored values the velocity and non-equilibrium parts (a constant
// one per segment, tried first, left binary16 5.8 % off on the crop).  The collision
// runs on offsets from the node's own reference (a pulled value is moved there by
// w_i (r_source - r_own)), with rho = 1 + r_own + sum_i h_i; Eq. 3's f_eq and the MRT
// equilibrium moments are linear in the density, so only the density offset changes.
// The references are fitted at each convergence check; the first sweep after it reads
// the state relative to the old references and writes it relative to the new ones.
// They live in the flow's rank records beside each half's occupancy and first node id
// (FlowHalf, 16 bytes), so a pull costs one load for both.
#include <algorithm>
#include <vector>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "lbm_internal.h"

namespace lbm {

constexpr uint64_t kFlowMagic = 0x4c424d464c4f5737ull;  // "LBMFLOW7"
constexpr int kFlowSums = 6;      // |du|^2, |u|^2, rho u (3), rho - 1
constexpr int kSampleMax = 65536;

struct FlowHeader {
    uint64_t magic;
    int32_t nx, ny, nz, cur;
    int64_t n_fluid, steps_done;
    double tau, force[3];
    int32_t variant, storage;
    double scale;  // binary16 storage: stored = scale * (f_i - w_i)
    int32_t collision;
    int32_t boundary;          // LBM_BOUNDARY_*
    double rho_in, rho_out;    // pressure boundaries
    int32_t sref;              // 1: offsets from reference densities (binary32, binary16)
    int32_t sref_pending;      // 1: href_next holds references of the last check that the
                               // next sweep moves the state to
};

// The flow sweep's record of a half row segment (32 voxels): its occupancy bits and the
// id of its first fluid node, as in the rank map, beside the linear reference density
// r(x) = a + b (x mod 32) the stored state of its nodes is relative to.
struct alignas(16) FlowHalf {
    uint32_t bits, base;
    float a, b;
};

__host__ __device__ inline int64_t half_index(int64_t seg, int x) { return 2 * seg + ((x >> 5) & 1); }
__device__ inline float half_ref(float a, float b, int x) {
    return __builtin_fmaf(b, (float)(x & 31), a);
}
// Node id at bit `bit` (= x % 64) of the half record holding it, or -1 for a solid voxel.
__device__ inline int flow_lookup(const FlowHalf &h, int bit) {
    const int b = bit & 31;
    if (!((h.bits >> b) & 1u)) return -1;
    return (int)(h.base + (uint32_t)__popc(h.bits & ((1u << b) - 1u)));
}

// Pressure boundaries: the populations entering through the inlet (e_x = +1) and the
// outlet (e_x = -1), five each, and their slot in the ghost-plane buffer
// [side][slot][ny nz].
#define LBM_GHOST_TABLES                                                                   \
    [[maybe_unused]] constexpr int GIN[5] = {1, 7, 9, 11, 13};                             \
    [[maybe_unused]] constexpr int GOUT[5] = {2, 8, 10, 12, 14};                           \
    [[maybe_unused]] constexpr int GSLOT[19] = {-1, 0, 0, -1, -1, -1, -1, 1, 1, 2, 2,      \
                                                3, 3, 4, 4, -1, -1, -1, -1};

// Storage policies: T is the stored type, R the collision arithmetic.
struct StoreF32 {
    using T = float;
    using R = float;
};
struct StoreF64 {
    using T = double;
    using R = double;
};
struct StoreF16 {
    using T = _Float16;
    using R = float;
};

static int pop_bytes(int32_t storage) {
    return storage == LBM_STORE_FP16 ? 2 : (storage == LBM_STORE_FP64 ? 8 : 4);
}

// Algorithmic HBM bytes per fluid-node update: 19 population loads and stores.
static double flow_bytes_per_update(int32_t storage) { return 38.0 * pop_bytes(storage); }

template <class P>
__device__ inline typename P::R from_store(typename P::T v, float inv_scale) {
    if constexpr (std::is_same<typename P::T, _Float16>::value)
        return (float)v * inv_scale;  // a power of two: exact
    else
        return v;
}

template <class P>
__device__ inline typename P::T to_store(typename P::R v, float scale) {
    if constexpr (std::is_same<typename P::T, _Float16>::value)
        return (_Float16)(v * scale);  // round to nearest even
    else
        return v;
}

template <class R>
__device__ inline R par(float f, double d) {
    if constexpr (std::is_same<R, double>::value)
        return d;
    else
        return f;
}

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
    void *f[2];
    FlowHalf *fh;      // half-segment records with the references (binary32, binary16)
    float2 *href_next; // references fitted at the last check, (a, b) per half segment
    float *dsnap;      // rho - 1 per node at the last check
    float *usnap;
    double *partials;
    void *ghost;     // pressure boundaries: ghost-plane populations [2][5][ny nz]
    int64_t stride;  // distance between population arrays (elements)
    size_t bytes;
};

static int64_t blocks_for(int64_t nf) { return (nf + 255) / 256; }

// Population i of fluid node m.  The nodes go in blocks of 256; each block keeps its 19
// arrays of 256 side by side (19 KB in binary32), so that the populations a wave pulls
// from its own and its neighbouring rows lie in few pages: with one array of the whole
// lattice per direction a 512^3 sweep took 7.7 M translation misses per launch, and this
// layout runs it 13 % faster.  A wave's 64 consecutive nodes still read and write 256 B
// runs.
__host__ __device__ inline int64_t pop19(int i, int64_t m) {
    return ((m >> 8) * 19 + i) * 256 + (m & 255);
}

static FlowWs carve_flow(void *base, const Grid &g, int64_t nf, int32_t storage) {
    FlowWs w;
    Carver c(base);
    w.hdr = c.take<FlowHeader>(1);
    w.counter = c.take<unsigned long long>(4);
    w.res = c.take<double>(32);
    w.total = c.take<int32_t>(1);
    w.rank = c.take<RankWord>(g.nsegs());
    const size_t nhalf = storage == LBM_STORE_FP64 ? 0 : 2 * (size_t)g.nsegs();
    w.fh = c.take<FlowHalf>(nhalf);
    w.href_next = c.take<float2>(nhalf);
    w.samp_vox = c.take<int64_t>(kSampleMax);
    w.samp_out = c.take<double>((size_t)kSampleMax * 19);
    w.samp_flag = c.take<uint8_t>(kSampleMax);
    int64_t nfp = nf < 1 ? 1 : nf;
    w.stride = (nfp + 255) / 256 * 256;  // whole blocks of 256 nodes (pop19)
    w.coords = c.take<uint32_t>(nfp);
    w.f[0] = c.take<char>((size_t)19 * w.stride * pop_bytes(storage));
    w.f[1] = c.take<char>((size_t)19 * w.stride * pop_bytes(storage));
    w.dsnap = c.take<float>(storage == LBM_STORE_FP64 ? 0 : (size_t)w.stride);
    w.usnap = c.take<float>((size_t)3 * w.stride);
    w.partials = c.take<double>((size_t)xcd_launch(blocks_for(nfp)) * kFlowSums);
    w.ghost = c.take<double>((size_t)10 * g.ny * g.nz);
    w.bytes = c.off;
    return w;
}

size_t flow_ws_bytes(const Grid &g, int64_t nf, int32_t storage) {
    return carve_flow(nullptr, g, nf, storage).bytes;
}

struct Sweep19 {
    Grid g;
    int64_t nf, stride, launched;
    int64_t launched_live;             // batched solves: blocks of the launch with work
    const uint32_t *__restrict__ coords;
    const RankWord *__restrict__ rank;
    const void *__restrict__ src;
    void *__restrict__ dst;
    const FlowHalf *__restrict__ fh;       // half records with the references read
    const float2 *__restrict__ href_next;  // references written (when reframe)
    int reframe;                           // 1: write relative to href_next
    float *__restrict__ dsnap;             // check variant: rho - 1 per node
    float omega, fpre, Fx, Fy, Fz, sq; // collision parameters for binary32 arithmetic
    double omega_d, fpre_d, Fd[3], sq_d;  // and for binary64 (sq: the MRT rate s_q)
    float scale, inv_scale;            // binary16 storage scale
    int64_t chunk;                     // XCD remap run length in blocks (0: none)
    // check variant
    float *__restrict__ usnap;
    float *__restrict__ u_out;
    double *__restrict__ partials;
    int update_snap;
    int with_rho;                      // u_out carries a fourth plane, rho - 1
    const void *__restrict__ ghost;    // pressure boundaries: [2][5][ny nz] ghost populations
};

// Kernel variants (chosen per solve from the working-set size, or forced):
//   REMAP: XCD-contiguous workgroup order, so neighbouring rows share an L2;
//   NT: populations are written with streaming (non-temporal) stores; right when the
//     arrays far exceed the 256 MB Infinity Cache, wrong when they fit in it.

// The MRT collision (Section 3.1, Eqs. 4-7, Appendix A) on the offsets f_i - w_i: their
// moments under the transformation matrix Q of Appendix A (rows: moments, columns: the
// velocities in the order above), relaxed towards the equilibrium moments A1-A9 (rho0 = 1,
// j including F/2; written as offsets from those of rest) at the rates of Eq. 7, plus
// Guo's source in moment space scaled by (1 - s_k/2); back through Q^-1 = Q^T / |Q_k|^2
// (Q's rows are orthogonal).
#define LBM_MRT_Q                                                                                  \
    constexpr int MQ[19][19] = {                                                                   \
        {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},                                 \
        {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},                   \
        {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},                          \
        {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},                            \
        {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},                            \
        {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},                            \
        {0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},                            \
        {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},                            \
        {0, 0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},                            \
        {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},                         \
        {0, -4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},                           \
        {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},                           \
        {0, 0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},                           \
        {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},                               \
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},                               \
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},                               \
        {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},                             \
        {0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1},                             \
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1}};

constexpr int mrt_norm2(int k) {
    LBM_MRT_Q
    int s = 0;
    for (int i = 0; i < 19; i++) s += MQ[k][i] * MQ[k][i];
    return s;
}

// Relaxation class of moment k under Eq. 7: 0 conserved, 1 rate 1/tau, 2 rate s_q.
constexpr int mrt_class(int k) {
    return (k == 0 || k == 3 || k == 5 || k == 7) ? 0
           : (k == 4 || k == 6 || k == 8 || k >= 16) ? 2
                                                       : 1;
}

// Rows of Q are even or odd under e -> -e (density, energy and stress moments even; the
// momentum, heat flux and third-order moments odd), so each transform works on the sums
// and differences of the nine pairs of opposite velocities.
constexpr int kMrtOpp[19] = {0, 2, 1, 4, 3, 6, 5, 10, 9, 8, 7, 14, 13, 12, 11, 18, 17, 16, 15};
constexpr bool mrt_even(int k) {
    LBM_MRT_Q
    for (int i = 0; i < 19; i++)
        if (MQ[k][i] != MQ[k][kMrtOpp[i]]) return false;
    return true;
}
constexpr bool mrt_odd(int k) {
    LBM_MRT_Q
    for (int i = 0; i < 19; i++)
        if (MQ[k][i] != -MQ[k][kMrtOpp[i]]) return false;
    return true;
}
constexpr bool mrt_rows_split() {
    for (int k = 0; k < 19; k++)
        if (!mrt_even(k) && !mrt_odd(k)) return false;
    return true;
}
static_assert(mrt_rows_split(), "every row of Q is even or odd under e -> -e");

template <class R>
__device__ inline void mrt_collide(const R (&f)[19], R drho, R jx, R jy, R jz, R ux, R uy, R uz,
                                   R Fx, R Fy, R Fz, R s_nu, R s_q, R (&out)[19]) {
    LBM_D3Q19_TABLES
    LBM_MRT_Q
    const R W0 = R(1) / R(3), W1 = R(1) / R(18), W2 = R(1) / R(36);
    const R uF = ux * Fx + uy * Fy + uz * Fz;
    // pair sums and differences of f and of Guo's source w_i [3 (e.F - u.F) + 9 (e.u)(e.F)]
    // (the source's sum over a pair is 2 w_i [9 (e.u)(e.F) - 3 u.F], its difference
    // 6 w_i e.F)
    R fs[19], fd[19], ss[19], sd[19];
#pragma unroll
    for (int i = 1; i < 19; i++) {
        if (OPP[i] < i) continue;
        const R w = i < 7 ? W1 : W2;
        const R eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        const R eF = EX[i] * Fx + EY[i] * Fy + EZ[i] * Fz;
        fs[i] = f[i] + f[OPP[i]];
        fd[i] = f[i] - f[OPP[i]];
        ss[i] = R(2) * w * (R(9) * eu * eF - R(3) * uF);
        sd[i] = R(6) * w * eF;
    }
    const R s0 = W0 * (R(-3) * uF);
    const R jj = jx * jx + jy * jy + jz * jz;
    const R t9 = R(3) * jx * jx - jj, t11 = jy * jy - jz * jz;
    const R meq[19] = {drho, R(-11) * drho + R(19) * jj, R(3) * drho - R(5.5) * jj,
                       jx, R(-2) / R(3) * jx, jy, R(-2) / R(3) * jy, jz, R(-2) / R(3) * jz,
                       t9, R(-0.5) * t9, t11, R(-0.5) * t11, jx * jy, jy * jz, jx * jz,
                       R(0), R(0), R(0)};
    R ms[19];
#pragma unroll
    for (int k = 0; k < 19; k++) {
        const bool ev = mrt_even(k);
        R m = 0, fm = 0;
        if (ev && MQ[k][0] != 0) {
            m = R(MQ[k][0]) * f[0];
            fm = R(MQ[k][0]) * s0;
        }
#pragma unroll
        for (int i = 1; i < 19; i++) {
            if (OPP[i] < i || MQ[k][i] == 0) continue;
            m += R(MQ[k][i]) * (ev ? fs[i] : fd[i]);
            fm += R(MQ[k][i]) * (ev ? ss[i] : sd[i]);
        }
        const R sk = mrt_class(k) == 0 ? R(0) : (mrt_class(k) == 1 ? s_nu : s_q);
        ms[k] = (m - sk * (m - meq[k]) + (R(1) - R(0.5) * sk) * fm) * R(1.0 / mrt_norm2(k));
    }
    // back through Q^T / |Q_k|^2: for each pair the even rows give E, the odd ones O, and
    // the pair's members are E + O and E - O
    {
        R v = 0;
#pragma unroll
        for (int k = 0; k < 19; k++)
            if (mrt_even(k) && MQ[k][0] != 0) v += R(MQ[k][0]) * ms[k];
        out[0] = v;
    }
#pragma unroll
    for (int i = 1; i < 19; i++) {
        if (OPP[i] < i) continue;
        R e = 0, o = 0;
#pragma unroll
        for (int k = 0; k < 19; k++) {
            if (MQ[k][i] == 0) continue;
            if (mrt_even(k))
                e += R(MQ[k][i]) * ms[k];
            else
                o += R(MQ[k][i]) * ms[k];
        }
        out[i] = e + o;
        out[OPP[i]] = e - o;
    }
}

// The same collision in its two-relaxation-time form (Eq. 7 relaxes every even
// non-conserved moment at 1/tau and every odd one at s_q, towards the incompressible
// equilibrium of Appendix A): for each pair of opposite velocities the even part of the
// offsets relaxes at s+ = 1/tau towards w_i [drho + 9/2 (e.j)^2 - 3/2 j^2], the odd part
// at s- = s_q towards 3 w_i e.j (j = rho u including F/2); Guo's source splits alike,
// each part scaled by (1 - s/2).  fpre = 1 - s+/2.
template <class R>
__device__ inline void trt_collide(const R (&f)[19], R drho, R jx, R jy, R jz, R ux, R uy, R uz,
                                   R Fx, R Fy, R Fz, R s_nu, R s_q, R fpre, R (&out)[19]) {
    LBM_D3Q19_TABLES
    const R W0 = R(1) / R(3), W1 = R(1) / R(18), W2 = R(1) / R(36);
    const R jj15 = R(1.5) * (jx * jx + jy * jy + jz * jz);
    const R uF3 = R(3) * (ux * Fx + uy * Fy + uz * Fz);
    const R mpre = R(1) - R(0.5) * s_q;
    out[0] = f[0] - s_nu * (f[0] - W0 * (drho - jj15)) - fpre * W0 * uF3;
#pragma unroll
    for (int i = 1; i < 19; i++) {
        if (OPP[i] < i) continue;  // each pair once, from its first member
        const int k = OPP[i];
        const R w = i < 7 ? W1 : W2;
        const R ej = EX[i] * jx + EY[i] * jy + EZ[i] * jz;
        const R eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        const R eF = EX[i] * Fx + EY[i] * Fy + EZ[i] * Fz;
        const R even = R(0.5) * (f[i] + f[k]) - w * (drho + R(4.5) * ej * ej - jj15);
        const R odd = R(0.5) * (f[i] - f[k]) - w * R(3) * ej;
        const R se = fpre * w * (R(9) * eu * eF - uF3);
        const R so = mpre * w * R(3) * eF;
        const R de = se - s_nu * even, dd = so - s_q * odd;
        out[i] = f[i] + de + dd;
        out[k] = f[k] + de - dd;
    }
}

// The update of fluid node n at (x, y, z) whose 18 pull sources are resolved: ids[i] is
// the node at x - e_i, -1 when that voxel is solid (half-way bounce-back), -2 a ghost
// node beyond an x face (pressure boundaries); rs[i] the reference density at the source
// (rs[0]: at the node), binary32 and binary16 storage.
template <class P, bool CHECK, bool NT, int COLL, bool OPEN, class Off>
__device__ inline void node19(const Sweep19 &a, int64_t n, int x, int y, int z,
                              const int (&ids)[19], const float (&rs)[19],
                              int64_t half_own, double (&acc)[kFlowSums]) {
    using T = typename P::T;
    using R = typename P::R;
    LBM_D3Q19_TABLES
    const R W0 = R(1) / R(3), W1 = R(1) / R(18), W2 = R(1) / R(36);
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const R omega = par<R>(a.omega, a.omega_d), fpre = par<R>(a.fpre, a.fpre_d);
    const R Fx = par<R>(a.Fx, a.Fd[0]), Fy = par<R>(a.Fy, a.Fd[1]), Fz = par<R>(a.Fz, a.Fd[2]);
    // element offsets pop19(i, node): 32-bit while 19 * stride fits (fewer registers),
    // 64-bit beyond
    Off off[19];
    off[0] = (Off)pop19(0, n);
#pragma unroll
    for (int i = 1; i < 19; i++)
        off[i] = ids[i] >= 0 ? (Off)pop19(i, ids[i]) : (Off)pop19(OPP[i], n);
    R f[19];
#pragma unroll
    for (int i = 0; i < 19; i++) f[i] = from_store<P>(src[off[i]], a.inv_scale);
    if constexpr (OPEN) {
        // sources beyond an x face: the ghost planes of the pressure boundaries (-2), at
        // [side][slot][z_s ny + y_s] with (y_s, z_s) the source's row (periodic in y, z);
        // only the boundary nodes take this branch, so the indices are formed here
        LBM_GHOST_TABLES
        if (x == 0 || x == a.g.nx - 1) {
            const T *__restrict__ gh = static_cast<const T *>(a.ghost);
            const int ny = a.g.ny, nz = a.g.nz;
#pragma unroll
            for (int i = 1; i < 19; i++) {
                if (EX[i] == 0 || ids[i] != -2) continue;
                const int side = EX[i] == 1 ? 0 : 1;
                int ys = y - EY[i], zs = z - EZ[i];
                ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
                zs = zs < 0 ? zs + nz : (zs >= nz ? zs - nz : zs);
                f[i] = from_store<P>(gh[((side * 5 + GSLOT[i]) * nz + zs) * ny + ys], a.inv_scale);
            }
        }
    }
    constexpr bool kRef = !std::is_same<T, double>::value;
    if constexpr (kRef) {
        // move pulled values to offsets from the node's own segment reference (sources in
        // another segment; a ghost value is relative to its boundary node's segment,
        // which rs[i] holds); the rest population and bounced ones are the node's own
#pragma unroll
        for (int i = 1; i < 19; i++)
            if (ids[i] >= 0 || (OPEN && ids[i] == -2))  // one rounding, in every variant
                f[i] = __builtin_fmaf(i < 7 ? 1.f / 18.f : 1.f / 36.f, rs[i] - rs[0], f[i]);
    }

    // drho: the density offset from 1 + rs[0] (from 1 for binary64)
    R drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < 19; i++) {
        drho += f[i];
        if (EX[i]) jx += EX[i] > 0 ? f[i] : -f[i];
        if (EY[i]) jy += EY[i] > 0 ? f[i] : -f[i];
        if (EZ[i]) jz += EZ[i] > 0 ? f[i] : -f[i];
    }
    const R rho = kRef ? (R(1) + R(rs[0])) + drho : R(1) + drho;
    const R inv = R(1) / rho;
    const R mx = jx + R(0.5) * Fx, my = jy + R(0.5) * Fy, mz = jz + R(0.5) * Fz;
    const R ux = mx * inv, uy = my * inv, uz = mz * inv;
    R posts[19];
    if constexpr (COLL == LBM_COLLIDE_MRT) {
        mrt_collide<R>(f, drho, mx, my, mz, ux, uy, uz, Fx, Fy, Fz, omega, par<R>(a.sq, a.sq_d),
                       posts);
    } else if constexpr (COLL == LBM_COLLIDE_TRT) {
        trt_collide<R>(f, drho, mx, my, mz, ux, uy, uz, Fx, Fy, Fz, omega, par<R>(a.sq, a.sq_d),
                       fpre, posts);
    } else {
        const R uu15 = R(1.5) * (ux * ux + uy * uy + uz * uz);
        const R uF = ux * Fx + uy * Fy + uz * Fz;
#pragma unroll
        for (int i = 0; i < 19; i++) {
            const R w = i == 0 ? W0 : (i < 7 ? W1 : W2);
            const R eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
            const R eF = EX[i] * Fx + EY[i] * Fy + EZ[i] * Fz;
            const R feq = w * (drho + rho * (R(3) * eu + R(4.5) * eu * eu - uu15));
            const R srcf = fpre * w * (R(3) * (eF - uF) + R(9) * eu * eF);
            posts[i] = f[i] - omega * (f[i] - feq) + srcf;
        }
    }
    R shift = 0;  // the first sweep of a check interval moves to the new references
    if constexpr (kRef)
        if (a.reframe) {
            const float2 nx = a.href_next[half_own];
            shift = R(rs[0]) - R(half_ref(nx.x, nx.y, x));
        }
#pragma unroll
    for (int i = 0; i < 19; i++) {
        const R w = i == 0 ? W0 : (i < 7 ? W1 : W2);
        R post = posts[i];
        if constexpr (kRef) post = __builtin_fmaf(w, shift, post);
        const T out = to_store<P>(post, a.scale);
        if (NT)
            __builtin_nontemporal_store(out, &dst[pop19(i, n)]);
        else
            dst[pop19(i, n)] = out;
    }
    if (CHECK) {
        const R drho_abs = kRef ? R(rs[0]) + drho : drho;  // rho - 1
        if constexpr (kRef) a.dsnap[n] = (float)drho_abs;
        const double dux = (double)ux - (double)a.usnap[n];
        const double duy = (double)uy - (double)a.usnap[a.stride + n];
        const double duz = (double)uz - (double)a.usnap[2 * a.stride + n];
        acc[0] += dux * dux + duy * duy + duz * duz;
        acc[1] += (double)ux * ux + (double)uy * uy + (double)uz * uz;
        acc[2] += (double)jx + 0.5 * (double)Fx;
        acc[3] += (double)jy + 0.5 * (double)Fy;
        acc[4] += (double)jz + 0.5 * (double)Fz;
        acc[5] += kRef ? (double)rs[0] + (double)drho : (double)drho;
        if (a.update_snap) {
            a.usnap[n] = (float)ux;
            a.usnap[a.stride + n] = (float)uy;
            a.usnap[2 * a.stride + n] = (float)uz;
        }
        if (a.u_out) {
            const int64_t v = a.g.lin(x, y, z), nv = a.g.nvox();
            a.u_out[v] = (float)ux;
            a.u_out[nv + v] = (float)uy;
            a.u_out[2 * nv + v] = (float)uz;
            if (a.with_rho) a.u_out[3 * nv + v] = (float)drho_abs;
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

// The update of fluid node n (n < a.nf): its coordinates, the 18 pull sources from the
// rank map (one batch of loads), then node19.
template <class P, bool CHECK, bool NT, int COLL, bool OPEN, class Off>
__device__ inline void sweep19_node(const Sweep19 &a, int64_t n, double (&acc)[kFlowSums]) {
    LBM_D3Q19_TABLES
    LBM_GHOST_TABLES
    const uint32_t c = a.coords[n];
    const int x = c & 1023, y = (c >> 10) & 1023, z = c >> 20;
    const Grid &g = a.g;
    // per-axis pieces of the rank word and bit of x-1, x, x+1 (periodic, or with pressure
    // boundaries the node's own x standing in beyond a face), etc.
    int xs[3], ys[3], zs[3];
    if (OPEN) {
        xs[0] = x == 0 ? x : x - 1; xs[1] = x; xs[2] = x == g.nx - 1 ? x : x + 1;
    } else {
        xs[0] = x == 0 ? g.nx - 1 : x - 1; xs[1] = x; xs[2] = x == g.nx - 1 ? 0 : x + 1;
    }
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
    // the 18 rank records (with the references) are loaded as one batch, then the 19
    // populations as another
    constexpr bool kRef = !std::is_same<P, StoreF64>::value;
    float rs[19];
    int ids[19];
    const int64_t half_own = half_index((int64_t)wx[1] + wy[1] + wz[1], x);
    if constexpr (kRef) {
        FlowHalf rh[19];
#pragma unroll
        for (int i = 1; i < 19; i++)
            rh[i] = a.fh[half_index((int64_t)wx[1 - EX[i]] + wy[1 - EY[i]] + wz[1 - EZ[i]],
                                    bx[1 - EX[i]])];
        const float2 own = *reinterpret_cast<const float2 *>(&a.fh[half_own].a);
        rs[0] = half_ref(own.x, own.y, x);
#pragma unroll
        for (int i = 1; i < 19; i++) {
            ids[i] = flow_lookup(rh[i], bx[1 - EX[i]]);
            rs[i] = half_ref(rh[i].a, rh[i].b, bx[1 - EX[i]]);
        }
    } else {
        RankHalf rh[19];
#pragma unroll
        for (int i = 1; i < 19; i++)
            rh[i] = rank_half(a.rank, (int64_t)wx[1 - EX[i]] + wy[1 - EY[i]] + wz[1 - EZ[i]],
                              bx[1 - EX[i]]);
#pragma unroll
        for (int i = 0; i < 19; i++) rs[i] = 0.f;
#pragma unroll
        for (int i = 1; i < 19; i++) ids[i] = half_lookup(rh[i], bx[1 - EX[i]]);
    }
    ids[0] = 0;
#pragma unroll
    for (int i = 1; i < 19; i++) {
        if (OPEN && ((EX[i] == 1 && x == 0) || (EX[i] == -1 && x == g.nx - 1))) {
            // the source is a ghost node; its boundary node (looked up at this x) decides:
            // fluid -> the ghost's population, solid -> bounce back
            ids[i] = ids[i] >= 0 ? -2 : -1;
        }
    }
    node19<P, CHECK, NT, COLL, OPEN, Off>(a, n, x, y, z, ids, rs, half_own, acc);
}

// One stream-collide step, one fluid node per thread.  CHECK also forms the FP64 partial
// sums of the convergence check and writes the velocity snapshot / field.
template <class P, bool CHECK, bool NT, int COLL, bool OPEN, class Off>
__global__ __launch_bounds__(256) void k_sweep19(Sweep19 a) {
    const int64_t lb = a.chunk ? xcd_block(blockIdx.x, a.chunk) : (int64_t)blockIdx.x;
    const int64_t n = lb * 256 + threadIdx.x;
    double acc[kFlowSums] = {0, 0, 0, 0, 0, 0};
    if (n < a.nf) sweep19_node<P, CHECK, NT, COLL, OPEN, Off>(a, n, acc);
    if (CHECK) write_partials<kFlowSums>(acc, lb, lb * 256 < a.nf, a.partials);
}

// ---------------------------------------------------------------- batched solves
// Many lattices in one launch, all with one set of collision parameters.  Lattice l owns
// the blocks [b0, b1) of the batch: its nodes are the local ids [0, nf) at offset
// n0 = 256 b0, and each of its arrays is a contiguous run at that offset with its own
// stride span = 256 (b1 - b0) (populations at 19 n0, snapshot at 3 n0), so that the state
// of consecutive lattices is one contiguous range, as in a single solve.  Launched block b
// runs the work that descs[b] describes: one 64-byte record, found with one scalar load.
struct BlkDesc19 {
    Grid g;          // the lattice's grid
    int32_t pb;      // physical block (partial-sum row)
    int32_t b0, b1;  // the lattice's blocks
    int32_t nf;      // its fluid nodes
    int64_t rk0;     // its first rank word (local ids)
    float *u_out;    // its velocity field, written at checks (nullable)
    int64_t pad;
};
static_assert(sizeof(BlkDesc19) == 64, "one record per launched block");

// Per lattice, for the reduction of a check: its physical blocks.
struct LatDesc {
    int64_t b0, b1;
};

template <bool CHECK, bool NT, int COLL>
__global__ __launch_bounds__(256) void k_sweep19b(Sweep19 a, const BlkDesc19 *__restrict__ descs) {
    const int64_t lb = a.chunk ? xcd_block(blockIdx.x, a.chunk) : (int64_t)blockIdx.x;
    double acc[kFlowSums] = {0, 0, 0, 0, 0, 0};
    const bool live = lb < a.launched_live;
    int64_t pb = 0;
    if (live) {
        const BlkDesc19 D = descs[lb];
        pb = D.pb;
        const int64_t n0 = (int64_t)D.b0 * 256;
        Sweep19 b = a;
        b.g = D.g;
        b.nf = D.nf;
        b.stride = (int64_t)(D.b1 - D.b0) * 256;
        b.coords = a.coords + n0;
        b.rank = a.rank + D.rk0;
        b.src = static_cast<const float *>(a.src) + 19 * n0;
        b.dst = static_cast<float *>(a.dst) + 19 * n0;
        b.fh = a.fh + 2 * D.rk0;
        b.href_next = a.href_next + 2 * D.rk0;
        b.dsnap = a.dsnap + n0;
        b.usnap = a.usnap + 3 * n0;
        b.u_out = D.u_out;
        const int64_t n = (pb - D.b0) * 256 + threadIdx.x;
        if (n < D.nf) sweep19_node<StoreF32, CHECK, NT, COLL, false, uint32_t>(b, n, acc);
    }
    if (CHECK) write_partials<kFlowSums>(acc, pb, live, a.partials);
}

// Pressure boundaries (Section 3.3), Guo's non-equilibrium extrapolation: the ghost node
// beyond boundary node b (x = 0 or nx - 1, same y, z) holds f(b) + f_eq(rho_bc, u_b) -
// f_eq(rho_b, u_b), with rho_b, u_b the moments of b's state (u_b = (j - F/2)/rho_b, the
// velocity of b's collision) and f_eq of Eq. 3; only the five populations entering the
// domain are kept, as offsets from w_i (1 + r) with r the reference density at b (from
// its half record fh; null for binary64 storage), in ghost[side][slot][z ny + y].  A
// ghost beside a solid b is solid (the sweep bounces back) and is not written.
template <class P>
__global__ __launch_bounds__(256) void k_ghost19(Grid g, const RankWord *__restrict__ rank,
                                                 const typename P::T *__restrict__ src,
                                                 const FlowHalf *__restrict__ fh,
                                                 float inv_scale, float scale,
                                                 typename P::R Fx, typename P::R Fy,
                                                 typename P::R Fz, typename P::R drho_in,
                                                 typename P::R drho_out,
                                                 typename P::T *__restrict__ ghost) {
    using R = typename P::R;
    LBM_D3Q19_TABLES
    LBM_GHOST_TABLES
    const int64_t m = (int64_t)g.ny * g.nz;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= 2 * m) return;
    const int side = (int)(t / m);
    const int64_t yz = t % m;
    const int y = (int)(yz % g.ny), z = (int)(yz / g.ny);
    const int xb = side ? g.nx - 1 : 0;
    const int id = node_at(rank, g, xb, y, z);
    if (id < 0) return;
    R ref = 0;
    if (fh) {
        const FlowHalf h = fh[half_index(g.seg(xb, y, z), xb)];
        ref = R(half_ref(h.a, h.b, xb));
    }
    R f[19], drho = 0, jx = 0, jy = 0, jz = 0;  // drho: offset from 1 + ref
#pragma unroll
    for (int i = 0; i < 19; i++) {
        f[i] = from_store<P>(src[pop19(i, id)], inv_scale);
        drho += f[i];
        jx += EX[i] * f[i];
        jy += EY[i] * f[i];
        jz += EZ[i] * f[i];
    }
    // the density jump from the offsets (rho_bc - 1) - (rho_b - 1): both near 0, so
    // binary32 keeps it to rounding (rho_bc - rho_b formed near 1 would lose ~1e-7)
    const R rho = (R(1) + ref) + drho, jump = ((side ? drho_out : drho_in) - ref) - drho;
    const R ux = (jx - R(0.5) * Fx) / rho, uy = (jy - R(0.5) * Fy) / rho, uz = (jz - R(0.5) * Fz) / rho;
    const R uu15 = R(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int k = 0; k < 5; k++) {
        const int i = side ? GOUT[k] : GIN[k];
        const R w = i < 7 ? R(1) / R(18) : R(1) / R(36);
        const R eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        const R v = f[i] + w * jump * (R(1) + R(3) * eu + R(4.5) * eu * eu - uu15);
        ghost[(side * 5 + k) * m + yz] = to_store<P>(v, scale);
    }
}

// rho - 1 of the initial state per node: the fourth plane of u_init with with_rho, else 0
// (the first segment references are its segment means).
__global__ __launch_bounds__(256) void k_flow_drho0(Grid g, int64_t nf,
                                                    const uint32_t *__restrict__ coords,
                                                    const float *__restrict__ u_init, int with_rho,
                                                    float *__restrict__ dsnap) {
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nf) return;
    float dr = 0.f;
    if (u_init && with_rho) {
        const uint32_t c = coords[n];
        dr = u_init[3 * g.nvox() + g.lin(c & 1023, (c >> 10) & 1023, c >> 20)];
    }
    dsnap[n] = dr;
}

// The half records from the rank map: occupancy and first node id of each half segment
// (their references are written by k_ref_commit).
__global__ __launch_bounds__(256) void k_flow_halves(int64_t nhalves,
                                                     const RankWord *__restrict__ rank,
                                                     FlowHalf *__restrict__ fh) {
    const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (h >= nhalves) return;
    const RankWord w = rank[h >> 1];
    FlowHalf r;
    r.bits = (h & 1) ? w.hi : w.lo;
    r.base = (h & 1) ? w.base_hi : w.base;
    r.a = 0.f;
    r.b = 0.f;
    fh[h] = r;
}

// The reference of each half segment: the least-squares line a + b (x mod 32) through
// rho - 1 of its fluid nodes (dsnap by node id; a half's ids are consecutive from its
// base, in x order); a constant for a single node, 0 without any.
__global__ __launch_bounds__(256) void k_half_fit(int64_t nhalves, const RankWord *__restrict__ rank,
                                                  const float *__restrict__ dsnap,
                                                  float2 *__restrict__ out) {
    const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (h >= nhalves) return;
    const RankWord w = rank[h >> 1];
    uint32_t bits = (h & 1) ? w.hi : w.lo;
    const uint32_t base = (h & 1) ? w.base_hi : w.base;
    double n = 0, sx = 0, sxx = 0, sy = 0, sxy = 0;
    for (uint32_t k = 0; bits; k++, bits &= bits - 1u) {
        const double xv = (double)(__ffs(bits) - 1), yv = (double)dsnap[base + k];
        n += 1.0;
        sx += xv;
        sxx += xv * xv;
        sy += yv;
        sxy += xv * yv;
    }
    float2 r = make_float2(0.f, 0.f);
    if (n > 0) {
        const double det = n * sxx - sx * sx;
        const double b = det > 0 ? (n * sxy - sx * sy) / det : 0.0;
        r = make_float2((float)((sy - b * sx) / n), (float)b);
    }
    out[h] = r;
}

// The references of the last check become those of the stored state.
__global__ __launch_bounds__(256) void k_ref_commit(int64_t nhalves, const float2 *__restrict__ next,
                                                    FlowHalf *__restrict__ fh) {
    const int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (h >= nhalves) return;
    const float2 r = next[h];
    fh[h].a = r.x;
    fh[h].b = r.y;
}

// The equilibrium (Eq. 3) of rho = 1 + drho and u from u_init (planes u_x, u_y, u_z and,
// with with_rho, rho - 1; rest and rho = 1 without it), stored as offsets from
// w_i (1 + r) with r the node's reference (from its half record fh; null: 0, binary64);
// the snapshot starts at that u.
template <class P>
__global__ __launch_bounds__(256) void k_flow_init(Grid g, int64_t nf, int64_t stride,
                                                   const uint32_t *__restrict__ coords,
                                                   const float *__restrict__ u_init, int with_rho,
                                                   typename P::T *__restrict__ f, float scale,
                                                   const FlowHalf *__restrict__ fh,
                                                   float *__restrict__ usnap) {
    using R = typename P::R;
    LBM_D3Q19_TABLES
    const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (n >= nf) return;
    const uint32_t c = coords[n];
    const int x = c & 1023, y = (c >> 10) & 1023, z = c >> 20;
    R ux = 0, uy = 0, uz = 0, dr = 0;
    if (u_init) {
        const int64_t v = g.lin(x, y, z), nv = g.nvox();
        ux = u_init[v]; uy = u_init[nv + v]; uz = u_init[2 * nv + v];
        if (with_rho) dr = u_init[3 * nv + v];
    }
    R ref = 0;
    if (fh) {
        const FlowHalf h = fh[half_index(g.seg(x, y, z), x)];
        ref = R(half_ref(h.a, h.b, x));
    }
    const R rho = R(1) + dr;
    const R uu15 = R(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int i = 0; i < 19; i++) {
        const R w = i == 0 ? R(1) / R(3) : (i < 7 ? R(1) / R(18) : R(1) / R(36));
        const R eu = EX[i] * ux + EY[i] * uy + EZ[i] * uz;
        // f_eq - w_i (1 + drho), plus w_i (drho - ref)
        const R dev = w * rho * (R(3) * eu + R(4.5) * eu * eu - uu15) + w * (dr - ref);
        f[pop19(i, n)] = to_store<P>(dev, scale);
    }
    usnap[n] = (float)ux; usnap[stride + n] = (float)uy; usnap[2 * stride + n] = (float)uz;
}

template <class P>
__global__ void k_flow_sample(Grid g, int64_t count,
                              const int64_t *__restrict__ vox, const RankWord *__restrict__ rank,
                              const typename P::T *__restrict__ f, float inv_scale,
                              const FlowHalf *__restrict__ fh, double *__restrict__ out,
                              uint8_t *__restrict__ flag) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= count) return;
    const int64_t v = vox[s];
    const int x = (int)(v % g.nx), y = (int)((v / g.nx) % g.ny), z = (int)(v / ((int64_t)g.nx * g.ny));
    const int id = node_at(rank, g, x, y, z);
    flag[s] = id >= 0;
    double ref = 0.0;
    if (fh && id >= 0) {
        const FlowHalf h = fh[half_index(g.seg(x, y, z), x)];
        ref = (double)half_ref(h.a, h.b, x);
    }
    for (int i = 0; i < 19; i++) {
        double v = id >= 0 ? (double)from_store<P>(f[pop19(i, id)], inv_scale) : 0.0;
        if (id >= 0)  // offsets are taken from w_i (1 + r) at the node
            v += (i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0)) * ref;
        out[s * 19 + i] = v;
    }
}

// Kernel variant: explicit bits, or chosen from the working set: when the two population
// arrays and the coordinates exceed the 256 MB Infinity Cache the sweep streams from HBM
// (plain workgroup order, non-temporal stores), otherwise it keeps the state in the
// cache (XCD-contiguous order, ordinary stores).
struct Variant19 {
    bool remap, nt;
    bool wide;  // 64-bit population offsets
};

static Variant19 pick_variant(int32_t v, int64_t stride, int32_t storage) {
    Variant19 m;
    m.wide = (v & LBM_VARIANT_OFF64) || 19 * stride > (int64_t)UINT32_MAX;
    if (v & LBM_VARIANT_EXPLICIT) {
        m.remap = v & LBM_VARIANT_REMAP;
        m.nt = v & LBM_VARIANT_NTSTORE;
        return m;
    }
    const bool stream = (2.0 * 19 * pop_bytes(storage) + 4.0) * (double)stride > kCacheBytes;
    m.remap = !stream;
    m.nt = stream;
    return m;
}

template <class P, bool CHECK, int COLL, class Off>
static void launch19o(const Sweep19 &a, const Variant19 &m, hipStream_t s) {
    const unsigned grid = (unsigned)a.launched;
    if constexpr (!std::is_same<P, StoreF16>::value) {
        if (a.ghost) {  // pressure boundaries
            if (m.nt) k_sweep19<P, CHECK, true, COLL, true, Off><<<grid, 256, 0, s>>>(a);
            else k_sweep19<P, CHECK, false, COLL, true, Off><<<grid, 256, 0, s>>>(a);
            return;
        }
    }
    if (m.nt) k_sweep19<P, CHECK, true, COLL, false, Off><<<grid, 256, 0, s>>>(a);
    else k_sweep19<P, CHECK, false, COLL, false, Off><<<grid, 256, 0, s>>>(a);
}

template <class P, bool CHECK, int COLL>
static void launch19p(const Sweep19 &a, const Variant19 &m, hipStream_t s) {
    if (m.wide || 19 * a.stride > (int64_t)UINT32_MAX) launch19o<P, CHECK, COLL, int64_t>(a, m, s);
    else launch19o<P, CHECK, COLL, uint32_t>(a, m, s);
}

template <bool CHECK, int COLL>
static void launch19c(const Sweep19 &a, const Variant19 &m, int32_t storage, hipStream_t s) {
    if (storage == LBM_STORE_FP16) launch19p<StoreF16, CHECK, COLL>(a, m, s);
    else if (storage == LBM_STORE_FP64) launch19p<StoreF64, CHECK, COLL>(a, m, s);
    else launch19p<StoreF32, CHECK, COLL>(a, m, s);
}

template <bool CHECK>
static void launch19(const Sweep19 &a, const Variant19 &m, int32_t storage, int32_t collision,
                     hipStream_t s) {
    if (collision == LBM_COLLIDE_MRT) launch19c<CHECK, LBM_COLLIDE_MRT>(a, m, storage, s);
    else if (collision == LBM_COLLIDE_TRT) launch19c<CHECK, LBM_COLLIDE_TRT>(a, m, storage, s);
    else launch19c<CHECK, LBM_COLLIDE_BGK>(a, m, storage, s);
}

// `steps` sweeps from buffer cur; the last one checks when check_last.  When the last check
// left new references (h.sref_pending), the first sweep moves the state to them, whichever
// entry point runs it, so that a solve split into steps and resumes goes through the same
// arithmetic as one run.
static lbm_status launch_sweeps(const FlowWs &w, const Grid &g, int64_t nf, FlowHeader &h,
                                const Variant19 &m, int &cur, int64_t steps, bool check_last,
                                float *u_out, int with_rho, hipStream_t s) {
    Sweep19 a;
    a.g = g;
    a.nf = nf;
    a.stride = w.stride;
    a.chunk = m.remap ? (blocks_for(nf) + kXcd - 1) / kXcd : 0;
    a.launched = a.chunk ? xcd_launch(blocks_for(nf), a.chunk) : blocks_for(nf);
    a.coords = w.coords;
    a.rank = w.rank;
    a.omega = (float)(1.0 / h.tau);
    a.fpre = (float)(1.0 - 0.5 / h.tau);
    a.Fx = (float)h.force[0];
    a.Fy = (float)h.force[1];
    a.Fz = (float)h.force[2];
    a.omega_d = 1.0 / h.tau;
    a.fpre_d = 1.0 - 0.5 / h.tau;
    a.sq_d = 8.0 * (2.0 * h.tau - 1.0) / (8.0 * h.tau - 1.0);  // Eq. 7
    a.sq = (float)a.sq_d;
    for (int k = 0; k < 3; k++) a.Fd[k] = h.force[k];
    a.scale = (float)h.scale;
    a.inv_scale = (float)(1.0 / h.scale);
    a.usnap = w.usnap;
    a.u_out = u_out;
    a.partials = w.partials;
    a.update_snap = 1;
    a.with_rho = with_rho;
    a.dsnap = w.dsnap;
    const bool open = h.boundary == LBM_BOUNDARY_PRESSURE;
    a.ghost = open ? w.ghost : nullptr;
    const unsigned gblocks = (unsigned)((2 * (int64_t)g.ny * g.nz + 255) / 256);
    for (int64_t t = 0; t < steps; t++) {
        a.src = w.f[cur];
        a.dst = w.f[cur ^ 1];
        a.reframe = 0;
        a.fh = h.sref ? w.fh : nullptr;
        a.href_next = w.href_next;
        const bool reframe = h.sref && h.sref_pending;
        if (reframe) {
            a.reframe = 1;
            h.sref_pending = 0;
        }
        if (open) {  // the ghost planes of this step, from the state it reads
            if (h.storage == LBM_STORE_FP64)
                k_ghost19<StoreF64><<<gblocks, 256, 0, s>>>(
                    g, w.rank, static_cast<const double *>(a.src), nullptr, 1.f, 1.f,
                    h.force[0], h.force[1], h.force[2], h.rho_in - 1.0, h.rho_out - 1.0,
                    static_cast<double *>(w.ghost));
            else
                k_ghost19<StoreF32><<<gblocks, 256, 0, s>>>(
                    g, w.rank, static_cast<const float *>(a.src), a.fh, 1.f, 1.f,
                    (float)h.force[0], (float)h.force[1], (float)h.force[2],
                    (float)(h.rho_in - 1.0), (float)(h.rho_out - 1.0),
                    static_cast<float *>(w.ghost));
            LBM_CHECK_LAUNCH();
        }
        if (check_last && t == steps - 1)
            launch19<true>(a, m, h.storage, h.collision, s);
        else
            launch19<false>(a, m, h.storage, h.collision, s);
        LBM_CHECK_LAUNCH();
        cur ^= 1;
        if (reframe) {  // the stored state is now relative to the new references
            const int64_t nh = 2 * g.nsegs();
            k_ref_commit<<<(unsigned)((nh + 255) / 256), 256, 0, s>>>(nh, w.href_next, w.fh);
            LBM_CHECK_LAUNCH();
        }
    }
    return LBM_OK;
}

// After a check interval: the segment means of the checked rho - 1 become the references
// the next interval moves to.
static lbm_status flow_next_refs(const FlowWs &w, const Grid &g, FlowHeader &h, hipStream_t s) {
    if (!h.sref) return LBM_OK;
    const int64_t nh = 2 * g.nsegs();
    k_half_fit<<<(unsigned)((nh + 255) / 256), 256, 0, s>>>(nh, w.rank, w.dsnap, w.href_next);
    LBM_CHECK_LAUNCH();
    h.sref_pending = 1;
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
size_t flow_ws_bytes_n(const int32_t n[3], int64_t nf, int32_t storage) {
    Grid g = make_grid(n);
    return flow_ws_bytes(g, nf < 0 ? g.nvox() : nf, storage);
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
    LBM_REQUIRE(std::isfinite(p->force[0]) && std::isfinite(p->force[1]) &&
                    std::isfinite(p->force[2]) && p->voxel_nm > 0 && std::isfinite(p->voxel_nm),
                LBM_E_INVAL, "the force must be finite and the voxel size positive and finite");
    LBM_REQUIRE(p->check_every >= 1, LBM_E_INVAL, "check_every must be >= 1");
    LBM_REQUIRE(p->fixed_steps > 0 || p->max_steps > 0, LBM_E_INVAL, "no step limit given");
    LBM_REQUIRE(p->steady_tol >= 0.0 && std::isfinite(p->steady_tol), LBM_E_INVAL,
                "steady_tol must be finite and >= 0");
    LBM_REQUIRE(p->storage == LBM_STORE_FP32 || p->storage == LBM_STORE_FP16 ||
                    p->storage == LBM_STORE_FP64,
                LBM_E_INVAL, "unknown storage %d", p->storage);
    LBM_REQUIRE((p->variant & ~kSolveVariantBits) == 0, LBM_E_INVAL, "unknown variant bits 0x%x",
                p->variant);
    LBM_REQUIRE(p->with_rho == 0 || p->with_rho == 1, LBM_E_INVAL, "with_rho must be 0 or 1");
    LBM_REQUIRE(p->collision == LBM_COLLIDE_BGK || p->collision == LBM_COLLIDE_MRT ||
                    p->collision == LBM_COLLIDE_TRT,
                LBM_E_INVAL,
                "unknown collision %d", p->collision);
    LBM_REQUIRE(p->boundary == LBM_BOUNDARY_PERIODIC || p->boundary == LBM_BOUNDARY_PRESSURE,
                LBM_E_INVAL, "unknown boundary %d", p->boundary);
    if (p->boundary == LBM_BOUNDARY_PRESSURE) {
        LBM_REQUIRE(p->storage != LBM_STORE_FP16, LBM_E_INVAL,
                    "pressure boundaries take binary32 or binary64 storage");
        LBM_REQUIRE(p->rho_in > 0 && p->rho_out > 0 && std::isfinite(p->rho_in) &&
                        std::isfinite(p->rho_out),
                    LBM_E_INVAL, "boundary densities must be positive");
        LBM_REQUIRE(p->force[0] + (p->rho_in - p->rho_out) / (3.0 * (n[0] + 1)) != 0.0,
                    LBM_E_INVAL, "no driving along x (F_x and rho_in - rho_out)");
    }
    st = check_device();
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g = make_grid(n);

    // the grid-sized part of the workspace comes first: count the fluid nodes there
    FlowWs w0 = carve_flow(workspace, g, 1, p->storage);
    LBM_REQUIRE(ws_bytes >= (size_t)((char *)w0.coords - (char *)workspace), LBM_E_NOMEM,
                "workspace of %zu bytes is below the grid part", ws_bytes);
    int64_t nf = 0;
    FlowHeader h;
    int64_t t0 = 0;
    int cur = 0;
    if (p->resume) {
        // checked against a plain count of the mask before the rank map is rebuilt, so
        // that a refused resume leaves the stored state usable
        LBM_TRY_HIP(hipMemcpyAsync(&h, w0.hdr, sizeof(h), hipMemcpyDeviceToHost, s));
        st = count_nonzero(g, fluid, w0.counter, &nf, s);
        if (st != LBM_OK) return st;
        LBM_REQUIRE(h.magic == kFlowMagic && h.nx == n[0] && h.ny == n[1] && h.nz == n[2] &&
                        h.n_fluid == nf && h.storage == p->storage &&
                        h.collision == p->collision && h.boundary == p->boundary,
                    LBM_E_INVAL,
                    "resume: the workspace holds no state for this geometry and storage");
        // the state continues only under the parameters it was computed with
        const bool press = p->boundary == LBM_BOUNDARY_PRESSURE;
        LBM_REQUIRE(h.tau == p->tau && h.force[0] == p->force[0] && h.force[1] == p->force[1] &&
                        h.force[2] == p->force[2] &&
                        (!press || (h.rho_in == p->rho_in && h.rho_out == p->rho_out)),
                    LBM_E_INVAL, "resume: tau, force or boundary densities differ from the state's");
        t0 = h.steps_done;
        cur = h.cur;
    }
    st = layout_count(g, fluid, w0.rank, w0.total, &nf, s);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(nf > 0, LBM_E_INVAL, "the fluid mask is empty");
    FlowWs w = carve_flow(workspace, g, nf, p->storage);
    LBM_REQUIRE(ws_bytes >= w.bytes, LBM_E_NOMEM,
                "workspace of %zu bytes; %zu needed for %lld fluid nodes", ws_bytes, w.bytes,
                (long long)nf);
    st = layout_fill(g, w.rank, w.coords, s);
    if (st != LBM_OK) return st;
    h.magic = kFlowMagic;
    h.nx = n[0]; h.ny = n[1]; h.nz = n[2];
    h.n_fluid = nf;
    h.tau = p->tau;
    h.variant = p->variant;
    h.storage = p->storage;
    h.collision = p->collision;
    h.boundary = p->boundary;
    h.rho_in = p->boundary == LBM_BOUNDARY_PRESSURE ? p->rho_in : 1.0;
    h.rho_out = p->boundary == LBM_BOUNDARY_PRESSURE ? p->rho_out : 1.0;
    h.sref = p->storage != LBM_STORE_FP64;
    if (!p->resume) h.sref_pending = 0;
    for (int a = 0; a < 3; a++) h.force[a] = p->force[a];
    if (!p->resume) {
        // binary16: a power of two S with S max|F| in [1, 2) (1 without a force)
        const double fmax = std::max(std::fabs(p->force[0]),
                                     std::max(std::fabs(p->force[1]), std::fabs(p->force[2])));
        h.scale = p->storage == LBM_STORE_FP16 && fmax > 0 ? std::ldexp(1.0, -std::ilogb(fmax)) : 1.0;
    }
    const Variant19 mode = pick_variant(p->variant, w.stride, h.storage);
    if (!p->resume) {
        const unsigned nb = (unsigned)blocks_for(nf);
        const float sc = (float)h.scale;
        const int wr = p->with_rho;
        if (h.sref) {
            // the half records, with the first references fitted to the initial density
            const int64_t nh = 2 * g.nsegs();
            const unsigned nhb = (unsigned)((nh + 255) / 256);
            k_flow_halves<<<nhb, 256, 0, s>>>(nh, w.rank, w.fh);
            LBM_CHECK_LAUNCH();
            k_flow_drho0<<<nb, 256, 0, s>>>(g, nf, w.coords, u_init, wr, w.dsnap);
            LBM_CHECK_LAUNCH();
            k_half_fit<<<nhb, 256, 0, s>>>(nh, w.rank, w.dsnap, w.href_next);
            LBM_CHECK_LAUNCH();
            k_ref_commit<<<nhb, 256, 0, s>>>(nh, w.href_next, w.fh);
            LBM_CHECK_LAUNCH();
        }
        if (h.storage == LBM_STORE_FP16)
            k_flow_init<StoreF16><<<nb, 256, 0, s>>>(g, nf, w.stride, w.coords, u_init, wr,
                                                     static_cast<_Float16 *>(w.f[0]), sc,
                                                     w.fh, w.usnap);
        else if (h.storage == LBM_STORE_FP64)
            k_flow_init<StoreF64><<<nb, 256, 0, s>>>(g, nf, w.stride, w.coords, u_init, wr,
                                                     static_cast<double *>(w.f[0]), sc,
                                                     nullptr, w.usnap);
        else
            k_flow_init<StoreF32><<<nb, 256, 0, s>>>(g, nf, w.stride, w.coords, u_init, wr,
                                                     static_cast<float *>(w.f[0]), sc,
                                                     w.fh, w.usnap);
        LBM_CHECK_LAUNCH();
    }
    if (u_out)
        LBM_TRY_HIP(hipMemsetAsync(u_out, 0, sizeof(float) * (p->with_rho ? 4 : 3) * g.nvox(), s));

    struct Events {  // released on every return
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e1) (void)hipEventDestroy(e1);
            if (e0) (void)hipEventDestroy(e0);
        }
    } ev;
    LBM_TRY_HIP(hipEventCreate(&ev.e0));
    LBM_TRY_HIP(hipEventCreate(&ev.e1));
    const hipEvent_t e0 = ev.e0, e1 = ev.e1;
    const int64_t limit = p->fixed_steps > 0 ? p->fixed_steps : p->max_steps;
    const int nc = p->check_every;
    double sums[kFlowSums] = {0, 0, 0, 0, 0, 0};
    double resid = INFINITY, sweep_ms = 0.0;
    SteadyEst est;
    bool converged = false, diverged = false, stalled = false;
    int64_t t = 0;
    lbm_status out = LBM_OK;
    while (t < limit) {
        // run to the next check (a multiple of n_c counted from the first step) or the limit
        const int64_t abs_t = t0 + t;
        int64_t chunk = nc - (abs_t % nc);
        if (chunk > limit - t) chunk = limit - t;
        LBM_TRY_HIP(hipEventRecord(e0, s));
        out = launch_sweeps(w, g, nf, h, mode, cur, chunk, true, u_out, p->with_rho, s);
        if (out != LBM_OK) break;
        LBM_TRY_HIP(hipEventRecord(e1, s));
        out = flow_next_refs(w, g, h, s);
        if (out != LBM_OK) break;
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
            est.push(resid);
            // binary16: a check interval with no change at all is a fixed point of the
            // rounded iteration (every per-step increment below half an ulp), not steady
            // state; the solve stops and says so
            if (p->fixed_steps <= 0 && h.storage == LBM_STORE_FP16 && sums[0] == 0.0 &&
                sums[1] > 0.0) {
                stalled = true;
                break;
            }
            if (p->fixed_steps <= 0 && resid < p->tol &&
                (p->steady_tol <= 0.0 || est.dist(nc) <= p->steady_tol)) {
                converged = true;
                break;
            }
        }
    }
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
    r->steady_dist = est.dist(nc);
    for (int a = 0; a < 3; a++) r->mean_rho_u[a] = sums[2 + a] / nvox;
    r->mass_dev = sums[5];
    // the driving: F_x, plus c_s^2 (rho_in - rho_out) over the nx + 1 spacings between the
    // ghost planes of pressure boundaries
    const double drive = p->force[0] + (h.boundary == LBM_BOUNDARY_PRESSURE
                                            ? (h.rho_in - h.rho_out) / (3.0 * (g.nx + 1))
                                            : 0.0);
    r->k_lattice = nu * r->mean_rho_u[0] / drive;
    const double dx = p->voxel_nm * 1e-9;
    r->k_m2 = r->k_lattice * dx * dx;
    r->k_mD = r->k_m2 / 9.869233e-16;
    r->sweep_ms = sweep_ms;
    const double updates = (double)nf * (double)t;
    r->mlups = sweep_ms > 0 ? updates / (sweep_ms * 1e3) : 0.0;
    r->gbps = sweep_ms > 0 ? updates * flow_bytes_per_update(h.storage) / (sweep_ms * 1e-3) / 1e9 : 0.0;
    if (diverged) {
        set_error("flow solve diverged (NaN/Inf) by step %lld", (long long)(t0 + t));
        return LBM_E_DIVERGED;
    }
    if (p->fixed_steps > 0 || converged) return LBM_OK;
    if (stalled) {
        set_error("binary16 state stalled after %lld steps (no change over a check interval)",
                  (long long)t);
        return LBM_W_NOT_CONVERGED;
    }
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
    w = carve_flow(workspace, g, h.n_fluid, h.storage);
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
    st = launch_sweeps(w, g, h.n_fluid, h, pick_variant(h.variant, w.stride, h.storage), cur, steps, false,
                       nullptr, 0, s);
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
    const unsigned nb = (unsigned)((count + 255) / 256);
    const float inv = (float)(1.0 / h.scale);
    if (h.storage == LBM_STORE_FP16)
        k_flow_sample<StoreF16><<<nb, 256, 0, s>>>(g, count, w.samp_vox, w.rank,
                                                   static_cast<const _Float16 *>(w.f[h.cur]), inv,
                                                   w.fh, w.samp_out, w.samp_flag);
    else if (h.storage == LBM_STORE_FP64)
        k_flow_sample<StoreF64><<<nb, 256, 0, s>>>(g, count, w.samp_vox, w.rank,
                                                   static_cast<const double *>(w.f[h.cur]), inv,
                                                   nullptr, w.samp_out, w.samp_flag);
    else
        k_flow_sample<StoreF32><<<nb, 256, 0, s>>>(g, count, w.samp_vox, w.rank,
                                                   static_cast<const float *>(w.f[h.cur]), inv,
                                                   w.fh, w.samp_out, w.samp_flag);
    LBM_CHECK_LAUNCH();
    LBM_TRY_HIP(hipMemcpyAsync(f_h, w.samp_out, sizeof(double) * 19 * count, hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipMemcpyAsync(fluid_h, w.samp_flag, count, hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return LBM_OK;
}

// ============================================================== batched flow solves
namespace lbm {

struct BatchWs {
    LatDesc *lats;
    BlkDesc19 *descs;
    int32_t *lat_ids, *total;
    double *res;
    RankWord *rank;
    uint32_t *coords;
    float *f[2];
    FlowHalf *fh;       // half records with the references (rank-map order, 2 per segment)
    float2 *href_next;
    float *dsnap;
    float *usnap;
    double *partials;
    int64_t stride, nblk, nrank;
    size_t bytes;
};

static BatchWs carve_batch(void *base, int count, const int32_t *n_h, const int64_t *nf_h) {
    BatchWs w;
    w.nblk = 0;
    w.nrank = 0;
    for (int l = 0; l < count; l++) {
        const Grid g = make_grid(n_h + 3 * l);
        w.nblk += blocks_for(nf_h[l] < 1 ? 1 : nf_h[l]);
        w.nrank += g.nsegs();
    }
    w.stride = w.nblk * 256;
    Carver c(base);
    w.lats = c.take<LatDesc>(count);
    w.descs = c.take<BlkDesc19>(w.nblk);
    w.lat_ids = c.take<int32_t>(count);
    w.total = c.take<int32_t>(count);
    w.res = c.take<double>((size_t)count * kFlowSums);
    w.rank = c.take<RankWord>(w.nrank);
    w.fh = c.take<FlowHalf>(2 * (size_t)w.nrank);
    w.href_next = c.take<float2>(2 * (size_t)w.nrank);
    w.coords = c.take<uint32_t>(w.stride);
    w.f[0] = c.take<float>((size_t)19 * w.stride);
    w.f[1] = c.take<float>((size_t)19 * w.stride);
    w.dsnap = c.take<float>(w.stride);
    w.usnap = c.take<float>((size_t)3 * w.stride);
    w.partials = c.take<double>((size_t)w.nblk * kFlowSums);
    w.bytes = c.off;
    return w;
}

template <bool CHECK>
static void launch19b(const Sweep19 &a, const Variant19 &m, int32_t collision,
                      const BlkDesc19 *descs, hipStream_t s) {
    const unsigned grid = (unsigned)a.launched;
    if (collision == LBM_COLLIDE_MRT) {
        if (m.nt) k_sweep19b<CHECK, true, LBM_COLLIDE_MRT><<<grid, 256, 0, s>>>(a, descs);
        else k_sweep19b<CHECK, false, LBM_COLLIDE_MRT><<<grid, 256, 0, s>>>(a, descs);
    } else if (collision == LBM_COLLIDE_TRT) {
        if (m.nt) k_sweep19b<CHECK, true, LBM_COLLIDE_TRT><<<grid, 256, 0, s>>>(a, descs);
        else k_sweep19b<CHECK, false, LBM_COLLIDE_TRT><<<grid, 256, 0, s>>>(a, descs);
    } else {
        if (m.nt) k_sweep19b<CHECK, true, LBM_COLLIDE_BGK><<<grid, 256, 0, s>>>(a, descs);
        else k_sweep19b<CHECK, false, LBM_COLLIDE_BGK><<<grid, 256, 0, s>>>(a, descs);
    }
}

// A lattice's place in the batch, for the per-lattice passes on the host side.
struct LatRef {
    int64_t nsegs, rk0, n0;
};

// `steps` sweeps of the lattices of group g from buffer cur; with `pending` the first one
// moves the state to the references of the last check; the last one checks, then the
// group's per-lattice sums go to w.res and each lattice's references are fitted to its
// checked rho - 1 (as in the single solve).
static lbm_status batch_steps(const BatchWs &w, Sweep19 a, const Variant19 &m, int32_t collision,
                              const BatchGroup &g, int cur, bool pending, int64_t steps,
                              bool check_last, const std::vector<LatRef> &lr,
                              const std::vector<int32_t> &lat_ids_h, hipStream_t s) {
    const int64_t n_live = g.n_blk;
    a.launched_live = n_live;
    a.chunk = m.remap ? (n_live + kXcd - 1) / kXcd : 0;
    a.launched = a.chunk ? xcd_launch(n_live, a.chunk) : n_live;
    const BlkDesc19 *descs = w.descs + g.blk_off;
    for (int64_t t = 0; t < steps; t++) {
        a.src = w.f[cur];
        a.dst = w.f[cur ^ 1];
        a.fh = w.fh;
        a.href_next = w.href_next;
        a.reframe = pending && t == 0;
        if (check_last && t == steps - 1) launch19b<true>(a, m, collision, descs, s);
        else launch19b<false>(a, m, collision, descs, s);
        LBM_CHECK_LAUNCH();
        cur ^= 1;
        if (a.reframe)  // the group's lattices are now relative to their new references
            for (int32_t k = 0; k < g.n_lat; k++) {
                const LatRef &L = lr[lat_ids_h[g.lat_off + k]];
                const int64_t nh = 2 * L.nsegs;
                k_ref_commit<<<(unsigned)((nh + 255) / 256), 256, 0, s>>>(
                    nh, w.href_next + 2 * L.rk0, w.fh + 2 * L.rk0);
                LBM_CHECK_LAUNCH();
            }
    }
    if (check_last) {
        k_lat_reduce<kFlowSums><<<(unsigned)g.n_lat, 256, 0, s>>>(w.partials, w.lats,
                                                                  w.lat_ids + g.lat_off, w.res);
        LBM_CHECK_LAUNCH();
        if (steps > 0)
            for (int32_t k = 0; k < g.n_lat; k++) {
                const LatRef &L = lr[lat_ids_h[g.lat_off + k]];
                const int64_t nh = 2 * L.nsegs;
                k_half_fit<<<(unsigned)((nh + 255) / 256), 256, 0, s>>>(
                    nh, w.rank + L.rk0, w.dsnap + L.n0, w.href_next + 2 * L.rk0);
                LBM_CHECK_LAUNCH();
            }
    }
    return LBM_OK;
}

// Binary32 flow state per fluid node: two population buffers, coordinate, snapshots.
constexpr double kBatchFlowNodeBytes = 2 * 19 * 4 + 4 + 12 + 4;

}  // namespace lbm

extern "C" size_t lbm_flow_batch_workspace(int32_t count, const int32_t *n_h, const int64_t *nf_h) {
    if (count < 1 || !n_h || !nf_h) return 0;
    for (int l = 0; l < count; l++)
        if (n_h[3 * l] < 1 || n_h[3 * l + 1] < 1 || n_h[3 * l + 2] < 1 || n_h[3 * l] > kMaxEdge ||
            n_h[3 * l + 1] > kMaxEdge || n_h[3 * l + 2] > kMaxEdge || nf_h[l] < 0)
            return 0;
    return carve_batch(nullptr, count, n_h, nf_h).bytes;
}

extern "C" lbm_status lbm_flow_solve_batch(int32_t count, const int32_t *n_h,
                                           const uint8_t *const *fluid, const int64_t *nf_h,
                                           const lbm_flow_params *p, lbm_batch_sched *sched,
                                           lbm_flow_result *r_h, float *const *u_out,
                                           void *workspace, size_t ws_bytes, void *stream) {
    LBM_REQUIRE(count >= 1 && n_h && fluid && nf_h && p && r_h && workspace, LBM_E_INVAL,
                "lbm_flow_solve_batch: null argument or empty batch");
    for (int l = 0; l < count; l++) {
        lbm_status st = validate_n(n_h + 3 * l);
        if (st != LBM_OK) return st;
        LBM_REQUIRE(fluid[l] && nf_h[l] >= 1, LBM_E_INVAL, "lattice %d: no fluid mask or node", l);
    }
    LBM_REQUIRE(p->tau > 0.5 && std::isfinite(p->tau), LBM_E_INVAL, "tau must exceed 1/2");
    LBM_REQUIRE(std::isfinite(p->force[0]) && std::isfinite(p->force[1]) &&
                    std::isfinite(p->force[2]) && p->voxel_nm > 0 && std::isfinite(p->voxel_nm),
                LBM_E_INVAL, "the force must be finite and the voxel size positive and finite");
    LBM_REQUIRE(p->check_every >= 1, LBM_E_INVAL, "check_every must be >= 1");
    LBM_REQUIRE(p->fixed_steps > 0 || p->max_steps > 0, LBM_E_INVAL, "no step limit given");
    LBM_REQUIRE(p->steady_tol >= 0.0 && std::isfinite(p->steady_tol), LBM_E_INVAL,
                "steady_tol must be finite and >= 0");
    LBM_REQUIRE(p->storage == LBM_STORE_FP32 && !p->resume && !p->with_rho, LBM_E_INVAL,
                "batched solves take binary32 storage, no resume, no density fields");
    LBM_REQUIRE(p->collision == LBM_COLLIDE_BGK || p->collision == LBM_COLLIDE_MRT ||
                    p->collision == LBM_COLLIDE_TRT,
                LBM_E_INVAL,
                "unknown collision %d", p->collision);
    LBM_REQUIRE((p->variant & ~(kVariantBits | LBM_VARIANT_NOGRAPH)) == 0, LBM_E_INVAL,
                "unknown variant bits 0x%x", p->variant);
    LBM_REQUIRE(p->force[0] != 0.0, LBM_E_INVAL, "batched solves report k along x: F_x must be nonzero");
    LBM_REQUIRE(p->boundary == LBM_BOUNDARY_PERIODIC, LBM_E_INVAL,
                "batched solves are periodic in x (no pressure boundaries)");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    const BatchWs w = carve_batch(workspace, count, n_h, nf_h);
    for (int l = 0; l < count; l++)
        LBM_REQUIRE(19 * blocks_for(nf_h[l]) * 256 <= (int64_t)UINT32_MAX, LBM_E_INVAL,
                    "lattice %d: %lld nodes exceed the 32-bit population offsets", l,
                    (long long)nf_h[l]);
    LBM_REQUIRE(ws_bytes >= w.bytes, LBM_E_NOMEM, "workspace of %zu bytes; %zu needed", ws_bytes,
                w.bytes);
    hipStream_t caller = static_cast<hipStream_t>(stream);
    BatchRes R;
    st = R.open(caller);
    if (st != LBM_OK) return st;
    hipStream_t s = R.s;

    // layout, lattice tables, initial state
    std::vector<LatDesc> lats(count);
    std::vector<BatchLat> bl(count);
    std::vector<BlkDesc19> blk(w.nblk);  // the record of each physical block
    std::vector<double> nvox(count);
    std::vector<LatRef> lref(count);
    int64_t n0 = 0, rk0 = 0, b0 = 0;
    for (int l = 0; l < count; l++) {
        const Grid g = make_grid(n_h + 3 * l);
        int64_t nf = 0;
        st = layout_count(g, fluid[l], w.rank + rk0, w.total + l, &nf, s);
        if (st != LBM_OK) return st;
        LBM_REQUIRE(nf == nf_h[l], LBM_E_INVAL, "lattice %d has %lld fluid nodes, not %lld", l,
                    (long long)nf, (long long)nf_h[l]);
        st = layout_fill(g, w.rank + rk0, w.coords + n0, s);
        if (st != LBM_OK) return st;
        const int64_t b1 = b0 + blocks_for(nf), span = (b1 - b0) * 256;
        // from rest: the half records with every reference 0
        k_flow_halves<<<(unsigned)((2 * g.nsegs() + 255) / 256), 256, 0, s>>>(
            2 * g.nsegs(), w.rank + rk0, w.fh + 2 * rk0);
        LBM_CHECK_LAUNCH();
        k_flow_init<StoreF32><<<(unsigned)blocks_for(nf), 256, 0, s>>>(
            g, nf, span, w.coords + n0, nullptr, 0, w.f[0] + 19 * n0, 1.f, w.fh + 2 * rk0,
            w.usnap + 3 * n0);
        LBM_CHECK_LAUNCH();
        lref[l] = LatRef{g.nsegs(), rk0, n0};
        float *uo = u_out ? u_out[l] : nullptr;
        if (uo) LBM_TRY_HIP(hipMemsetAsync(uo, 0, sizeof(float) * 3 * g.nvox(), s));
        lats[l] = LatDesc{b0, b1};
        bl[l] = BatchLat{b0, b1, nf, g.nx};
        nvox[l] = (double)g.nvox();
        for (int64_t b = b0; b < b1; b++)
            blk[b] = BlkDesc19{g, (int32_t)b, (int32_t)b0, (int32_t)b1, (int32_t)nf, rk0, uo, 0};
        n0 = b1 * 256;
        rk0 += g.nsegs();
        b0 = b1;
    }
    LBM_TRY_HIP(hipMemcpyAsync(w.lats, lats.data(), sizeof(LatDesc) * count, hipMemcpyHostToDevice, s));

    // the active lattices in groups; each group's block records in launch order
    std::vector<int32_t> act(count), blocks_h, lat_ids_h;
    std::vector<BlkDesc19> descs_h;
    for (int l = 0; l < count; l++) act[l] = l;
    std::vector<BatchGroup> groups;
    auto regroup = [&](double budget) -> lbm_status {
        groups = form_groups(act, bl, kBatchFlowNodeBytes, budget, blocks_h, lat_ids_h, nullptr);
        descs_h.resize(blocks_h.size());
        for (size_t k = 0; k < blocks_h.size(); k++) descs_h[k] = blk[blocks_h[k]];
        LBM_TRY_HIP(hipMemcpyAsync(w.lat_ids, lat_ids_h.data(), sizeof(int32_t) * lat_ids_h.size(),
                                   hipMemcpyHostToDevice, s));
        LBM_TRY_HIP(hipMemcpyAsync(w.descs, descs_h.data(), sizeof(BlkDesc19) * descs_h.size(),
                                   hipMemcpyHostToDevice, s));
        LBM_TRY_HIP(hipStreamSynchronize(s));  // the host vectors are reused
        R.reset_graphs(groups.size());
        return LBM_OK;
    };
    const int32_t vbits = p->variant & kVariantBits;
    auto group_mode = [&](const BatchGroup &g) {
        return pick_variant(vbits, (int64_t)g.nodes, LBM_STORE_FP32);
    };
    double live_nodes = 0.0;
    for (int l : act) live_nodes += (double)nf_h[l];

    Sweep19 a{};
    a.stride = w.stride;
    a.coords = w.coords;
    a.rank = w.rank;
    a.omega = (float)(1.0 / p->tau);
    a.fpre = (float)(1.0 - 0.5 / p->tau);
    a.Fx = (float)p->force[0];
    a.Fy = (float)p->force[1];
    a.Fz = (float)p->force[2];
    a.sq = (float)(8.0 * (2.0 * p->tau - 1.0) / (8.0 * p->tau - 1.0));  // Eq. 7
    a.omega_d = 1.0 / p->tau;
    a.fpre_d = 1.0 - 0.5 / p->tau;
    a.scale = 1.f;
    a.inv_scale = 1.f;
    a.usnap = w.usnap;
    a.dsnap = w.dsnap;
    a.partials = w.partials;
    a.update_snap = 1;

    const int64_t limit = p->fixed_steps > 0 ? p->fixed_steps : p->max_steps;
    const int nc = p->check_every;
    const bool use_graph = !(p->variant & LBM_VARIANT_NOGRAPH);
    int cur = 0;
    bool pending = false;  // references of a check not yet entered (none before the first)
    int64_t t = 0;
    double sweep_ms = 0.0, updates = 0.0, tune_ms = 0.0;

    // schedule: a given group budget, or the autotuner's: the first check intervals run
    // one candidate budget each (all give the same state), timed per node update, and the
    // fastest runs the rest
    const double cand[kBatchBudgets] = LBM_BATCH_BUDGETS;
    const bool tuning = !sched || sched->group_bytes == 0;
    int tune_k = tuning ? 0 : kBatchBudgets;
    double budget = tuning ? cand[0] : (double)sched->group_bytes, best_rate = INFINITY;
    st = regroup(budget);
    if (st != LBM_OK) return st;
    int32_t groups_run = tuning ? -1 : (int32_t)groups.size();

    std::vector<double> res((size_t)count * kFlowSums, 0.0), sums_l((size_t)count * kFlowSums, 0.0);
    std::vector<int64_t> steps_l(count, 0);
    std::vector<double> resid_l(count, INFINITY);
    std::vector<SteadyEst> est_l(count);
    std::vector<int> conv_l(count, 0);
    bool diverged = false;
    while (t < limit && !act.empty()) {
        const int64_t chunk = std::min<int64_t>(nc - (t % nc), limit - t);
        if (use_graph && chunk == nc && pending) {
            // capture what is missing first, so that the timed region holds kernels only;
            // one graph per group and buffer at the start of the interval
            const int key = cur;
            for (size_t gi = 0; gi < groups.size(); gi++) {
                hipGraphExec_t &ex = R.exec[gi * BatchRes::kKeys + key];
                if (ex) continue;
                LBM_TRY_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                st = batch_steps(w, a, group_mode(groups[gi]), p->collision, groups[gi], cur,
                                 true, chunk, true, lref, lat_ids_h, s);
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
        } else {
            LBM_TRY_HIP(hipEventRecord(R.e0, s));
            for (const BatchGroup &g : groups) {
                st = batch_steps(w, a, group_mode(g), p->collision, g, cur, pending, chunk,
                                 true, lref, lat_ids_h, s);
                if (st != LBM_OK) return st;
            }
        }
        LBM_TRY_HIP(hipEventRecord(R.e1, s));
        LBM_TRY_HIP(hipMemcpyAsync(res.data(), w.res, sizeof(double) * count * kFlowSums,
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
            // the next candidate, or the winner (unless it is the one just run)
            ++tune_k;
            regroup_now = tune_k < kBatchBudgets || budget != cand[kBatchBudgets - 1];
        }
        cur ^= (int)(chunk & 1);
        pending = true;  // the interval's check formed the next references
        t += chunk;
        std::vector<int32_t> keep;
        for (int l : act) {
            const double *sm = res.data() + (size_t)l * kFlowSums;
            std::copy(sm, sm + kFlowSums, sums_l.begin() + (size_t)l * kFlowSums);
            steps_l[l] = t;
            if (!std::isfinite(sm[0]) || !std::isfinite(sm[1]) || !std::isfinite(sm[2])) {
                diverged = true;
                continue;
            }
            bool done = false;
            if (t % nc == 0) {
                resid_l[l] = std::sqrt(sm[0]) / ((double)nc * std::sqrt(sm[1]));
                est_l[l].push(resid_l[l]);
                if (p->fixed_steps <= 0 && resid_l[l] < p->tol &&
                    (p->steady_tol <= 0.0 || est_l[l].dist(nc) <= p->steady_tol)) {
                    conv_l[l] = 1;
                    done = true;
                }
            }
            if (!done) keep.push_back(l);
        }
        if (diverged) break;
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
    st = R.close(caller);
    if (st != LBM_OK) return st;

    const double nu = (p->tau - 0.5) / 3.0;
    for (int l = 0; l < count; l++) {
        lbm_flow_result &r = r_h[l];
        std::memset(&r, 0, sizeof(r));
        const double *sm = sums_l.data() + (size_t)l * kFlowSums;
        r.steps = steps_l[l];
        r.n_fluid = nf_h[l];
        r.converged = conv_l[l];
        r.residual = resid_l[l];
        r.steady_dist = est_l[l].dist(nc);
        for (int k = 0; k < 3; k++) r.mean_rho_u[k] = sm[2 + k] / nvox[l];
        r.mass_dev = sm[5];
        r.k_lattice = nu * r.mean_rho_u[0] / p->force[0];
        const double dx = p->voxel_nm * 1e-9;
        r.k_m2 = r.k_lattice * dx * dx;
        r.k_mD = r.k_m2 / 9.869233e-16;
        r.sweep_ms = sweep_ms;  // of the whole batch
        r.mlups = sweep_ms > 0 ? updates / (sweep_ms * 1e3) : 0.0;
        r.gbps = sweep_ms > 0 ? updates * 152.0 / (sweep_ms * 1e-3) / 1e9 : 0.0;
    }
    if (diverged) {
        set_error("batched flow solve diverged (NaN/Inf) by step %lld", (long long)t);
        return LBM_E_DIVERGED;
    }
    for (int l = 0; l < count; l++)
        if (!conv_l[l] && p->fixed_steps <= 0) {
            set_error("lattice %d not converged after %lld steps", l, (long long)steps_l[l]);
            return LBM_W_NOT_CONVERGED;
        }
    return LBM_OK;
}
