// Internal declarations shared by the translation units of liblbm.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/lbm.h"

namespace lbm {

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);

#define LBM_TRY_HIP(call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::lbm::set_error("%s:%d: %s: %s", __FILE__, __LINE__, #call,                   \
                             hipGetErrorString(e_));                                       \
            return LBM_E_DEVICE;                                                           \
        }                                                                                  \
    } while (0)

#define LBM_CHECK_LAUNCH() LBM_TRY_HIP(hipGetLastError())

#define LBM_REQUIRE(cond, code, ...)                                                       \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            ::lbm::set_error(__VA_ARGS__);                                                 \
            return code;                                                                   \
        }                                                                                  \
    } while (0)

// Fails with LBM_E_DEVICE unless the current device is a gfx950.
lbm_status check_device();

// ---------------------------------------------------------------- workspace carving
// Hands out 256-byte aligned pieces of a caller-owned buffer; base may be null to
// measure the size.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        size_t a = (off + 255) & ~size_t(255);
        off = a + count * sizeof(T);
        return base ? reinterpret_cast<T *>(base + a) : nullptr;
    }
};

// ---------------------------------------------------------------- grid geometry
// Rows of the box (all x at one y, z) are cut into segments of 64 voxels along x;
// segment (x / 64, y, z) has index seg(x, y, z).  The fluid-node list holds each segment's
// nodes contiguously, in x order.  Segments follow each other in column order: the y-z
// cross-section is tiled by columns of kCol x kCol rows (columns z-major, then y; rows
// inside a column z-major), and each row's segments run in x order.  A wave of 64
// consecutive nodes is then a run along one row, and each of its pulls reads one short
// run of the list (the same run shifted to the neighbouring row or plane of the column),
// which keeps the cache lines a wave touches per load close to the minimum.
constexpr int kSegLog = 6;
constexpr int kSeg = 1 << kSegLog;
constexpr int kCol = 16;
constexpr int kMaxEdge = 1024;  // coordinates packed in 10 bits each

struct Grid {
    int nx, ny, nz;
    int nseg;      // segments per row
    int ncy, ncz;  // columns along y and z
    __host__ __device__ int64_t nvox() const { return (int64_t)nx * ny * nz; }
    __host__ __device__ int64_t nsegs() const { return (int64_t)nseg * ny * nz; }
    __host__ __device__ int64_t lin(int x, int y, int z) const {
        return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
    }
    __host__ __device__ int64_t seg(int x, int y, int z) const {
        return ((int64_t)z * ny + y) * nseg + (x >> kSegLog);
    }
};

inline Grid make_grid(const int32_t n[3]) {
    Grid g;
    g.nx = n[0]; g.ny = n[1]; g.nz = n[2];
    g.nseg = (n[0] + kSeg - 1) / kSeg;
    g.ncy = (n[1] + kCol - 1) / kCol;
    g.ncz = (n[2] + kCol - 1) / kCol;
    return g;
}

__host__ __device__ inline uint32_t pack_xyz(int x, int y, int z) {
    return (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20);
}

// Variant bits a solve accepts (a batched solve also LBM_VARIANT_NOGRAPH).
constexpr int32_t kVariantBits = LBM_VARIANT_EXPLICIT | LBM_VARIANT_REMAP | LBM_VARIANT_NTSTORE;
// ... and a single-lattice solve also LBM_VARIANT_OFF64.
constexpr int32_t kSolveVariantBits = kVariantBits | LBM_VARIANT_OFF64;

// ---------------------------------------------------------------- XCD-aware mapping
// Workgroups are dealt to the 8 XCDs round robin (workgroup b runs on XCD b % 8).
// Remap so that each XCD walks runs of `chunk` consecutive logical blocks, the 8 XCDs
// side by side: neighbouring rows of a column then share an L2.  The launch holds
// xcd_launch(blocks, chunk) workgroups (a multiple of 8 * chunk, so the map is a
// permutation of it); logical blocks >= blocks have no work.  chunk = ceil(blocks / 8)
// gives each XCD one contiguous eighth of the list.
constexpr int kXcd = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t chunk) {
    const int64_t x = b % kXcd, j = b / kXcd;
    return (j / chunk) * (kXcd * chunk) + x * chunk + j % chunk;
}
inline int64_t xcd_launch(int64_t blocks, int64_t chunk = 1) {
    const int64_t g = kXcd * (chunk > 0 ? chunk : 1);
    return (blocks + g - 1) / g * g;
}

// ---------------------------------------------------------------- steady state
// Distance of a converging field to its steady state, estimated from the decay of the
// convergence residual (Section 3.4 asks for the steady state; the residual alone bounds
// only the change per step).  When the field approaches its limit as a e^(-lambda t),
// the residual r = ||phi(t) - phi(t - n_c)|| / (n_c ||phi(t)||) falls by rho =
// e^(-lambda n_c) from one check to the next, and ||phi(t) - phi_inf|| / ||phi(t)|| =
// r n_c rho / (1 - rho).  rho is the geometric-mean ratio over the last kSteadyWindow
// check intervals (fewer at the start); no decay (rho >= 1) means no estimate (+inf).
constexpr int kSteadyWindow = 5;
struct SteadyEst {
    double r[kSteadyWindow + 1];
    int n = 0;
    void push(double v) {
        if (n == kSteadyWindow + 1) {
            for (int k = 0; k < kSteadyWindow; k++) r[k] = r[k + 1];
            n--;
        }
        r[n++] = v;
    }
    double dist(int nc) const {
        if (n < 1) return INFINITY;
        const double last = r[n - 1];
        if (last == 0.0) return 0.0;  // no change at all over the last interval
        if (n < 2 || !(last > 0.0) || !(r[0] > 0.0)) return INFINITY;
        const double rho = std::pow(last / r[0], 1.0 / (n - 1));
        if (!(rho < 1.0)) return INFINITY;
        return last * (double)nc * rho / (1.0 - rho);
    }
};

// Spread of the link-plane fluxes, (max - min) / |mean|: zero at steady state, where the
// same flux crosses every plane.  `floor` bounds the denominator from below (a medium
// without a path between the faces carries no steady flux at all).
inline double plane_spread(const double *planes, int count, double floor) {
    double mn = planes[0], mx = planes[0], mean = 0.0;
    for (int k = 0; k < count; k++) {
        mn = planes[k] < mn ? planes[k] : mn;
        mx = planes[k] > mx ? planes[k] : mx;
        mean += planes[k];
    }
    mean = std::fabs(mean / count);
    const double den = mean > floor ? mean : floor;
    return den > 0.0 ? (mx - mn) / den : INFINITY;
}

// ---------------------------------------------------------------- reductions
// Deterministic FP64 block reduction of NV values per thread.  Block size 256
// (4 waves of 64).  Thread 0 gets the block total in out[].
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *lds /* [4*NV] */, double (&out)[NV]) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double a = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        v[k] = a;
    }
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; k++) lds[wave * NV + k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; k++)
            out[k] = ((lds[k] + lds[NV + k]) + lds[2 * NV + k]) + lds[3 * NV + k];
}

// Sum `nblocks` rows of NV partials into res[NV] with one 256-thread block, in a fixed
// order (deterministic for a given nblocks).
// Batched solves: res[l][k] = the sum of the partial rows [b0, b1) of lattice lat_ids[l]
// (blockIdx.x = l), in a fixed order.  LD is the solve's lattice descriptor.
template <int NV, class LD>
__global__ __launch_bounds__(256) void k_lat_reduce(const double *__restrict__ partials,
                                                    const LD *__restrict__ lats,
                                                    const int32_t *__restrict__ lat_ids,
                                                    double *__restrict__ res) {
    __shared__ double lds[256];
    const int lat = lat_ids[blockIdx.x];
    const int64_t b0 = lats[lat].b0, b1 = lats[lat].b1;
    for (int k = 0; k < NV; k++) {
        double s = 0.0;
        for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) s += partials[b * NV + k];
        lds[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) res[lat * NV + k] = lds[0];
        __syncthreads();
    }
}

// Batched solves: the internal stream (ordered after the caller's stream by `join`),
// timing events and the captured graphs (kKeys per group: buffer parity and frame at
// the start of a check interval), released on every return.
struct BatchRes {
    static constexpr int kKeys = 4;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, join = nullptr;
    std::vector<hipGraphExec_t> exec;
    std::vector<hipGraph_t> graph;
    void reset_graphs(size_t groups) {
        for (size_t k = 0; k < exec.size(); k++) {
            if (exec[k]) (void)hipGraphExecDestroy(exec[k]);
            if (graph[k]) (void)hipGraphDestroy(graph[k]);
        }
        exec.assign(groups * kKeys, nullptr);
        graph.assign(groups * kKeys, nullptr);
    }
    lbm_status open(hipStream_t caller) {
        LBM_TRY_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        LBM_TRY_HIP(hipEventCreate(&e0));
        LBM_TRY_HIP(hipEventCreate(&e1));
        LBM_TRY_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
        LBM_TRY_HIP(hipEventRecord(join, caller));
        LBM_TRY_HIP(hipStreamWaitEvent(s, join, 0));
        return LBM_OK;
    }
    // later work on the caller's stream waits for everything issued on ours
    lbm_status close(hipStream_t caller) {
        LBM_TRY_HIP(hipEventRecord(join, s));
        LBM_TRY_HIP(hipStreamWaitEvent(caller, join, 0));
        return LBM_OK;
    }
    // On an error return the caller's stream was not joined: wait here for the work
    // already issued, so that none of it can touch the workspace after the call
    // returns (on success the solve has synchronised at its last check already).
    ~BatchRes() {
        if (s) (void)hipStreamSynchronize(s);
        reset_graphs(0);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (join) (void)hipEventDestroy(join);
        if (s) (void)hipStreamDestroy(s);
    }
};

// A group of active lattices that run a whole check interval together, one group after
// the other, so that a group whose state fits the Infinity Cache keeps it there.
struct BatchGroup {
    int64_t blk_off, n_blk;  // its run of the device block list
    int32_t lat_off, n_lat;  // its run of the device lattice-id list
    int64_t pl_off, n_pl;    // its run of the device plane list (Knudsen)
    double nodes;            // fluid nodes
};

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

// The Infinity Cache (MALL) of the device: a sweep whose state fits it runs
// cache-resident, a larger one streams from HBM.
constexpr double kCacheBytes = 256e6;

// Group budgets the autotuner of a batched solve tries, one check interval each: the
// whole batch as one group, then groups of at most 128, 192, 256 and 384 MB of state
// (the Infinity Cache holds 256 MB; a group a little larger still reuses part of it).
constexpr int kBatchBudgets = 5;
#define LBM_BATCH_BUDGETS {-1.0, 128e6, 192e6, 256e6, 384e6}

struct BatchLat {
    int64_t b0, b1, nf;
    int32_t nx;
};

// Splits the active lattices, in order, into groups of at most `budget` bytes of working
// set at `per_node` bytes per fluid node (budget <= 0: one group; a lattice above the
// budget is a group of its own) and fills the concatenated lists: blocks, lattice ids and,
// when `planes` is given, (lattice, x) pairs of every plane.
std::vector<BatchGroup> form_groups(const std::vector<int32_t> &act,
                                    const std::vector<BatchLat> &lat, double per_node,
                                    double budget, std::vector<int32_t> &blocks,
                                    std::vector<int32_t> &lat_ids, std::vector<int32_t> *planes);

lbm_status reduce_partials(const double *partials, int64_t nblocks, int nv, double *res,
                           hipStream_t s);

// ---------------------------------------------------------------- sparse layout
// Node ids are found through the rank map: one 16-byte word per row segment, holding
// the segment's 64-bit occupancy (bit x % 64) and the id of its first fluid node, so a
// voxel's id is base + popcount(bits below it).  At 1/4 byte per voxel the map stays
// cache resident.
// Each 32-bit half of the occupancy is stored beside the id of its own first fluid node,
// so that a lookup may load the 8 bytes of one half.  The flow sweep does (18 lookups in
// flight per node: half the registers lets its moment-space collision run 6 waves per
// SIMD instead of 4, 4.5 % faster at 512^3); the mass-transport sweeps load whole words,
// which measured faster for them (D3Q7 at 128^3: 10.2 against 10.8 us per step).
struct alignas(16) RankWord {
    uint32_t lo, base;     // occupancy bits 0-31; id of the segment's first fluid node
    uint32_t hi, base_hi;  // occupancy bits 32-63; id of the first fluid node among them
};
struct alignas(8) RankHalf {
    uint32_t bits, base;
};

// The half of segment word `seg` that holds bit `bit` (= x % 64).
__device__ inline RankHalf rank_half(const RankWord *__restrict__ rank, int64_t seg, int bit) {
    return reinterpret_cast<const RankHalf *>(rank + seg)[bit >> 5];
}

// Node id at bit `bit` (= x % 64) of the half h holding it, or -1 for a solid voxel.
__device__ inline int half_lookup(const RankHalf h, int bit) {
    const int b = bit & 31;
    if (!((h.bits >> b) & 1u)) return -1;
    return (int)(h.base + (uint32_t)__popc(h.bits & ((1u << b) - 1u)));
}

// Node id at bit `bit` (= x % 64) of the whole word w, or -1 for a solid voxel.
__device__ inline int rank_lookup(const RankWord w, int bit) {
    const uint64_t bits = (uint64_t)w.hi << 32 | w.lo;
    if (!((bits >> bit) & 1)) return -1;
    return (int)(w.base + (uint32_t)__popcll(bits & ((1ull << bit) - 1)));
}

// Node id of the in-domain voxel (x, y, z), or -1.
__device__ inline int node_at(const RankWord *__restrict__ rank, const Grid &g, int x, int y, int z) {
    return half_lookup(rank_half(rank, g.seg(x, y, z), x & (kSeg - 1)), x & (kSeg - 1));
}

// layout_count: the rank map's occupancy bits and bases (g.nsegs() words; ids start at
// id_base); the number of fluid nodes goes to *nf_h (host sync); total_d is one int32 of
// device scratch.
// layout_fill: the upper-half bases of the rank words, and coords[id] = packed
// x | y<<10 | z<<20 of every fluid node.
lbm_status layout_count(const Grid &g, const uint8_t *fluid, RankWord *rank, int32_t *total_d,
                        int64_t *nf_h, hipStream_t s, uint32_t id_base = 0);
lbm_status layout_fill(const Grid &g, RankWord *rank, uint32_t *coords, hipStream_t s);

// Counting kernel usable by several entry points.
lbm_status count_nonzero(const Grid &g, const uint8_t *mask, unsigned long long *dcount,
                         int64_t *count_h, hipStream_t s);

}  // namespace lbm
