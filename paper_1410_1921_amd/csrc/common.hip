// Errors, device check, counting, the sparse fluid-node layout and the fixed-order
// FP64 reduction of per-block partial sums.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "lbm_internal.h"

namespace lbm {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

lbm_status check_device() {
    int dev = 0;
    LBM_TRY_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    LBM_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    LBM_REQUIRE(std::strncmp(prop.gcnArchName, "gfx950", 6) == 0, LBM_E_DEVICE,
                "device %d is %s; this library is built for gfx950 only", dev, prop.gcnArchName);
    return LBM_OK;
}

// ---------------------------------------------------------------- counting
__global__ __launch_bounds__(256) void k_count(const uint8_t *__restrict__ m, int64_t n,
                                               unsigned long long *out) {
    unsigned long long c = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        c += m[i] != 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, c);
}

lbm_status count_nonzero(const Grid &g, const uint8_t *mask, unsigned long long *dcount,
                         int64_t *count_h, hipStream_t s) {
    LBM_TRY_HIP(hipMemsetAsync(dcount, 0, sizeof(unsigned long long), s));
    int64_t blocks = (g.nvox() + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_count<<<(unsigned)blocks, 256, 0, s>>>(mask, g.nvox(), dcount);
    LBM_CHECK_LAUNCH();
    unsigned long long h = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&h, dcount, sizeof(h), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    *count_h = (int64_t)h;
    return LBM_OK;
}

// ---------------------------------------------------------------- fixed-order reduction
// One block of 1024 threads (enough loads in flight to read the rows at cache speed):
// thread t adds rows t, t + 1024, ... in that order, each wave folds its 64 lanes with a
// fixed shuffle tree, and thread k < nv adds the 16 wave sums of sum k in wave order.
// All nv sums go through one pass; the order of every addition is fixed, so the result
// is bitwise reproducible.
constexpr int kMaxSums = 8;
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_reduce_partials(const double *__restrict__ p,
                                                                    int64_t nblocks, int nv,
                                                                    double *__restrict__ res) {
    __shared__ double lds[kMaxSums][kReduceThreads / 64];
    double a[kMaxSums];
#pragma unroll
    for (int k = 0; k < kMaxSums; k++) a[k] = 0.0;
#pragma unroll 4
    for (int64_t b = threadIdx.x; b < nblocks; b += kReduceThreads) {
        const double *row = p + b * nv;
#pragma unroll
        for (int k = 0; k < kMaxSums; k++)
            if (k < nv) a[k] += row[k];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < kMaxSums; k++) a[k] += __shfl_down(a[k], off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < kMaxSums; k++) lds[k][wave] = a[k];
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        double t = 0.0;
        for (int w = 0; w < kReduceThreads / 64; w++) t += lds[threadIdx.x][w];
        res[threadIdx.x] = t;
    }
}

lbm_status reduce_partials(const double *partials, int64_t nblocks, int nv, double *res,
                           hipStream_t s) {
    LBM_REQUIRE(nv >= 1 && nv <= kMaxSums, LBM_E_INVAL, "reduce_partials: %d sums", nv);
    k_reduce_partials<<<1, kReduceThreads, 0, s>>>(partials, nblocks, nv, res);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

// ---------------------------------------------------------------- sparse layout
// One wave per row segment: its ballot is the segment's occupancy.  The count goes to
// the base field until the scan turns it into the segment's first node id.
__global__ __launch_bounds__(256) void k_seg_count(Grid g, const uint8_t *__restrict__ fluid,
                                                   RankWord *__restrict__ rank) {
    const int64_t sg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (sg >= g.nsegs()) return;  // uniform per wave
    const int sx = (int)(sg % g.nseg);
    const int64_t row = sg / g.nseg;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    const int x = sx * kSeg + lane;
    const bool flag = x < g.nx && fluid[g.lin(x, y, z)] != 0;
    const uint64_t ball = __ballot(flag);
    if (lane == 0) {
        RankWord r;
        r.lo = (uint32_t)ball;
        r.hi = (uint32_t)(ball >> 32);
        r.base = (uint32_t)__popcll(ball);
        r.base_hi = 0;
        rank[sg] = r;
    }
}

// Row of position r in column order over the padded cross-section; false outside.
__device__ inline bool column_row(const Grid &g, int64_t r, int &y, int &z) {
    const int64_t col = r / (kCol * kCol);
    const int q = (int)(r % (kCol * kCol));
    z = (int)(col / g.ncy) * kCol + q / kCol;
    y = (int)(col % g.ncy) * kCol + q % kCol;
    return y < g.ny && z < g.nz;
}

// Exclusive scan, in list order, of the segment counts held in rank[].base, in place,
// offset by id_base (the id of the lattice's first node); the count goes to *total.
// One block of 1024 threads, each over a run of rows.
__global__ __launch_bounds__(1024) void k_seg_scan(RankWord *__restrict__ rank, Grid g,
                                                   int32_t *__restrict__ total, uint32_t id_base) {
    __shared__ int64_t part[1024];
    const int64_t nrows = (int64_t)g.ncz * g.ncy * kCol * kCol;
    const int64_t per = (nrows + 1023) / 1024;
    const int64_t lo = threadIdx.x * per, hi = lo + per < nrows ? lo + per : nrows;
    int64_t sum = 0;
    int y, z;
    for (int64_t r = lo; r < hi; r++) {
        if (!column_row(g, r, y, z)) continue;
        const int64_t s0 = g.seg(0, y, z);
        for (int sx = 0; sx < g.nseg; sx++) sum += rank[s0 + sx].base;
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < 1024; i++) {
            const int64_t v = part[i];
            part[i] = run;
            run += v;
        }
        *total = (int32_t)run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x] + id_base;
    for (int64_t r = lo; r < hi; r++) {
        if (!column_row(g, r, y, z)) continue;
        const int64_t s0 = g.seg(0, y, z);
        for (int sx = 0; sx < g.nseg; sx++) {
            const uint32_t v = rank[s0 + sx].base;
            rank[s0 + sx].base = (uint32_t)run;
            run += v;
        }
    }
}

// One wave per row segment: the id of the first fluid node of the word's upper half, and
// the packed coordinates of the segment's nodes.
__global__ __launch_bounds__(256) void k_seg_fill(Grid g, RankWord *__restrict__ rank,
                                                  uint32_t *__restrict__ coords) {
    const int64_t sg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (sg >= g.nsegs()) return;
    const RankWord w = rank[sg];
    if (lane == 0) rank[sg].base_hi = w.base + (uint32_t)__popc(w.lo);
    const uint64_t bits = (uint64_t)w.hi << 32 | w.lo;
    if (!((bits >> lane) & 1)) return;
    const int sx = (int)(sg % g.nseg);
    const int64_t row = sg / g.nseg;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    const uint32_t id = w.base + (uint32_t)__popcll(bits & ((1ull << lane) - 1));
    coords[id] = pack_xyz(sx * kSeg + lane, y, z);
}

lbm_status layout_count(const Grid &g, const uint8_t *fluid, RankWord *rank, int32_t *total_d,
                        int64_t *nf_h, hipStream_t s, uint32_t id_base) {
    const int64_t blocks = (g.nsegs() + 3) / 4;
    k_seg_count<<<(unsigned)blocks, 256, 0, s>>>(g, fluid, rank);
    LBM_CHECK_LAUNCH();
    k_seg_scan<<<1, 1024, 0, s>>>(rank, g, total_d, id_base);
    LBM_CHECK_LAUNCH();
    int32_t total = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&total, total_d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    *nf_h = total;
    return LBM_OK;
}

std::vector<BatchGroup> form_groups(const std::vector<int32_t> &act,
                                    const std::vector<BatchLat> &lat, double per_node,
                                    double budget, std::vector<int32_t> &blocks,
                                    std::vector<int32_t> &lat_ids, std::vector<int32_t> *planes) {
    std::vector<BatchGroup> groups;
    blocks.clear();
    lat_ids.clear();
    if (planes) planes->clear();
    double bytes = 0.0;
    for (int32_t l : act) {
        const BatchLat &L = lat[l];
        const double b = per_node * (double)L.nf;
        if (groups.empty() || (budget > 0 && bytes > 0 && bytes + b > budget)) {
            BatchGroup g;
            g.blk_off = (int64_t)blocks.size();
            g.lat_off = (int32_t)lat_ids.size();
            g.pl_off = planes ? (int64_t)planes->size() / 2 : 0;
            g.n_blk = g.n_lat = g.n_pl = 0;
            g.nodes = 0.0;
            groups.push_back(g);
            bytes = 0.0;
        }
        BatchGroup &g = groups.back();
        for (int64_t k = L.b0; k < L.b1; k++) blocks.push_back((int32_t)k);
        lat_ids.push_back(l);
        if (planes)
            for (int x = 0; x < L.nx; x++) {
                planes->push_back(l);
                planes->push_back(x);
            }
        g.n_blk += L.b1 - L.b0;
        g.n_lat += 1;
        g.n_pl += planes ? L.nx : 0;
        g.nodes += (double)L.nf;
        bytes += b;
    }
    return groups;
}

lbm_status layout_fill(const Grid &g, RankWord *rank, uint32_t *coords, hipStream_t s) {
    k_seg_fill<<<(unsigned)((g.nsegs() + 3) / 4), 256, 0, s>>>(g, rank, coords);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_count(const int32_t n[3], const uint8_t *mask, int64_t *count_h,
                                void *workspace, size_t ws_bytes, void *stream) {
    LBM_REQUIRE(n && mask && count_h && workspace, LBM_E_INVAL, "lbm_count: null argument");
    LBM_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1, LBM_E_INVAL, "lbm_count: bad size");
    LBM_REQUIRE(ws_bytes >= 256, LBM_E_NOMEM, "lbm_count: workspace below 256 bytes");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    Grid g = make_grid(n);
    return count_nonzero(g, mask, static_cast<unsigned long long *>(workspace), count_h,
                         static_cast<hipStream_t>(stream));
}

extern "C" const char *lbm_last_error(void) { return lbm::g_err; }
