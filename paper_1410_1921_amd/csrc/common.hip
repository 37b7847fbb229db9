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
__global__ __launch_bounds__(256) void k_reduce_partials(const double *__restrict__ p,
                                                         int64_t nblocks, int nv,
                                                         double *__restrict__ res) {
    __shared__ double lds[256];
    for (int k = 0; k < nv; k++) {
        double a = 0.0;
        for (int64_t b = threadIdx.x; b < nblocks; b += 256) a += p[b * nv + k];
        lds[threadIdx.x] = a;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) lds[threadIdx.x] += lds[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) res[k] = lds[0];
        __syncthreads();
    }
}

lbm_status reduce_partials(const double *partials, int64_t nblocks, int nv, double *res,
                           hipStream_t s) {
    k_reduce_partials<<<1, 256, 0, s>>>(partials, nblocks, nv, res);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

// ---------------------------------------------------------------- sparse layout
// One workgroup per brick, one thread per voxel slot of the brick.
__device__ inline bool brick_voxel(const Grid &g, int64_t brick, int t, int &x, int &y, int &z) {
    int bx = (int)(brick % g.nbx);
    int by = (int)((brick / g.nbx) % g.nby);
    int bz = (int)(brick / ((int64_t)g.nbx * g.nby));
    x = (bx << kBrickLog) | (t & (kBrick - 1));
    y = (by << kBrickLog) | ((t >> kBrickLog) & (kBrick - 1));
    z = (bz << kBrickLog) | (t >> (2 * kBrickLog));
    return x < g.nx && y < g.ny && z < g.nz;
}

__global__ __launch_bounds__(kBrickVox) void k_brick_count(Grid g, const uint8_t *__restrict__ fluid,
                                                           int32_t *__restrict__ bcount) {
    int x, y, z;
    int64_t brick = blockIdx.x;
    bool in = brick_voxel(g, brick, threadIdx.x, x, y, z);
    int flag = in && fluid[g.lin(x, y, z)] != 0;
    int c = __syncthreads_count(flag);
    if (threadIdx.x == 0) bcount[brick] = c;
}

// Exclusive scan of nb counts in place, total at [nb]; one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(int32_t *__restrict__ a, int64_t nb) {
    __shared__ int64_t part[1024];
    int64_t per = (nb + 1023) / 1024;
    int64_t lo = threadIdx.x * per, hi = lo + per < nb ? lo + per : nb;
    int64_t sum = 0;
    for (int64_t i = lo; i < hi; i++) sum += a[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < 1024; i++) {
            int64_t v = part[i];
            part[i] = run;
            run += v;
        }
        a[nb] = (int32_t)run;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t i = lo; i < hi; i++) {
        int32_t v = a[i];
        a[i] = (int32_t)run;
        run += v;
    }
}

__global__ __launch_bounds__(kBrickVox) void k_brick_fill(Grid g, const uint8_t *__restrict__ fluid,
                                                          const int32_t *__restrict__ boff,
                                                          int32_t *__restrict__ idmap,
                                                          uint32_t *__restrict__ coords) {
    __shared__ int wave_tot[kBrickVox / 64];
    int x, y, z;
    int64_t brick = blockIdx.x;
    bool in = brick_voxel(g, brick, threadIdx.x, x, y, z);
    bool flag = in && fluid[g.lin(x, y, z)] != 0;
    uint64_t ball = __ballot(flag);
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int before = __popcll(ball & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    if (lane == 0) wave_tot[wave] = __popcll(ball);
    __syncthreads();
    int base = boff[brick];
    for (int w = 0; w < wave; w++) base += wave_tot[w];
    int32_t id = flag ? base + before : -1;
    idmap[brick * kBrickVox + threadIdx.x] = id;
    if (flag) coords[id] = pack_xyz(x, y, z);
}

lbm_status layout_count(const Grid &g, const uint8_t *fluid, int32_t *bcount, int64_t *nf_h,
                        hipStream_t s) {
    int64_t nb = g.nbricks();
    k_brick_count<<<(unsigned)nb, kBrickVox, 0, s>>>(g, fluid, bcount);
    LBM_CHECK_LAUNCH();
    k_scan<<<1, 1024, 0, s>>>(bcount, nb);
    LBM_CHECK_LAUNCH();
    int32_t total = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&total, bcount + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    *nf_h = total;
    return LBM_OK;
}

lbm_status layout_fill(const Grid &g, const uint8_t *fluid, const int32_t *boff, int32_t *idmap,
                       uint32_t *coords, hipStream_t s) {
    k_brick_fill<<<(unsigned)g.nbricks(), kBrickVox, 0, s>>>(g, fluid, boff, idmap, coords);
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
