// Internal declarations shared by the translation units of liblbm.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

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
// Bricks of 8x8x8 voxels; inside a brick voxels run x fastest.  The fluid-node list is
// ordered brick by brick (bricks x fastest), so a brick's nodes are contiguous.
constexpr int kBrickLog = 3;
constexpr int kBrick = 1 << kBrickLog;
constexpr int kBrickVox = kBrick * kBrick * kBrick;
constexpr int kMaxEdge = 1024;  // coordinates packed in 10 bits each

struct Grid {
    int nx, ny, nz;
    int nbx, nby, nbz;
    __host__ __device__ int64_t nvox() const { return (int64_t)nx * ny * nz; }
    __host__ __device__ int64_t nbricks() const { return (int64_t)nbx * nby * nbz; }
    __host__ __device__ int64_t lin(int x, int y, int z) const {
        return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
    }
    // brick-major voxel slot of in-domain coordinates
    __host__ __device__ int64_t slot(int x, int y, int z) const {
        int64_t b = ((int64_t)(z >> kBrickLog) * nby + (y >> kBrickLog)) * nbx + (x >> kBrickLog);
        int l = (((z & (kBrick - 1)) << kBrickLog | (y & (kBrick - 1))) << kBrickLog) |
                (x & (kBrick - 1));
        return b * kBrickVox + l;
    }
};

inline Grid make_grid(const int32_t n[3]) {
    Grid g;
    g.nx = n[0]; g.ny = n[1]; g.nz = n[2];
    g.nbx = (n[0] + kBrick - 1) / kBrick;
    g.nby = (n[1] + kBrick - 1) / kBrick;
    g.nbz = (n[2] + kBrick - 1) / kBrick;
    return g;
}

__host__ __device__ inline uint32_t pack_xyz(int x, int y, int z) {
    return (uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20);
}

// ---------------------------------------------------------------- XCD-aware mapping
// Workgroups are dealt to the 8 XCDs round robin (workgroup b runs on XCD b % 8).
// Remap so that each XCD walks one contiguous run of logical blocks: neighbouring
// bricks then share an L2.  `launched` is a multiple of 8.
constexpr int kXcd = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t launched) {
    int64_t per = launched / kXcd;
    return (b % kXcd) * per + b / kXcd;
}
inline int64_t xcd_launch(int64_t blocks) { return (blocks + kXcd - 1) / kXcd * kXcd; }

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
lbm_status reduce_partials(const double *partials, int64_t nblocks, int nv, double *res,
                           hipStream_t s);

// ---------------------------------------------------------------- sparse layout
// The fluid-node list (node ids brick by brick) and the brick-major id map.
// layout_count: per-brick fluid counts turned into exclusive offsets in bcount
// [nbricks + 1]; the total goes to *nf_h (host sync).
// layout_fill: idmap[slot] = node id or -1, coords[id] = packed x | y<<10 | z<<20.
lbm_status layout_count(const Grid &g, const uint8_t *fluid, int32_t *bcount, int64_t *nf_h,
                        hipStream_t s);
lbm_status layout_fill(const Grid &g, const uint8_t *fluid, const int32_t *boff, int32_t *idmap,
                       uint32_t *coords, hipStream_t s);

// Counting kernel usable by several entry points.
lbm_status count_nonzero(const Grid &g, const uint8_t *mask, unsigned long long *dcount,
                         int64_t *count_h, hipStream_t s);

}  // namespace lbm
