// Structure characterisation on the GPU (Section 4.1): 18-neighbour connected-component
// labelling with transport flags, the 13-direction chord pore size, and the exact
// squared Euclidean distance map with its maximum-inscribed-sphere pore width.
// Everything is integer except the final FP64 formulas, which are evaluated in the
// stated order (this file is compiled with -ffp-contract=off).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "lbm_internal.h"

namespace lbm {

constexpr int32_t kInf = 0x3fffffff;

// ================================================================ labelling
__global__ __launch_bounds__(256) void k_ccl_init(int64_t nv, const uint8_t *__restrict__ pore,
                                                  int32_t *__restrict__ L) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < nv) L[v] = pore[v] ? (int32_t)v : -1;
}

__device__ inline int32_t ccl_root(int32_t *L, int32_t v) {
    int32_t p = __hip_atomic_load(&L[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (p != v) {
        v = p;
        p = __hip_atomic_load(&L[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return v;
}

// Union of the trees of a and b: the larger root is pointed at the smaller one, so the
// final root of every component is its smallest index.  When the atomic finds that b
// was no longer a root, the merge continues with b's new parent.
__device__ inline void ccl_unite(int32_t *L, int32_t a, int32_t b) {
    for (;;) {
        a = ccl_root(L, a);
        b = ccl_root(L, b);
        if (a == b) return;
        if (a > b) { int32_t t = a; a = b; b = t; }
        const int32_t old = atomicMin(&L[b], a);
        if (old == b) return;
        b = old;
    }
}

// Each of the 9 neighbour offsets of the forward half of the 18-neighbourhood is taken
// once per voxel, so every link of the neighbourhood graph is visited.
__global__ __launch_bounds__(256) void k_ccl_merge(Grid g, const uint8_t *__restrict__ pore,
                                                   int32_t *L) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= g.nvox() || !pore[v]) return;
    const int x = (int)(v % g.nx), y = (int)((v / g.nx) % g.ny), z = (int)(v / ((int64_t)g.nx * g.ny));
    for (int dz = 0; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                const int m = (dx != 0) + (dy != 0) + (dz != 0);
                if (m == 0 || m == 3) continue;
                if (dz == 0 && (dy < 0 || (dy == 0 && dx < 0))) continue;
                const int xx = x + dx;
                if (xx < 0 || xx >= g.nx) continue;  // open in x
                int yy = y + dy, zz = z + dz;        // periodic in y and z
                yy = yy < 0 ? yy + g.ny : (yy >= g.ny ? yy - g.ny : yy);
                zz = zz >= g.nz ? zz - g.nz : zz;
                const int64_t u = g.lin(xx, yy, zz);
                if (pore[u]) ccl_unite(L, (int32_t)v, (int32_t)u);
            }
}

__global__ __launch_bounds__(256) void k_ccl_compress(int64_t nv, int32_t *L) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    const int32_t l = L[v];
    if (l >= 0) L[v] = ccl_root(L, (int32_t)v);
}

__global__ __launch_bounds__(256) void k_ccl_faces(Grid g, const int32_t *__restrict__ L,
                                                   uint8_t *__restrict__ fin,
                                                   uint8_t *__restrict__ fout) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= (int64_t)g.ny * g.nz) return;
    const int y = (int)(k % g.ny), z = (int)(k / g.ny);
    const int32_t a = L[g.lin(0, y, z)], b = L[g.lin(g.nx - 1, y, z)];
    if (a >= 0) fin[a] = 1;
    if (b >= 0) fout[b] = 1;
}

__global__ __launch_bounds__(256) void k_ccl_finish(int64_t nv, const int32_t *__restrict__ L,
                                                    const uint8_t *__restrict__ fin,
                                                    const uint8_t *__restrict__ fout,
                                                    uint8_t *__restrict__ transport,
                                                    unsigned long long *counts) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned long long c[3] = {0, 0, 0};
    if (v < nv) {
        const int32_t l = L[v];
        const int t = l >= 0 && fin[l] && fout[l];
        if (transport) transport[v] = (uint8_t)t;
        c[0] = l >= 0;
        c[1] = t;
        c[2] = l == (int32_t)v;
    }
#pragma unroll
    for (int k = 0; k < 3; k++) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c[k] += __shfl_down(c[k], off, 64);
        if ((threadIdx.x & 63) == 0 && c[k]) atomicAdd(&counts[k], c[k]);
    }
}

// ================================================================ 13-direction chords
// The 13 line directions: 3 axes, 6 face diagonals, 4 body diagonals.
__constant__ int8_t kDir13[13][3] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {1, 1, 0},  {1, -1, 0},
                                     {1, 0, 1},  {1, 0, -1}, {0, 1, 1},  {0, 1, -1}, {1, 1, 1},
                                     {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};

// One thread per line of direction d: walks the line from the face where it enters the
// box and adds each run's voxel count to every voxel of the run.
__global__ __launch_bounds__(256) void k_chords(Grid g, int d, const uint8_t *__restrict__ pore,
                                                int32_t *__restrict__ cnt) {
    const int dx = kDir13[d][0], dy = kDir13[d][1], dz = kDir13[d][2];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t fx = (int64_t)g.ny * g.nz, fy = (int64_t)g.nx * g.nz, fz = (int64_t)g.nx * g.ny;
    const int x0 = dx > 0 ? 0 : g.nx - 1, y0 = dy > 0 ? 0 : g.ny - 1, z0 = dz > 0 ? 0 : g.nz - 1;
    int x, y, z;
    if (t < fx) {  // entering through the x face
        if (dx == 0) return;
        x = x0; y = (int)(t % g.ny); z = (int)(t / g.ny);
    } else if (t < fx + fy) {
        if (dy == 0) return;
        const int64_t k = t - fx;
        x = (int)(k % g.nx); y = y0; z = (int)(k / g.nx);
        if (dx != 0 && x == x0) return;  // already started from the x face
    } else if (t < fx + fy + fz) {
        if (dz == 0) return;
        const int64_t k = t - fx - fy;
        x = (int)(k % g.nx); y = (int)(k / g.nx); z = z0;
        if ((dx != 0 && x == x0) || (dy != 0 && y == y0)) return;
    } else {
        return;
    }
    int run = 0;
    for (;;) {
        const bool in = x >= 0 && x < g.nx && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
        const bool p = in && pore[g.lin(x, y, z)];
        if (p) {
            run++;
        } else if (run > 0) {
            int bx = x, by = y, bz = z;
            for (int k = 0; k < run; k++) {
                bx -= dx; by -= dy; bz -= dz;
                cnt[g.lin(bx, by, bz)] += run;
            }
            run = 0;
        }
        if (!in) break;
        x += dx; y += dy; z += dz;
    }
}

__global__ __launch_bounds__(256) void k_chord_final(int64_t nv, const uint8_t *__restrict__ pore,
                                                     const int32_t *__restrict__ A,
                                                     const int32_t *__restrict__ B,
                                                     const int32_t *__restrict__ C, double s2,
                                                     double s3, double *__restrict__ diam) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    if (!pore[v]) {
        diam[v] = 0.0;
        return;
    }
    const double a = (double)A[v], b = (double)B[v], c = (double)C[v];
    const double t1 = s2 * b;
    const double t2 = a + t1;
    const double t3 = s3 * c;
    const double t4 = t2 + t3;
    diam[v] = t4 / 13.0;
}

// ================================================================ distance map
// Squared distance to the nearest solid voxel along x (two scans per row).
__global__ __launch_bounds__(256) void k_edt_x(Grid g, const uint8_t *__restrict__ pore,
                                               int32_t *__restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= (int64_t)g.ny * g.nz) return;
    const int64_t base = r * g.nx;
    int last = -1;
    for (int x = 0; x < g.nx; x++) {
        if (!pore[base + x]) last = x;
        out[base + x] = last < 0 ? kInf : (x - last);  // distance, squared below
    }
    int next = -1;
    for (int x = g.nx - 1; x >= 0; x--) {
        if (!pore[base + x]) next = x;
        int d = out[base + x];
        if (next >= 0 && next - x < d) d = next - x;
        out[base + x] = d >= kInf ? kInf : d * d;
    }
}

// One more axis of the separable minimum: out(p) = min_t in(p with axis = t) + (p_a - t)^2,
// searched outwards from p until the distance term alone reaches the best value.
__global__ __launch_bounds__(256) void k_edt_axis(Grid g, int axis, const int32_t *__restrict__ in,
                                                  int32_t *__restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= g.nvox()) return;
    const int64_t stride = axis == 1 ? (int64_t)g.nx : (int64_t)g.nx * g.ny;
    const int len = axis == 1 ? g.ny : g.nz;
    const int p = axis == 1 ? (int)((v / g.nx) % g.ny) : (int)(v / ((int64_t)g.nx * g.ny));
    int best = in[v];
    for (int r = 1; r < len && r * r < best; r++) {
        const int r2 = r * r;
        if (p - r >= 0) {
            const int a = in[v - r * stride];
            if (a < kInf && a + r2 < best) best = a + r2;
        }
        if (p + r < len) {
            const int b = in[v + r * stride];
            if (b < kInf && b + r2 < best) best = b + r2;
        }
    }
    out[v] = best;
}

__global__ __launch_bounds__(256) void k_max_i32(int64_t nv, const int32_t *__restrict__ a,
                                                 const uint8_t *__restrict__ pore, int *out) {
    int m = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += (int64_t)gridDim.x * 256)
        if (pore[i] && a[i] > m) m = a[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_down(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// Widest inscribed ball covering each pore voxel: max E(c) over centres c with
// |p - c|^2 < E(c), searched over the cube of half-width R = ceil(sqrt(max E)); solid
// voxels have E = 0 and never qualify.  width[] maps E to 2 sqrt(E) - 1 (built on the
// host, correctly rounded).
__global__ __launch_bounds__(256) void k_mis(Grid g, int R, int emax_all,
                                             const int32_t *__restrict__ E,
                                             const uint8_t *__restrict__ pore,
                                             const double *__restrict__ width,
                                             double *__restrict__ diam) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= g.nvox()) return;
    if (!pore[v]) {
        diam[v] = 0.0;
        return;
    }
    const int x = (int)(v % g.nx), y = (int)((v / g.nx) % g.ny), z = (int)(v / ((int64_t)g.nx * g.ny));
    int best = 0;
    const int z0 = z - R < 0 ? 0 : z - R, z1 = z + R >= g.nz ? g.nz - 1 : z + R;
    const int y0 = y - R < 0 ? 0 : y - R, y1 = y + R >= g.ny ? g.ny - 1 : y + R;
    const int x0 = x - R < 0 ? 0 : x - R, x1 = x + R >= g.nx ? g.nx - 1 : x + R;
    for (int zz = z0; zz <= z1; zz++) {
        const int dz2 = (zz - z) * (zz - z);
        if (dz2 >= emax_all) continue;
        for (int yy = y0; yy <= y1; yy++) {
            const int dyz2 = dz2 + (yy - y) * (yy - y);
            if (dyz2 >= emax_all) continue;
            const int64_t row = g.lin(0, yy, zz);
            for (int xx = x0; xx <= x1; xx++) {
                const int d2 = dyz2 + (xx - x) * (xx - x);
                const int e = E[row + xx];
                if (e > d2 && e > best) best = e;
            }
        }
    }
    diam[v] = width[best];
}

}  // namespace lbm

using namespace lbm;

static lbm_status check_n(const int32_t n[3]) {
    LBM_REQUIRE(n, LBM_E_INVAL, "null size");
    LBM_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && n[0] <= kMaxEdge && n[1] <= kMaxEdge &&
                    n[2] <= kMaxEdge,
                LBM_E_INVAL, "sizes must lie in [1, %d]", kMaxEdge);
    return LBM_OK;
}

namespace lbm {
size_t label_ws_bytes_n(const int32_t n[3]) {
    Grid g = make_grid(n);
    Carver c(nullptr);
    c.take<unsigned long long>(4);
    c.take<uint8_t>(g.nvox());
    c.take<uint8_t>(g.nvox());
    return c.off;
}
size_t diam_ws_bytes_n(const int32_t n[3]) {
    Grid g = make_grid(n);
    Carver c(nullptr);
    c.take<unsigned long long>(4);
    c.take<int32_t>(g.nvox());
    c.take<int32_t>(g.nvox());
    c.take<int32_t>(g.nvox());
    c.take<double>(3 * (size_t)kMaxEdge * kMaxEdge + 1);
    return c.off;
}
}  // namespace lbm

namespace lbm {
// Zero fill of scratch memory by a kernel (no memset node in a caller's captured graph).
__global__ __launch_bounds__(256) void k_zero_bytes(uint8_t *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = 0;
}

// The labelling passes on scratch holding 4 counters and two voxel flag arrays (cleared
// here: by memsets, or by fill kernels when `fill` is set), then the stats (host sync).
static lbm_status label_run(const Grid &g, const uint8_t *pore, int32_t *label, uint8_t *transport,
                            lbm_label_stats *stats_h, unsigned long long *counts, uint8_t *fin,
                            uint8_t *fout, bool fill, hipStream_t s) {
    const int64_t nv = g.nvox();
    const unsigned blocks = (unsigned)((nv + 255) / 256);
    if (fill) {
        k_zero_bytes<<<1, 256, 0, s>>>(reinterpret_cast<uint8_t *>(counts),
                                        4 * sizeof(unsigned long long));
        LBM_CHECK_LAUNCH();
        const unsigned zb = (unsigned)std::min<int64_t>((nv + 255) / 256, 4096);
        k_zero_bytes<<<zb, 256, 0, s>>>(fin, nv);
        LBM_CHECK_LAUNCH();
        k_zero_bytes<<<zb, 256, 0, s>>>(fout, nv);
        LBM_CHECK_LAUNCH();
    } else {
        LBM_TRY_HIP(hipMemsetAsync(counts, 0, 4 * sizeof(unsigned long long), s));
        LBM_TRY_HIP(hipMemsetAsync(fin, 0, nv, s));
        LBM_TRY_HIP(hipMemsetAsync(fout, 0, nv, s));
    }
    k_ccl_init<<<blocks, 256, 0, s>>>(nv, pore, label);
    LBM_CHECK_LAUNCH();
    k_ccl_merge<<<blocks, 256, 0, s>>>(g, pore, label);
    LBM_CHECK_LAUNCH();
    k_ccl_compress<<<blocks, 256, 0, s>>>(nv, label);
    LBM_CHECK_LAUNCH();
    k_ccl_faces<<<(unsigned)(((int64_t)g.ny * g.nz + 255) / 256), 256, 0, s>>>(g, label, fin, fout);
    LBM_CHECK_LAUNCH();
    k_ccl_finish<<<blocks, 256, 0, s>>>(nv, label, fin, fout, transport, counts);
    LBM_CHECK_LAUNCH();
    unsigned long long h[3];
    LBM_TRY_HIP(hipMemcpyAsync(h, counts, sizeof(h), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    stats_h->n_pore = (int64_t)h[0];
    stats_h->n_transport = (int64_t)h[1];
    stats_h->n_components = (int64_t)h[2];
    stats_h->porosity = (double)h[0] / (double)nv;
    stats_h->connectivity = h[0] ? (double)h[1] / (double)h[0] : 0.0;
    return LBM_OK;
}

// Scratch of lbm_label_noalloc: 256 bytes of counters and the two face-flag arrays of a
// volume of up to LBM_LABEL_NOALLOC_MAX_VOXELS voxels (32 MiB + 256 B in all), one copy per
// device for the life of the process.  Host code uses the per-device address from
// hipGetSymbolAddress, never the symbol itself.
constexpr int64_t kNoallocVox = LBM_LABEL_NOALLOC_MAX_VOXELS;
static __device__ __align__(256) uint8_t scratch[256 + 2 * kNoallocVox];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static lbm_status scratch_address(void **out) {
    int dev = -1;
    LBM_TRY_HIP(hipGetDevice(&dev));
    LBM_REQUIRE(dev >= 0 && dev < kMaxDevices, LBM_E_DEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        LBM_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        LBM_REQUIRE(p, LBM_E_DEVICE, "no address for the scratch array on device %d", dev);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace lbm

extern "C" lbm_status lbm_label(const int32_t n[3], const uint8_t *pore, int32_t *label,
                                uint8_t *transport, lbm_label_stats *stats_h, void *workspace,
                                size_t ws_bytes, void *stream) {
    lbm_status st = check_n(n);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(pore && label && stats_h && workspace, LBM_E_INVAL, "lbm_label: null argument");
    LBM_REQUIRE(ws_bytes >= label_ws_bytes_n(n), LBM_E_NOMEM, "lbm_label: workspace too small");
    st = check_device();
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g = make_grid(n);
    Carver c(workspace);
    unsigned long long *counts = c.take<unsigned long long>(4);
    uint8_t *fin = c.take<uint8_t>(g.nvox());
    uint8_t *fout = c.take<uint8_t>(g.nvox());
    return label_run(g, pore, label, transport, stats_h, counts, fin, fout, false, s);
}

extern "C" lbm_status lbm_label_noalloc(const int32_t n[3], const uint8_t *pore, int32_t *label,
                                        uint8_t *transport, lbm_label_stats *stats_h,
                                        void *stream) {
    lbm_status st = check_n(n);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(pore && label && stats_h, LBM_E_INVAL, "lbm_label_noalloc: null argument");
    const Grid g = make_grid(n);
    LBM_REQUIRE(g.nvox() <= kNoallocVox, LBM_E_NOMEM,
                "lbm_label_noalloc: %lld voxels exceed its scratch of %lld voxels",
                (long long)g.nvox(), (long long)kNoallocVox);
    st = check_device();
    if (st != LBM_OK) return st;
    void *base = nullptr;
    st = scratch_address(&base);
    if (st != LBM_OK) return st;
    uint8_t *b = static_cast<uint8_t *>(base);
    return label_run(g, pore, label, transport, stats_h, reinterpret_cast<unsigned long long *>(b),
                     b + 256, b + 256 + g.nvox(), true, static_cast<hipStream_t>(stream));
}

extern "C" lbm_status lbm_pore_diameter(const int32_t n[3], const uint8_t *pore, int32_t method,
                                        double *diam, void *workspace, size_t ws_bytes,
                                        void *stream) {
    lbm_status st = check_n(n);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(pore && diam && workspace, LBM_E_INVAL, "lbm_pore_diameter: null argument");
    LBM_REQUIRE(method == LBM_PSD_CHORD13 || method == LBM_PSD_MIS, LBM_E_INVAL,
                "unknown pore-size method %d", method);
    LBM_REQUIRE(ws_bytes >= diam_ws_bytes_n(n), LBM_E_NOMEM, "lbm_pore_diameter: workspace too small");
    st = check_device();
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Grid g = make_grid(n);
    const int64_t nv = g.nvox();
    const unsigned blocks = (unsigned)((nv + 255) / 256);
    Carver c(workspace);
    unsigned long long *counter = c.take<unsigned long long>(4);
    int32_t *a = c.take<int32_t>(nv);
    int32_t *b = c.take<int32_t>(nv);
    int32_t *cc = c.take<int32_t>(nv);
    double *width = c.take<double>(3 * (size_t)kMaxEdge * kMaxEdge + 1);
    if (method == LBM_PSD_CHORD13) {
        LBM_TRY_HIP(hipMemsetAsync(a, 0, nv * sizeof(int32_t), s));
        LBM_TRY_HIP(hipMemsetAsync(b, 0, nv * sizeof(int32_t), s));
        LBM_TRY_HIP(hipMemsetAsync(cc, 0, nv * sizeof(int32_t), s));
        const int64_t starts = (int64_t)g.ny * g.nz + (int64_t)g.nx * g.nz + (int64_t)g.nx * g.ny;
        for (int d = 0; d < 13; d++) {
            int32_t *dst = d < 3 ? a : (d < 9 ? b : cc);
            k_chords<<<(unsigned)((starts + 255) / 256), 256, 0, s>>>(g, d, pore, dst);
            LBM_CHECK_LAUNCH();
        }
        k_chord_final<<<blocks, 256, 0, s>>>(nv, pore, a, b, cc, std::sqrt(2.0), std::sqrt(3.0), diam);
        LBM_CHECK_LAUNCH();
        LBM_TRY_HIP(hipStreamSynchronize(s));
        return LBM_OK;
    }
    // maximum inscribed sphere
    int64_t n_pore = 0;
    st = count_nonzero(g, pore, counter, &n_pore, s);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(n_pore < nv, LBM_E_INVAL, "the domain holds no solid voxel: no distance map");
    if (n_pore == 0) {  // all solid: no pore width anywhere
        LBM_TRY_HIP(hipMemsetAsync(diam, 0, nv * sizeof(double), s));
        LBM_TRY_HIP(hipStreamSynchronize(s));
        return LBM_OK;
    }
    k_edt_x<<<(unsigned)(((int64_t)g.ny * g.nz + 255) / 256), 256, 0, s>>>(g, pore, a);
    LBM_CHECK_LAUNCH();
    k_edt_axis<<<blocks, 256, 0, s>>>(g, 1, a, b);
    LBM_CHECK_LAUNCH();
    k_edt_axis<<<blocks, 256, 0, s>>>(g, 2, b, a);
    LBM_CHECK_LAUNCH();
    int *dmax = reinterpret_cast<int *>(counter);
    LBM_TRY_HIP(hipMemsetAsync(dmax, 0, sizeof(int), s));
    k_max_i32<<<(unsigned)(blocks < 4096 ? blocks : 4096), 256, 0, s>>>(nv, a, pore, dmax);
    LBM_CHECK_LAUNCH();
    int emax = 0;
    LBM_TRY_HIP(hipMemcpyAsync(&emax, dmax, sizeof(int), hipMemcpyDeviceToHost, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    LBM_REQUIRE(emax >= 1 && (size_t)emax <= 3 * (size_t)kMaxEdge * kMaxEdge, LBM_E_DEVICE,
                "distance map maximum %d out of range", emax);
    std::vector<double> tab((size_t)emax + 1);
    for (int e = 0; e <= emax; e++) tab[e] = 2.0 * std::sqrt((double)e) - 1.0;
    LBM_TRY_HIP(hipMemcpyAsync(width, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s));
    int R = (int)std::ceil(std::sqrt((double)emax));
    k_mis<<<blocks, 256, 0, s>>>(g, R, emax, a, pore, width, diam);
    LBM_CHECK_LAUNCH();
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return LBM_OK;
}
