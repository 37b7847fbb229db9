// Layers of the warm-start U-Net: 3x3x3 convolution (forward, input gradient, weight
// gradient) as implicit GEMMs on the bf16 matrix cores, 2x2x2 mean pooling, nearest
// upsampling, the ReLU gradient, the 1x1x1 output head with its masked squared-error
// loss, Adam, and the conversions between the solver's fields and network tensors.
//
// Tensors are channels-last bf16: element (voxel v, channel c) at v * cs + c, with v =
// x + nx (y + ny z); a view is a pointer to its first channel plus the channel stride cs,
// so the [skip, upsampled] concatenation of a decoder input is two views of one buffer.
// Weights are [27][cout][cin], tap t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1); products
// accumulate in binary32.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <initializer_list>

#include "../../include/lbm_nn.h"
#include "lbm_internal.h"

namespace lbm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// binary32 -> bfloat16, round to nearest even (finite inputs)
__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// D = A B + C for 16x16 tiles, K = 16.  Lane l = 16 q + r holds A[m = r][k = 4q .. 4q+3],
// B[k = 4q .. 4q+3][n = r] and D[m = 4q .. 4q+3][n = r].
__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

struct NnGrid {
    int nx, ny, nz;
    int64_t nvox;
};

__device__ inline void tap_offset(int t, int flip, int &dx, int &dy, int &dz) {
    dz = t / 9 - 1;
    dy = (t / 3) % 3 - 1;
    dx = t % 3 - 1;
    if (flip) {
        dx = -dx;
        dy = -dy;
        dz = -dz;
    }
}

// y[v][c] = act(bias[c] + sum_t sum_k x[v + d_t][k] w[t][c][k]) for NB blocks of 16
// output channels; d_t negated with flip.  One wave per 16 consecutive voxels.
template <int NB>
__global__ __launch_bounds__(256) void k_conv3d(NnGrid g, const uint16_t *__restrict__ x, int x_cs,
                                                int cin, const uint16_t *__restrict__ w,
                                                const float *__restrict__ bias,
                                                uint16_t *__restrict__ y, int y_cs, int relu,
                                                int flip) {
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int64_t m0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (m0 >= g.nvox) return;  // uniform per wave; nvox is a multiple of 16
    const int64_t va = m0 + r;
    const int ax = (int)(va % g.nx), ay = (int)((va / g.nx) % g.ny), az = (int)(va / ((int64_t)g.nx * g.ny));
    const int cout = NB * 16;
    f32x4 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; nb++) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 27; t++) {
        int dx, dy, dz;
        tap_offset(t, flip, dx, dy, dz);
        const int sx = ax + dx, sy = ay + dy, sz = az + dz;
        const bool ok = sx >= 0 && sx < g.nx && sy >= 0 && sy < g.ny && sz >= 0 && sz < g.nz;
        const int64_t sv = ok ? ((int64_t)sz * g.ny + sy) * g.nx + sx : 0;
        const uint16_t *xp = x + sv * x_cs + 4 * q;
        const uint16_t *wp = w + ((int64_t)t * cout + r) * cin + 4 * q;
        for (int kc = 0; kc < cin; kc += 16) {
            const bf16x4 a = ok ? *reinterpret_cast<const bf16x4 *>(xp + kc) : bf16x4{0, 0, 0, 0};
#pragma unroll
            for (int nb = 0; nb < NB; nb++) {
                const bf16x4 b = *reinterpret_cast<const bf16x4 *>(wp + (int64_t)nb * 16 * cin + kc);
                acc[nb] = mfma16(a, b, acc[nb]);
            }
        }
    }
#pragma unroll
    for (int nb = 0; nb < NB; nb++) {
        const int c = nb * 16 + r;
        const float bc = bias ? bias[c] : 0.f;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            float v = acc[nb][j] + bc;
            if (relu) v = v > 0.f ? v : 0.f;
            y[(m0 + 4 * q + j) * y_cs + c] = f2bf(v);
        }
    }
}

// The same convolution on grids whose three sizes are multiples of 4: one wave per brick
// of 4 x 4 x 4 voxels (blockIdx.x, x fastest) and block of 16 output channels
// (blockIdx.y), the brick's four z planes of 16 voxels as four output tiles that share
// each weight load.  Per block of 16 input channels the wave copies the 6 x 6 x 6 halo of
// x around its brick (zero outside the grid) into LDS as loaded, voxel-major, and reads
// each tap's shifted operand from there.
__global__ __launch_bounds__(64) void k_conv3d_bricks(NnGrid g, const uint16_t *__restrict__ x, int x_cs,
                                                      int cin, const uint16_t *__restrict__ w,
                                                      int cout, const float *__restrict__ bias,
                                                      uint16_t *__restrict__ y, int y_cs, int relu,
                                                      int flip) {
    __shared__ __align__(16) uint16_t sx[216 * 16];  // [halo voxel][channel]
    const int lane = threadIdx.x, r = lane & 15, q = lane >> 4;
    const int bx = g.nx / 4, by = g.ny / 4;
    const int64_t b = blockIdx.x;
    const int nb = blockIdx.y;
    const int x0 = 4 * (int)(b % bx), y0 = 4 * (int)((b / bx) % by), z0 = 4 * (int)(b / ((int64_t)bx * by));
    f32x4 acc[4];
#pragma unroll
    for (int sp = 0; sp < 4; sp++) acc[sp] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < cin; kc += 16) {
        __syncthreads();  // the previous channel block's operands are read
        for (int h = lane; h < 216; h += 64) {
            const int sxv = x0 - 1 + h % 6, syv = y0 - 1 + (h / 6) % 6, szv = z0 - 1 + h / 36;
            uint4 lo = uint4{0u, 0u, 0u, 0u}, hi = uint4{0u, 0u, 0u, 0u};
            if (sxv >= 0 && sxv < g.nx && syv >= 0 && syv < g.ny && szv >= 0 && szv < g.nz) {
                const int64_t v = ((int64_t)szv * g.ny + syv) * g.nx + sxv;
                const uint4 *src = reinterpret_cast<const uint4 *>(x + v * x_cs + kc);
                lo = src[0];
                hi = src[1];
            }
            uint4 *dst = reinterpret_cast<uint4 *>(sx + h * 16);
            dst[0] = lo;
            dst[1] = hi;
        }
        __syncthreads();
        const uint16_t *wp = w + ((int64_t)nb * 16 + r) * cin + kc + 4 * q;
        for (int t = 0; t < 27; t++) {
            int dx, dy, dz;
            tap_offset(t, flip, dx, dy, dz);
            // B[k = 4 q .. 4 q + 3][n = r]: w[t][nb 16 + r][kc + 4 q ..]
            const bf16x4 bw = *reinterpret_cast<const bf16x4 *>(wp + (int64_t)t * cout * cin);
#pragma unroll
            for (int sp = 0; sp < 4; sp++) {
                // A[m = r][k = 4 q ..]: plane voxel r = (r & 3, r >> 2) of plane sp, shifted
                const int h = (1 + (r & 3) + dx) + 6 * (1 + (r >> 2) + dy) + 36 * (1 + sp + dz);
                const bf16x4 a = *reinterpret_cast<const bf16x4 *>(sx + h * 16 + 4 * q);
                acc[sp] = mfma16(a, bw, acc[sp]);
            }
        }
    }
    // D[m = 4 q + j][n = r]: plane voxel (j, q) of plane sp, output channel nb 16 + r
    const int c = nb * 16 + r;
    const float bc = bias ? bias[c] : 0.f;
#pragma unroll
    for (int sp = 0; sp < 4; sp++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            float v = acc[sp][j] + bc;
            if (relu) v = v > 0.f ? v : 0.f;
            const int64_t vox = ((int64_t)(z0 + sp) * g.ny + y0 + q) * g.nx + x0 + j;
            y[vox * y_cs + c] = f2bf(v);
        }
}

// Partial weight gradients over one chunk of voxels for tap t = blockIdx.y and output
// block cb = blockIdx.z: part[chunk][t][co][ci] = sum_v g[v][co] x[v + d_t][ci] for
// NBI blocks of 16 input channels; the centre tap also forms part_b[chunk][co] = sum_v
// g[v][co].  One wave per block.
template <int NBI>
__global__ __launch_bounds__(64) void k_conv3d_wgrad(NnGrid g, const uint16_t *__restrict__ x,
                                                     int x_cs, const uint16_t *__restrict__ gy,
                                                     int g_cs, int cout, int64_t chunk,
                                                     float *__restrict__ part,
                                                     float *__restrict__ part_b) {
    const int lane = threadIdx.x, r = lane & 15, q = lane >> 4;
    const int64_t ch = blockIdx.x;
    const int t = blockIdx.y, cb = blockIdx.z;
    const int cin = NBI * 16;
    int dx, dy, dz;
    tap_offset(t, 0, dx, dy, dz);
    const int64_t v_lo = ch * chunk, v_hi = v_lo + chunk < g.nvox ? v_lo + chunk : g.nvox;
    f32x4 acc[NBI];
#pragma unroll
    for (int ib = 0; ib < NBI; ib++) acc[ib] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 accb = f32x4{0.f, 0.f, 0.f, 0.f};
    const short one = (short)0x3f80;  // bfloat16 1.0
    const bf16x4 ones = bf16x4{one, one, one, one};
    for (int64_t v0 = v_lo; v0 < v_hi; v0 += 16) {
        bf16x4 a;
        int64_t src[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int64_t v = v0 + 4 * q + j;
            a[j] = (short)gy[v * g_cs + cb * 16 + r];
            const int vx = (int)(v % g.nx), vy = (int)((v / g.nx) % g.ny), vz = (int)(v / ((int64_t)g.nx * g.ny));
            const int sx = vx + dx, sy = vy + dy, sz = vz + dz;
            src[j] = sx >= 0 && sx < g.nx && sy >= 0 && sy < g.ny && sz >= 0 && sz < g.nz
                         ? ((int64_t)sz * g.ny + sy) * g.nx + sx
                         : -1;
        }
#pragma unroll
        for (int ib = 0; ib < NBI; ib++) {
            bf16x4 b;
#pragma unroll
            for (int j = 0; j < 4; j++) b[j] = src[j] >= 0 ? (short)x[src[j] * x_cs + ib * 16 + r] : (short)0;
            acc[ib] = mfma16(a, b, acc[ib]);
        }
        if (t == 13) accb = mfma16(a, ones, accb);
    }
#pragma unroll
    for (int ib = 0; ib < NBI; ib++)
#pragma unroll
        for (int j = 0; j < 4; j++)
            part[((ch * 27 + t) * cout + cb * 16 + 4 * q + j) * cin + ib * 16 + r] = acc[ib][j];
    if (t == 13 && r == 0)
#pragma unroll
        for (int j = 0; j < 4; j++) part_b[ch * cout + cb * 16 + 4 * q + j] = accb[j];
}

// The same weight gradient on grids whose three sizes are multiples of 4, with its
// operands staged in LDS.  The voxels go in bricks of 4 x 4 x 4 (x fastest inside a
// brick); one matrix-core step takes K = 16 voxels, one z plane of a brick.  A wave owns
// one chunk of bricks (blockIdx.x), one block of 16 output channels and one of 16 input
// channels (blockIdx.y), and all 27 taps: per brick it copies the brick's gy (64 voxels x
// 16 channels) and the 6 x 6 x 6 halo of x around it (zero outside the grid) into LDS as
// loaded, voxel-major, and reads each operand across voxels from there, so every tap
// reuses one load of gy and one of x.  Partial sums as in k_conv3d_wgrad.
__global__ __launch_bounds__(64) void k_conv3d_wgrad_bricks(NnGrid g, const uint16_t *__restrict__ x,
                                                            int x_cs, int cin,
                                                            const uint16_t *__restrict__ gy,
                                                            int g_cs, int cout, int64_t bricks,
                                                            float *__restrict__ part,
                                                            float *__restrict__ part_b) {
    __shared__ __align__(16) uint16_t sg[64 * 16];   // [brick voxel][channel]
    __shared__ __align__(16) uint16_t sx[216 * 16];  // [halo voxel][channel]
    const int lane = threadIdx.x, r = lane & 15, q = lane >> 4;
    const int64_t ch = blockIdx.x;
    const int ncb = cout / 16;
    const int cb = (int)blockIdx.y % ncb, ib = (int)blockIdx.y / ncb;
    const int bx = g.nx / 4, by = g.ny / 4, bz = g.nz / 4;
    const int64_t nb = (int64_t)bx * by * bz;
    const int64_t b_lo = ch * bricks;
    const int64_t b_hi = b_lo + bricks < nb ? b_lo + bricks : nb;
    const bool want_b = ib == 0;
    f32x4 acc[27];
#pragma unroll
    for (int t = 0; t < 27; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    f32x4 accb = f32x4{0.f, 0.f, 0.f, 0.f};
    const short one = (short)0x3f80;  // bfloat16 1.0
    const bf16x4 ones = bf16x4{one, one, one, one};
    for (int64_t b = b_lo; b < b_hi; b++) {
        const int x0 = 4 * (int)(b % bx), y0 = 4 * (int)((b / bx) % by), z0 = 4 * (int)(b / ((int64_t)bx * by));
        __syncthreads();  // the previous brick's operands are read
        {
            // lane k copies brick voxel k = x + 4 y + 16 z: 16 channels, 32 bytes
            const int64_t v = ((int64_t)(z0 + (lane >> 4)) * g.ny + y0 + ((lane >> 2) & 3)) * g.nx +
                              x0 + (lane & 3);
            const uint4 *src = reinterpret_cast<const uint4 *>(gy + v * g_cs + cb * 16);
            uint4 *dst = reinterpret_cast<uint4 *>(sg + lane * 16);
            dst[0] = src[0];
            dst[1] = src[1];
        }
        for (int h = lane; h < 216; h += 64) {
            const int sxv = x0 - 1 + h % 6, syv = y0 - 1 + (h / 6) % 6, szv = z0 - 1 + h / 36;
            uint4 lo = uint4{0u, 0u, 0u, 0u}, hi = uint4{0u, 0u, 0u, 0u};
            if (sxv >= 0 && sxv < g.nx && syv >= 0 && syv < g.ny && szv >= 0 && szv < g.nz) {
                const int64_t v = ((int64_t)szv * g.ny + syv) * g.nx + sxv;
                const uint4 *src = reinterpret_cast<const uint4 *>(x + v * x_cs + ib * 16);
                lo = src[0];
                hi = src[1];
            }
            uint4 *dst = reinterpret_cast<uint4 *>(sx + h * 16);
            dst[0] = lo;
            dst[1] = hi;
        }
        __syncthreads();
        // A[m = output channel r][k = 4 q + j] = gy at brick voxel (j, q, s) of plane s
        bf16x4 a[4];
#pragma unroll
        for (int sp = 0; sp < 4; sp++)
#pragma unroll
            for (int j = 0; j < 4; j++) a[sp][j] = (short)sg[(16 * sp + 4 * q + j) * 16 + r];
        if (want_b)
#pragma unroll
            for (int sp = 0; sp < 4; sp++) accb = mfma16(a[sp], ones, accb);
#pragma unroll
        for (int t = 0; t < 27; t++) {
            const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
#pragma unroll
            for (int sp = 0; sp < 4; sp++) {
                // B[k = 4 q + j][n = input channel r] = x at that voxel + (dx, dy, dz)
                bf16x4 bv;
                const int h0 = (1 + dx) + 6 * (q + 1 + dy) + 36 * (sp + 1 + dz);
#pragma unroll
                for (int j = 0; j < 4; j++) bv[j] = (short)sx[(h0 + j) * 16 + r];
                acc[t] = mfma16(a[sp], bv, acc[t]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 27; t++)
#pragma unroll
        for (int j = 0; j < 4; j++)
            part[((ch * 27 + t) * cout + cb * 16 + 4 * q + j) * cin + ib * 16 + r] = acc[t][j];
    if (want_b && r == 0)
#pragma unroll
        for (int j = 0; j < 4; j++) part_b[ch * cout + cb * 16 + 4 * q + j] = accb[j];
}

// out[i] (+)= sum_c part[c * count + i] over c = 0 .. nparts - 1 in a fixed order: 16
// threads per output each sum one contiguous sixteenth of the partials in order, then
// the sixteen sums are added in order (256 threads: 16 outputs x 16 groups).
__global__ __launch_bounds__(256) void k_sum_parts(const float *__restrict__ part, int64_t nparts,
                                                   int64_t count, float *__restrict__ out,
                                                   int accumulate) {
    __shared__ float lds[16][17];
    const int o = threadIdx.x & 15, gr = threadIdx.x >> 4;
    const int64_t i = (int64_t)blockIdx.x * 16 + o;
    const int64_t per = (nparts + 15) / 16;
    const int64_t c0 = gr * per, c1 = c0 + per < nparts ? c0 + per : nparts;
    float s = 0.f;
    if (i < count)
        for (int64_t c = c0; c < c1; c++) s += part[c * count + i];
    lds[gr][o] = s;
    __syncthreads();
    if (gr == 0 && i < count) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < 16; k++) t += lds[k][o];
        out[i] = accumulate ? out[i] + t : t;
    }
}

// wt[t][ci][co] = w[t][co][ci] (bf16), the weights of the input-gradient convolution.
__global__ __launch_bounds__(256) void k_transpose_w(const uint16_t *__restrict__ w, int cout,
                                                     int cin, uint16_t *__restrict__ wt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)27 * cout * cin;
    if (i >= n) return;
    const int64_t t = i / ((int64_t)cout * cin), rem = i % ((int64_t)cout * cin);
    const int co = (int)(rem / cin), ci = (int)(rem % cin);
    wt[(t * cin + ci) * cout + co] = w[i];
}

// The elementwise layers take V consecutive channels per thread: V = 4 (one 8-byte
// access) when the channel count, the strides and the pointers allow it, else V = 1.
template <int V>
__device__ inline void ldv(const uint16_t *p, uint16_t (&o)[V]) {
    if constexpr (V == 4) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        o[0] = (uint16_t)(u.x & 0xffffu); o[1] = (uint16_t)(u.x >> 16);
        o[2] = (uint16_t)(u.y & 0xffffu); o[3] = (uint16_t)(u.y >> 16);
    } else {
#pragma unroll
        for (int k = 0; k < V; k++) o[k] = p[k];
    }
}
template <int V>
__device__ inline void stv(uint16_t *p, const uint16_t (&o)[V]) {
    if constexpr (V == 4) {
        uint2 u;
        u.x = (uint32_t)o[0] | ((uint32_t)o[1] << 16);
        u.y = (uint32_t)o[2] | ((uint32_t)o[3] << 16);
        *reinterpret_cast<uint2 *>(p) = u;
    } else {
#pragma unroll
        for (int k = 0; k < V; k++) p[k] = o[k];
    }
}

// 2x2x2 mean of the fine grid n (even sizes) onto the coarse grid.
template <int V>
__global__ __launch_bounds__(256) void k_pool2(NnGrid f, int c, const uint16_t *__restrict__ x,
                                               int x_cs, uint16_t *__restrict__ y, int y_cs,
                                               int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int cx = f.nx / 2, cy = f.ny / 2, cz = f.nz / 2;
    const int64_t ncv = (int64_t)cx * cy * cz;
    const int cv = c / V;
    if (i >= ncv * cv) return;
    const int64_t v = i / cv;
    const int ch = (int)(i % cv) * V;
    const int X = (int)(v % cx), Y = (int)((v / cx) % cy), Z = (int)(v / ((int64_t)cx * cy));
    float s[V];
#pragma unroll
    for (int k = 0; k < V; k++) s[k] = 0.f;
    for (int m = 0; m < 8; m++) {
        const int64_t fv = ((int64_t)(2 * Z + (m >> 2)) * f.ny + 2 * Y + ((m >> 1) & 1)) * f.nx + 2 * X + (m & 1);
        uint16_t e[V];
        ldv<V>(x + fv * x_cs + ch, e);
#pragma unroll
        for (int k = 0; k < V; k++) s[k] += bf2f(e[k]);
    }
    uint16_t o[V];
    if (accumulate) ldv<V>(y + v * y_cs + ch, o);
#pragma unroll
    for (int k = 0; k < V; k++) {
        float t = s[k] * 0.125f;
        if (accumulate) t += bf2f(o[k]);
        o[k] = f2bf(t);
    }
    stv<V>(y + v * y_cs + ch, o);
}

// Adjoint of the mean pooling: each fine voxel gets 1/8 of its parent's gradient.
template <int V>
__global__ __launch_bounds__(256) void k_pool2_bwd(NnGrid f, int c, const uint16_t *__restrict__ gy,
                                                   int gy_cs, uint16_t *__restrict__ gx, int gx_cs,
                                                   int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int cv = c / V;
    if (i >= f.nvox * cv) return;
    const int64_t v = i / cv;
    const int ch = (int)(i % cv) * V;
    const int x = (int)(v % f.nx), y = (int)((v / f.nx) % f.ny), z = (int)(v / ((int64_t)f.nx * f.ny));
    const int64_t pv = ((int64_t)(z / 2) * (f.ny / 2) + y / 2) * (f.nx / 2) + x / 2;
    uint16_t e[V], o[V];
    ldv<V>(gy + pv * gy_cs + ch, e);
    if (accumulate) ldv<V>(gx + v * gx_cs + ch, o);
#pragma unroll
    for (int k = 0; k < V; k++) {
        float t = 0.125f * bf2f(e[k]);
        if (accumulate) t += bf2f(o[k]);
        o[k] = f2bf(t);
    }
    stv<V>(gx + v * gx_cs + ch, o);
}

// Nearest upsampling from the coarse grid to the fine grid f (each fine voxel copies its
// parent), and its adjoint (each parent sums its 8 children).
template <int V>
__global__ __launch_bounds__(256) void k_up2(NnGrid f, int c, const uint16_t *__restrict__ x,
                                             int x_cs, uint16_t *__restrict__ y, int y_cs) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int cv = c / V;
    if (i >= f.nvox * cv) return;
    const int64_t v = i / cv;
    const int ch = (int)(i % cv) * V;
    const int xx = (int)(v % f.nx), yy = (int)((v / f.nx) % f.ny), zz = (int)(v / ((int64_t)f.nx * f.ny));
    const int64_t pv = ((int64_t)(zz / 2) * (f.ny / 2) + yy / 2) * (f.nx / 2) + xx / 2;
    uint16_t e[V];
    ldv<V>(x + pv * x_cs + ch, e);
    stv<V>(y + v * y_cs + ch, e);
}

template <int V>
__global__ __launch_bounds__(256) void k_up2_bwd(NnGrid f, int c, const uint16_t *__restrict__ gy,
                                                 int gy_cs, uint16_t *__restrict__ gx, int gx_cs) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int cx = f.nx / 2, cy = f.ny / 2, cz = f.nz / 2;
    const int cv = c / V;
    if (i >= (int64_t)cx * cy * cz * cv) return;
    const int64_t v = i / cv;
    const int ch = (int)(i % cv) * V;
    const int X = (int)(v % cx), Y = (int)((v / cx) % cy), Z = (int)(v / ((int64_t)cx * cy));
    float s[V];
#pragma unroll
    for (int k = 0; k < V; k++) s[k] = 0.f;
    for (int m = 0; m < 8; m++) {
        const int64_t fv = ((int64_t)(2 * Z + (m >> 2)) * f.ny + 2 * Y + ((m >> 1) & 1)) * f.nx + 2 * X + (m & 1);
        uint16_t e[V];
        ldv<V>(gy + fv * gy_cs + ch, e);
#pragma unroll
        for (int k = 0; k < V; k++) s[k] += bf2f(e[k]);
    }
    uint16_t o[V];
#pragma unroll
    for (int k = 0; k < V; k++) o[k] = f2bf(s[k]);
    stv<V>(gx + v * gx_cs + ch, o);
}

// g = gy where the layer's output y > 0, else 0 (the ReLU gradient).
template <int V>
__global__ __launch_bounds__(256) void k_relu_bwd(int64_t nvox, int c, const uint16_t *__restrict__ y,
                                                  int y_cs, const uint16_t *__restrict__ gy,
                                                  int gy_cs, uint16_t *__restrict__ gout, int g_cs) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int cv = c / V;
    if (i >= nvox * cv) return;
    const int64_t v = i / cv;
    const int ch = (int)(i % cv) * V;
    uint16_t yv[V], gv[V], o[V];
    ldv<V>(y + v * y_cs + ch, yv);
    ldv<V>(gy + v * gy_cs + ch, gv);
    // positive bfloat16: sign bit clear and not zero
#pragma unroll
    for (int k = 0; k < V; k++) o[k] = (yv[k] != 0 && !(yv[k] & 0x8000u)) ? gv[k] : (uint16_t)0;
    stv<V>(gout + v * g_cs + ch, o);
}

// 8-byte channel groups for c channels at the given strides and pointers
static bool vec4(int c, std::initializer_list<int> cs, std::initializer_list<const void *> ptrs) {
    if (c % 4) return false;
    for (int s : cs)
        if (s % 4) return false;
    for (const void *p : ptrs)
        if (reinterpret_cast<uintptr_t>(p) % 8) return false;
    return true;
}

constexpr int kHeadMaxOut = 8;
constexpr int kHeadCin = 16;

// The 1x1x1 head: out[o][v] = bh[o] + sum_c wh[o][c] x[v][c] (binary32, planar).  With a
// target: go[o][v] = 2 wt[o] mask[v] (out - target) / n_mask (the gradient of the loss
// sum_o wt[o] mask (out - target)^2 / n_mask), gx = wh^T go (bf16) and the per-block
// partial sums of the loss.
__global__ __launch_bounds__(256) void k_head(int64_t nvox, const uint16_t *__restrict__ x, int x_cs,
                                              int no, const float *__restrict__ wh,
                                              const float *__restrict__ bh,
                                              float *__restrict__ out,
                                              const float *__restrict__ target,
                                              const uint8_t *__restrict__ mask,
                                              const float *__restrict__ wt, double inv_n,
                                              float *__restrict__ gout, uint16_t *__restrict__ gx,
                                              int gx_cs, double *__restrict__ loss_part) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double loss = 0.0;
    if (v < nvox) {
        float xv[kHeadCin];
#pragma unroll
        for (int c = 0; c < kHeadCin; c++) xv[c] = bf2f(x[v * x_cs + c]);
        float go[kHeadMaxOut];
        for (int o = 0; o < no; o++) {
            float s = bh[o];
#pragma unroll
            for (int c = 0; c < kHeadCin; c++) s += wh[o * kHeadCin + c] * xv[c];
            if (out) out[o * nvox + v] = s;
            go[o] = 0.f;
            if (target && mask[v]) {
                const double d = (double)s - (double)target[o * nvox + v];
                loss += (double)wt[o] * d * d * inv_n;
                go[o] = (float)(2.0 * (double)wt[o] * d * inv_n);
            }
            if (target) gout[o * nvox + v] = go[o];
        }
        if (target && gx) {
#pragma unroll
            for (int c = 0; c < kHeadCin; c++) {
                float s = 0.f;
                for (int o = 0; o < no; o++) s += wh[o * kHeadCin + c] * go[o];
                gx[v * gx_cs + c] = f2bf(s);
            }
        }
    }
    if (!target) return;
    __shared__ double lds[4];
    for (int off = 32; off > 0; off >>= 1) loss += __shfl_down(loss, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = loss;
    __syncthreads();
    if (threadIdx.x == 0) loss_part[blockIdx.x] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// Per-chunk partial gradients of the head weights for output o = blockIdx.y:
// part[chunk][o][c] = sum_v go[o][v] x[v][c] (c < 16) and part[chunk][o][16] = sum_v go.
__global__ __launch_bounds__(256) void k_head_wgrad(int64_t nvox, const uint16_t *__restrict__ x,
                                                    int x_cs, const float *__restrict__ gout,
                                                    int64_t chunk, double *__restrict__ part) {
    constexpr int NV = kHeadCin + 1;
    const int o = blockIdx.y;
    const int64_t lo = (int64_t)blockIdx.x * chunk, hi = lo + chunk < nvox ? lo + chunk : nvox;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) acc[k] = 0.0;
    for (int64_t v = lo + threadIdx.x; v < hi; v += 256) {
        const double go = gout[o * nvox + v];
#pragma unroll
        for (int c = 0; c < kHeadCin; c++) acc[c] += go * (double)bf2f(x[v * x_cs + c]);
        acc[kHeadCin] += go;
    }
    __shared__ double lds[4][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        double a = acc[k];
        for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
        if (lane == 0) lds[wave][k] = a;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        const int k = threadIdx.x;
        part[((int64_t)blockIdx.x * gridDim.y + o) * NV + k] = ((lds[0][k] + lds[1][k]) + lds[2][k]) + lds[3][k];
    }
}

// Fixed-order sums: the loss (each thread one contiguous 1/256 of the block partials in
// order, then the 256 sums in order), gwh[o][c] and gbh[o].
__global__ __launch_bounds__(256) void k_head_final(const double *__restrict__ loss_part, int64_t nb,
                                                    const double *__restrict__ part, int64_t nch,
                                                    int no, double *__restrict__ loss,
                                                    float *__restrict__ gwh, float *__restrict__ gbh) {
    constexpr int NV = kHeadCin + 1;
    __shared__ double lds[256];
    const int k = threadIdx.x;
    if (k < no * NV) {
        double s = 0.0;
        for (int64_t c = 0; c < nch; c++) s += part[c * no * NV + k];
        const int o = k / NV, c = k % NV;
        if (c < kHeadCin) gwh[o * kHeadCin + c] = (float)s;
        else gbh[o] = (float)s;
    }
    const int64_t per = (nb + 255) / 256, b0 = k * per, b1 = b0 + per < nb ? b0 + per : nb;
    double s = 0.0;
    for (int64_t b = b0; b < b1; b++) s += loss_part[b];
    lds[k] = s;
    __syncthreads();
    if (k == 0) {
        double t = 0.0;
        for (int i = 0; i < 256; i++) t += lds[i];
        *loss = t;
    }
}

// One Adam step (bias-corrected), binary32 master weights; refreshes their bf16 copy.
__global__ __launch_bounds__(256) void k_adam(int64_t n, float *__restrict__ w,
                                              const float *__restrict__ g, float *__restrict__ m,
                                              float *__restrict__ v, uint16_t *__restrict__ wb,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
}

__global__ __launch_bounds__(256) void k_to_bf16(int64_t n, const float *__restrict__ src,
                                                 uint16_t *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = f2bf(src[i]);
}

// The network input: channel 0 the pore mask, channel 1 the pore diameter / d_scale,
// channels 2 .. cs - 1 zero.
__global__ __launch_bounds__(256) void k_make_input(int64_t nvox, const uint8_t *__restrict__ mask,
                                                    const double *__restrict__ diam,
                                                    double inv_scale, uint16_t *__restrict__ x,
                                                    int cs) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nvox) return;
    for (int c = 0; c < cs; c++) {
        float val = 0.f;
        if (c == 0) val = mask[v] ? 1.f : 0.f;
        else if (c == 1) val = (float)(diam[v] * inv_scale);
        x[v * cs + c] = f2bf(val);
    }
}

// fields[k][v] = mask[v] ? out[k][v] * scale[k] : 0.
__global__ __launch_bounds__(256) void k_to_fields(int64_t nvox, int nk, const float *__restrict__ out,
                                                   const uint8_t *__restrict__ mask,
                                                   const float *__restrict__ scale,
                                                   float *__restrict__ fields) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= nvox * nk) return;
    const int64_t v = i % nvox;
    const int k = (int)(i / nvox);
    fields[i] = mask[v] ? out[i] * scale[k] : 0.f;
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

static lbm_status check_grid(const int32_t n[3], NnGrid &g) {
    LBM_REQUIRE(n && n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && n[0] <= 4096 && n[1] <= 4096 &&
                    n[2] <= 4096,
                LBM_E_INVAL, "network grid sizes must lie in [1, 4096]");
    g.nx = n[0];
    g.ny = n[1];
    g.nz = n[2];
    g.nvox = (int64_t)n[0] * n[1] * n[2];
    return LBM_OK;
}

static bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

static int64_t wgrad_chunk(int64_t nvox) {
    int64_t nch = nvox / 1024;
    if (nch < 1) nch = 1;
    if (nch > 1024) nch = 1024;
    int64_t chunk = (nvox + nch - 1) / nch;
    return (chunk + 15) / 16 * 16;
}

}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_nn_conv3d(const int32_t n[3], const uint16_t *x, int32_t x_cs, int32_t cin,
                                    const uint16_t *w, const float *bias, uint16_t *y, int32_t y_cs,
                                    int32_t cout, int32_t flags, void *stream) {
    NnGrid g;
    lbm_status st = check_grid(n, g);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(x && w && y, LBM_E_INVAL, "lbm_nn_conv3d: null tensor");
    LBM_REQUIRE(g.nvox % 16 == 0, LBM_E_INVAL, "lbm_nn_conv3d: voxel count must be a multiple of 16");
    LBM_REQUIRE(cin >= 16 && cin % 16 == 0 && cin <= x_cs && x_cs % 4 == 0, LBM_E_INVAL,
                "lbm_nn_conv3d: cin must be a positive multiple of 16 within the stride %d", x_cs);
    LBM_REQUIRE(cout <= y_cs && aligned8(x) && aligned8(w), LBM_E_INVAL,
                "lbm_nn_conv3d: cout beyond the output stride, or a misaligned tensor");
    LBM_REQUIRE((flags & ~(LBM_NN_RELU | LBM_NN_FLIP)) == 0, LBM_E_INVAL, "lbm_nn_conv3d: flags");
    st = check_device();
    if (st != LBM_OK) return st;
    const unsigned grid = (unsigned)((g.nvox / 16 + 3) / 4);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int relu = (flags & LBM_NN_RELU) != 0, flip = (flags & LBM_NN_FLIP) != 0;
    // bricks: grid sizes multiples of 4 and 16-byte input rows (the halo is copied as
    // 16-byte vectors)
    if (g.nx % 4 == 0 && g.ny % 4 == 0 && g.nz % 4 == 0 && x_cs % 8 == 0 &&
        reinterpret_cast<uintptr_t>(x) % 16 == 0) {
        LBM_REQUIRE(cout == 16 || cout == 32 || cout == 48 || cout == 64 || cout == 96 ||
                        cout == 128 || cout == 192,
                    LBM_E_INVAL, "lbm_nn_conv3d: cout %d not supported", cout);
        k_conv3d_bricks<<<dim3((unsigned)(g.nvox / 64), (unsigned)(cout / 16)), 64, 0, s>>>(
            g, x, x_cs, cin, w, cout, bias, y, y_cs, relu, flip);
        LBM_CHECK_LAUNCH();
        return LBM_OK;
    }
    switch (cout) {
    case 16: k_conv3d<1><<<grid, 256, 0, s>>>(g, x, x_cs, cin, w, bias, y, y_cs, relu, flip); break;
    case 32: k_conv3d<2><<<grid, 256, 0, s>>>(g, x, x_cs, cin, w, bias, y, y_cs, relu, flip); break;
    case 48: k_conv3d<3><<<grid, 256, 0, s>>>(g, x, x_cs, cin, w, bias, y, y_cs, relu, flip); break;
    case 64: k_conv3d<4><<<grid, 256, 0, s>>>(g, x, x_cs, cin, w, bias, y, y_cs, relu, flip); break;
    case 96: k_conv3d<6><<<grid, 256, 0, s>>>(g, x, x_cs, cin, w, bias, y, y_cs, relu, flip); break;
    case 128: k_conv3d<8><<<grid, 256, 0, s>>>(g, x, x_cs, cin, w, bias, y, y_cs, relu, flip); break;
    case 192: k_conv3d<12><<<grid, 256, 0, s>>>(g, x, x_cs, cin, w, bias, y, y_cs, relu, flip); break;
    default: set_error("lbm_nn_conv3d: cout %d not supported", cout); return LBM_E_INVAL;
    }
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" size_t lbm_nn_wgrad_workspace(const int32_t n[3], int32_t cin, int32_t cout) {
    if (!n || n[0] < 1 || n[1] < 1 || n[2] < 1 || cin < 1 || cout < 1) return 0;
    const int64_t nvox = (int64_t)n[0] * n[1] * n[2];
    const int64_t nch = (nvox + wgrad_chunk(nvox) - 1) / wgrad_chunk(nvox);
    return (size_t)nch * ((size_t)27 * cout * cin + cout) * sizeof(float) + 256;
}

extern "C" lbm_status lbm_nn_conv3d_wgrad(const int32_t n[3], const uint16_t *x, int32_t x_cs,
                                          int32_t cin, const uint16_t *gy, int32_t g_cs,
                                          int32_t cout, float *dw, float *db, int32_t accumulate,
                                          void *workspace, size_t ws_bytes, void *stream) {
    NnGrid g;
    lbm_status st = check_grid(n, g);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(x && gy && dw && workspace, LBM_E_INVAL, "lbm_nn_conv3d_wgrad: null argument");
    LBM_REQUIRE(g.nvox % 16 == 0, LBM_E_INVAL, "lbm_nn_conv3d_wgrad: voxel count must be a multiple of 16");
    LBM_REQUIRE(cin % 16 == 0 && cin >= 16 && cin <= x_cs && cout % 16 == 0 && cout >= 16 &&
                    cout <= g_cs,
                LBM_E_INVAL, "lbm_nn_conv3d_wgrad: channel counts must be multiples of 16 within the strides");
    LBM_REQUIRE(ws_bytes >= lbm_nn_wgrad_workspace(n, cin, cout), LBM_E_NOMEM,
                "lbm_nn_conv3d_wgrad: workspace below %zu bytes", lbm_nn_wgrad_workspace(n, cin, cout));
    st = check_device();
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t chunk = wgrad_chunk(g.nvox);
    int64_t nch = (g.nvox + chunk - 1) / chunk;  // the workspace's partial rows
    float *part = static_cast<float *>(workspace);
    float *part_b = part + nch * 27 * (int64_t)cout * cin;
    // the brick kernel copies 16-channel rows as 16-byte vectors: aligned rows only
    const bool rows16 = x_cs % 8 == 0 && g_cs % 8 == 0 && reinterpret_cast<uintptr_t>(x) % 16 == 0 &&
                        reinterpret_cast<uintptr_t>(gy) % 16 == 0;
    if (g.nx % 4 == 0 && g.ny % 4 == 0 && g.nz % 4 == 0 && rows16) {
        // bricks of 64 voxels, as many per chunk as the chunk has voxels (rounded up):
        // at most nch chunks
        const int64_t nb = g.nvox / 64, bricks = (chunk + 63) / 64;
        const int64_t nbc = (nb + bricks - 1) / bricks;
        k_conv3d_wgrad_bricks<<<dim3((unsigned)nbc, (unsigned)((cout / 16) * (cin / 16))), 64, 0, s>>>(
            g, x, x_cs, cin, gy, g_cs, cout, bricks, part, part_b);
        LBM_CHECK_LAUNCH();
        nch = nbc;
    } else {
    const dim3 grid((unsigned)nch, 27, (unsigned)(cout / 16));
    switch (cin) {
    case 16: k_conv3d_wgrad<1><<<grid, 64, 0, s>>>(g, x, x_cs, gy, g_cs, cout, chunk, part, part_b); break;
    case 32: k_conv3d_wgrad<2><<<grid, 64, 0, s>>>(g, x, x_cs, gy, g_cs, cout, chunk, part, part_b); break;
    case 48: k_conv3d_wgrad<3><<<grid, 64, 0, s>>>(g, x, x_cs, gy, g_cs, cout, chunk, part, part_b); break;
    case 64: k_conv3d_wgrad<4><<<grid, 64, 0, s>>>(g, x, x_cs, gy, g_cs, cout, chunk, part, part_b); break;
    case 96: k_conv3d_wgrad<6><<<grid, 64, 0, s>>>(g, x, x_cs, gy, g_cs, cout, chunk, part, part_b); break;
    case 128: k_conv3d_wgrad<8><<<grid, 64, 0, s>>>(g, x, x_cs, gy, g_cs, cout, chunk, part, part_b); break;
    case 192: k_conv3d_wgrad<12><<<grid, 64, 0, s>>>(g, x, x_cs, gy, g_cs, cout, chunk, part, part_b); break;
    default: set_error("lbm_nn_conv3d_wgrad: cin %d not supported", cin); return LBM_E_INVAL;
    }
    LBM_CHECK_LAUNCH();
    }
    const int64_t count = (int64_t)27 * cout * cin;
    k_sum_parts<<<(unsigned)((count + 15) / 16), 256, 0, s>>>(part, nch, count, dw, accumulate);
    LBM_CHECK_LAUNCH();
    if (db) {
        k_sum_parts<<<(unsigned)((cout + 15) / 16), 256, 0, s>>>(part_b, nch, cout, db, accumulate);
        LBM_CHECK_LAUNCH();
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_transpose_weights(const uint16_t *w, int32_t cout, int32_t cin,
                                               uint16_t *wt, void *stream) {
    LBM_REQUIRE(w && wt && cout >= 1 && cin >= 1, LBM_E_INVAL, "lbm_nn_transpose_weights: arguments");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    const int64_t n = (int64_t)27 * cout * cin;
    k_transpose_w<<<nblk(n), 256, 0, static_cast<hipStream_t>(stream)>>>(w, cout, cin, wt);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

static lbm_status pool_args(const int32_t n[3], int32_t c, const void *a, int32_t a_cs,
                            const void *b, int32_t b_cs, NnGrid &g) {
    lbm_status st = check_grid(n, g);
    if (st != LBM_OK) return st;
    LBM_REQUIRE(a && b && c >= 1 && c <= a_cs && c <= b_cs, LBM_E_INVAL,
                "pooling: null tensor or channel count beyond a stride");
    LBM_REQUIRE(n[0] % 2 == 0 && n[1] % 2 == 0 && n[2] % 2 == 0, LBM_E_INVAL,
                "pooling: the fine grid must have even sizes");
    return check_device();
}

extern "C" lbm_status lbm_nn_pool2(const int32_t n_fine[3], int32_t c, const uint16_t *x, int32_t x_cs,
                                   uint16_t *y, int32_t y_cs, int32_t accumulate, void *stream) {
    NnGrid g;
    lbm_status st = pool_args(n_fine, c, x, x_cs, y, y_cs, g);
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (vec4(c, {x_cs, y_cs}, {x, y}))
        k_pool2<4><<<nblk(g.nvox / 8 * (c / 4)), 256, 0, s>>>(g, c, x, x_cs, y, y_cs, accumulate);
    else
        k_pool2<1><<<nblk(g.nvox / 8 * c), 256, 0, s>>>(g, c, x, x_cs, y, y_cs, accumulate);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_pool2_bwd(const int32_t n_fine[3], int32_t c, const uint16_t *gy,
                                       int32_t gy_cs, uint16_t *gx, int32_t gx_cs, int32_t accumulate,
                                       void *stream) {
    NnGrid g;
    lbm_status st = pool_args(n_fine, c, gy, gy_cs, gx, gx_cs, g);
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (vec4(c, {gy_cs, gx_cs}, {gy, gx}))
        k_pool2_bwd<4><<<nblk(g.nvox * (c / 4)), 256, 0, s>>>(g, c, gy, gy_cs, gx, gx_cs, accumulate);
    else
        k_pool2_bwd<1><<<nblk(g.nvox * c), 256, 0, s>>>(g, c, gy, gy_cs, gx, gx_cs, accumulate);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_up2(const int32_t n_fine[3], int32_t c, const uint16_t *x, int32_t x_cs,
                                 uint16_t *y, int32_t y_cs, void *stream) {
    NnGrid g;
    lbm_status st = pool_args(n_fine, c, x, x_cs, y, y_cs, g);
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (vec4(c, {x_cs, y_cs}, {x, y}))
        k_up2<4><<<nblk(g.nvox * (c / 4)), 256, 0, s>>>(g, c, x, x_cs, y, y_cs);
    else
        k_up2<1><<<nblk(g.nvox * c), 256, 0, s>>>(g, c, x, x_cs, y, y_cs);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_up2_bwd(const int32_t n_fine[3], int32_t c, const uint16_t *gy,
                                     int32_t gy_cs, uint16_t *gx, int32_t gx_cs, void *stream) {
    NnGrid g;
    lbm_status st = pool_args(n_fine, c, gy, gy_cs, gx, gx_cs, g);
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (vec4(c, {gy_cs, gx_cs}, {gy, gx}))
        k_up2_bwd<4><<<nblk(g.nvox / 8 * (c / 4)), 256, 0, s>>>(g, c, gy, gy_cs, gx, gx_cs);
    else
        k_up2_bwd<1><<<nblk(g.nvox / 8 * c), 256, 0, s>>>(g, c, gy, gy_cs, gx, gx_cs);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_relu_bwd(int64_t nvox, int32_t c, const uint16_t *y, int32_t y_cs,
                                      const uint16_t *gy, int32_t gy_cs, uint16_t *g, int32_t g_cs,
                                      void *stream) {
    LBM_REQUIRE(nvox >= 0 && y && gy && g && c >= 1 && c <= y_cs && c <= gy_cs && c <= g_cs,
                LBM_E_INVAL, "lbm_nn_relu_bwd: arguments");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    if (nvox == 0) return LBM_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (vec4(c, {y_cs, gy_cs, g_cs}, {y, gy, g}))
        k_relu_bwd<4><<<nblk(nvox * (c / 4)), 256, 0, s>>>(nvox, c, y, y_cs, gy, gy_cs, g, g_cs);
    else
        k_relu_bwd<1><<<nblk(nvox * c), 256, 0, s>>>(nvox, c, y, y_cs, gy, gy_cs, g, g_cs);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

static int64_t head_chunk(int64_t nvox) {
    int64_t nch = nvox / 8192;
    if (nch < 1) nch = 1;
    if (nch > 256) nch = 256;
    return (nvox + nch - 1) / nch;
}

extern "C" size_t lbm_nn_head_workspace(int64_t nvox, int32_t no) {
    if (nvox < 1 || no < 1) return 0;
    const int64_t nb = (nvox + 255) / 256, chunk = head_chunk(nvox), nch = (nvox + chunk - 1) / chunk;
    Carver c(nullptr);
    c.take<double>(nb);
    c.take<double>(nch * no * (kHeadCin + 1));
    c.take<double>(1);
    c.take<float>(nvox * no);
    return c.off + 256;
}

extern "C" lbm_status lbm_nn_head(int64_t nvox, const uint16_t *x, int32_t x_cs, int32_t no,
                                  const float *wh, const float *bh, float *out, const float *target,
                                  const uint8_t *mask, const float *wt, double n_mask, uint16_t *gx,
                                  int32_t gx_cs, float *gwh, float *gbh, double *loss_h,
                                  void *workspace, size_t ws_bytes, void *stream) {
    LBM_REQUIRE(nvox >= 1 && x && wh && bh && x_cs >= kHeadCin && no >= 1 && no <= kHeadMaxOut,
                LBM_E_INVAL, "lbm_nn_head: arguments (16 input channels, 1..8 outputs)");
    LBM_REQUIRE(!target || (mask && wt && gwh && gbh && loss_h && workspace && n_mask > 0),
                LBM_E_INVAL, "lbm_nn_head: a target needs mask, weights, gradient outputs and n_mask > 0");
    LBM_REQUIRE(!gx || gx_cs >= kHeadCin, LBM_E_INVAL, "lbm_nn_head: gradient stride");
    LBM_REQUIRE(!target || ws_bytes >= lbm_nn_head_workspace(nvox, no), LBM_E_NOMEM,
                "lbm_nn_head: workspace below %zu bytes", lbm_nn_head_workspace(nvox, no));
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nb = (nvox + 255) / 256, chunk = head_chunk(nvox), nch = (nvox + chunk - 1) / chunk;
    Carver c(workspace);
    double *loss_part = c.take<double>(nb);
    double *part = c.take<double>(nch * no * (kHeadCin + 1));
    double *dloss = c.take<double>(1);
    float *gout = c.take<float>(nvox * no);
    k_head<<<(unsigned)nb, 256, 0, s>>>(nvox, x, x_cs, no, wh, bh, out, target, mask, wt,
                                        target ? 1.0 / n_mask : 0.0, target ? gout : nullptr,
                                        target ? gx : nullptr, gx_cs, loss_part);
    LBM_CHECK_LAUNCH();
    if (target) {
        k_head_wgrad<<<dim3((unsigned)nch, (unsigned)no), 256, 0, s>>>(nvox, x, x_cs, gout, chunk, part);
        LBM_CHECK_LAUNCH();
        k_head_final<<<1, 256, 0, s>>>(loss_part, nb, part, nch, no, dloss, gwh, gbh);
        LBM_CHECK_LAUNCH();
        LBM_TRY_HIP(hipMemcpyAsync(loss_h, dloss, sizeof(double), hipMemcpyDeviceToHost, s));
        LBM_TRY_HIP(hipStreamSynchronize(s));
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_adam(int64_t n, float *w, const float *g, float *m, float *v,
                                  uint16_t *w_bf16, float lr, float beta1, float beta2, float eps,
                                  int64_t step, void *stream) {
    LBM_REQUIRE(n >= 0 && w && g && m && v && step >= 1 && lr > 0 && eps > 0 && beta1 >= 0 &&
                    beta1 < 1 && beta2 >= 0 && beta2 < 1,
                LBM_E_INVAL, "lbm_nn_adam: arguments");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    if (n == 0) return LBM_OK;
    const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
    k_adam<<<nblk(n), 256, 0, static_cast<hipStream_t>(stream)>>>(n, w, g, m, v, w_bf16, lr, beta1,
                                                                 beta2, eps, c1, c2);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_to_bf16(int64_t n, const float *src, uint16_t *dst, void *stream) {
    LBM_REQUIRE(n >= 0 && src && dst, LBM_E_INVAL, "lbm_nn_to_bf16: arguments");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    if (n == 0) return LBM_OK;
    k_to_bf16<<<nblk(n), 256, 0, static_cast<hipStream_t>(stream)>>>(n, src, dst);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_make_input(int64_t nvox, const uint8_t *mask, const double *diam,
                                        double d_scale, uint16_t *x, int32_t x_cs, void *stream) {
    LBM_REQUIRE(nvox >= 0 && mask && diam && x && x_cs >= 2 && x_cs % 4 == 0 && d_scale > 0,
                LBM_E_INVAL, "lbm_nn_make_input: arguments");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    if (nvox == 0) return LBM_OK;
    k_make_input<<<nblk(nvox), 256, 0, static_cast<hipStream_t>(stream)>>>(nvox, mask, diam,
                                                                          1.0 / d_scale, x, x_cs);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" lbm_status lbm_nn_to_fields(int64_t nvox, int32_t nk, const float *out, const uint8_t *mask,
                                       const float *scale, float *fields, void *stream) {
    LBM_REQUIRE(nvox >= 0 && nk >= 1 && out && mask && scale && fields, LBM_E_INVAL,
                "lbm_nn_to_fields: arguments");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    if (nvox == 0) return LBM_OK;
    k_to_fields<<<nblk(nvox * nk), 256, 0, static_cast<hipStream_t>(stream)>>>(nvox, nk, out, mask,
                                                                              scale, fields);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}
