// Reconstruction of an organic-matter nanostructure by random placement of pore
// spheres (Section 2, Steps 1-3).  The trial loop is inherently sequential (each
// acceptance depends on every sphere accepted before it), so it runs on the host, with a
// uniform cell grid to find the spheres a trial can touch; the finished mask is copied
// to the device.  Floating-point expressions are written in one fixed order and this
// file is compiled with -ffp-contract=off, so the decisions are those of the plain
// definition on every x86-64 host with the same C library.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lbm_internal.h"

namespace lbm {
namespace {

constexpr double kPi = 3.141592653589793;

// SplitMix64 (Steele, Lea & Flood 2014): the state advances by the golden gamma and the
// output is the variant-13 finaliser of the new state.
struct SplitMix64 {
    uint64_t state;
    uint64_t next() {
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
    // floor(u * 1024 * n), the product taken exactly
    int64_t centre(int n) {
        const unsigned __int128 p = (unsigned __int128)(next() >> 11) * (uint64_t)(1024ll * n);
        return (int64_t)(p >> 53);
    }
    // Marsaglia polar method, first normal of the pair
    double normal() {
        for (;;) {
            double a = 2.0 * uniform() - 1.0;
            double b = 2.0 * uniform() - 1.0;
            double q = a * a + b * b;
            if (q > 0.0 && q < 1.0) return a * std::sqrt(-2.0 * std::log(q) / q);
        }
    }
};

double ball_volume(double r) { return 4.0 * kPi * r * r * r / 3.0; }

// Volume shared by two spheres of radii r1, r2 whose centres are s apart.
double lens(double r1, double r2, double s) {
    if (s >= r1 + r2) return 0.0;
    const double rmin = r1 < r2 ? r1 : r2;
    if (s <= std::fabs(r1 - r2)) return ball_volume(rmin);
    const double t = r1 + r2 - s;
    const double q = r1 - r2;
    return kPi * t * t * (s * s + 2.0 * s * (r1 + r2) - 3.0 * q * q) / (12.0 * s);
}

struct Sphere {
    int64_t c[3], d;
};

// Uniform grid of cells of `cell` fixed-point units holding the indices of the spheres
// whose centres fall in them.
struct CellGrid {
    int64_t cell;
    int dims[3];
    std::vector<std::vector<int32_t>> cells;
    CellGrid(const int n[3], double d_mean) {
        cell = (int64_t)std::max(1.0, std::floor(d_mean)) * 1024;
        for (int a = 0; a < 3; a++) dims[a] = (int)((1024ll * n[a] + cell - 1) / cell);
        cells.resize((size_t)dims[0] * dims[1] * dims[2]);
    }
    int coord(int a, int64_t v) const {
        int64_t k = v / cell;
        return (int)std::min<int64_t>(std::max<int64_t>(k, 0), dims[a] - 1);
    }
    void add(const Sphere &s, int32_t id) {
        cells[((size_t)coord(2, s.c[2]) * dims[1] + coord(1, s.c[1])) * dims[0] + coord(0, s.c[0])]
            .push_back(id);
    }
};

}  // namespace
}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_reconstruct(const lbm_recon_params *p, uint8_t *pore, int64_t *spheres_h,
                                      int64_t sphere_cap, lbm_recon_stats *stats_h, void *stream) {
    LBM_REQUIRE(p && pore && stats_h, LBM_E_INVAL, "lbm_reconstruct: null argument");
    LBM_REQUIRE(p->n[0] >= 1 && p->n[1] >= 1 && p->n[2] >= 1 && p->n[0] <= kMaxEdge &&
                    p->n[1] <= kMaxEdge && p->n[2] <= kMaxEdge,
                LBM_E_INVAL, "sizes must lie in [1, %d]", kMaxEdge);
    LBM_REQUIRE(p->porosity > 0.0 && p->porosity < 1.0, LBM_E_INVAL, "porosity must lie in (0,1)");
    LBM_REQUIRE(p->overlap_tol >= 0.0 && p->overlap_tol <= 1.0, LBM_E_INVAL,
                "overlap tolerance must lie in [0,1]");
    LBM_REQUIRE(p->p_overlap >= 0.0 && p->p_overlap <= 1.0, LBM_E_INVAL,
                "overlap probability must lie in [0,1]");
    LBM_REQUIRE(p->d_mean > 0.0 && p->d_std >= 0.0 && std::isfinite(p->d_mean) &&
                    std::isfinite(p->d_std) && std::isfinite(p->d_min),
                LBM_E_INVAL, "bad diameter law");
    LBM_REQUIRE(!spheres_h || sphere_cap >= 0, LBM_E_INVAL, "negative sphere capacity");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;

    const int n[3] = {p->n[0], p->n[1], p->n[2]};
    const int64_t nvox = (int64_t)n[0] * n[1] * n[2];
    const int64_t target = (int64_t)std::ceil(p->porosity * (double)nvox);
    const int64_t max_trials = p->max_trials > 0 ? p->max_trials : 100000000ll;
    const double xi = p->overlap_tol;
    std::vector<uint8_t> mask((size_t)nvox, 0);
    std::vector<Sphere> acc;
    CellGrid grid(n, p->d_mean);
    SplitMix64 rng{p->seed};
    int64_t npore = 0, trials = 0, dq_max = 0;
    lbm_status result = LBM_OK;
    while (npore < target) {
        if (trials >= max_trials) {
            result = LBM_E_RECON_STALL;
            break;
        }
        trials++;
        bool must = false;
        if (!acc.empty()) {
            const double up = rng.uniform();
            must = xi > 0.0 && up < p->p_overlap;
        }
        Sphere s;
        for (int a = 0; a < 3; a++) s.c[a] = rng.centre(n[a]);
        double d;
        do {
            d = p->d_mean + p->d_std * rng.normal();
        } while (d < p->d_min);
        s.d = llround(d * 1024.0);
        const double r1 = (double)s.d / 2048.0;
        // spheres that can touch the trial have centres within (d + d_max)/2
        const int64_t reach = (s.d + dq_max) / 2 + 2;
        int lo[3], hi[3];
        for (int a = 0; a < 3; a++) {
            lo[a] = grid.coord(a, s.c[a] - reach);
            hi[a] = grid.coord(a, s.c[a] + reach);
        }
        bool ok = true, any = false;
        for (int cz = lo[2]; cz <= hi[2] && ok; cz++)
            for (int cy = lo[1]; cy <= hi[1] && ok; cy++)
                for (int cx = lo[0]; cx <= hi[0] && ok; cx++) {
                    const auto &cell = grid.cells[((size_t)cz * grid.dims[1] + cy) * grid.dims[0] + cx];
                    for (int32_t j : cell) {
                        const Sphere &o = acc[j];
                        const double dx = (double)(s.c[0] - o.c[0]) / 1024.0;
                        const double dy = (double)(s.c[1] - o.c[1]) / 1024.0;
                        const double dz = (double)(s.c[2] - o.c[2]) / 1024.0;
                        const double sep = std::sqrt(dx * dx + dy * dy + dz * dz);
                        const double r2 = (double)o.d / 2048.0;
                        const double v = lens(r1, r2, sep);
                        if (v > 0.0) any = true;
                        if (v > xi * ball_volume(r1 < r2 ? r1 : r2)) {
                            ok = false;
                            break;
                        }
                    }
                }
        if (must && !any) ok = false;
        if (!ok) continue;
        grid.add(s, (int32_t)acc.size());
        acc.push_back(s);
        dq_max = std::max(dq_max, s.d);
        // mark the voxels whose centres lie in the sphere (clipped to the box)
        int vlo[3], vhi[3];
        for (int a = 0; a < 3; a++) {
            const int64_t l = (s.c[a] - s.d / 2) / 1024 - 2, h = (s.c[a] + s.d / 2) / 1024 + 2;
            vlo[a] = (int)std::max<int64_t>(l, 0);
            vhi[a] = (int)std::min<int64_t>(h, n[a] - 1);
        }
        const int64_t d2 = s.d * s.d;
        for (int k = vlo[2]; k <= vhi[2]; k++) {
            const int64_t ez = 1024ll * k + 512 - s.c[2];
            for (int j = vlo[1]; j <= vhi[1]; j++) {
                const int64_t ey = 1024ll * j + 512 - s.c[1];
                const int64_t eyz = ey * ey + ez * ez;
                uint8_t *row = mask.data() + ((int64_t)k * n[1] + j) * n[0];
                for (int i = vlo[0]; i <= vhi[0]; i++) {
                    const int64_t ex = 1024ll * i + 512 - s.c[0];
                    if (4 * (ex * ex + eyz) <= d2 && !row[i]) {
                        row[i] = 1;
                        npore++;
                    }
                }
            }
        }
    }
    stats_h->n_spheres = (int64_t)acc.size();
    stats_h->n_trials = trials;
    stats_h->n_pore = npore;
    stats_h->porosity = (double)npore / (double)nvox;
    if (spheres_h) {
        const int64_t m = std::min<int64_t>((int64_t)acc.size(), sphere_cap);
        for (int64_t i = 0; i < m; i++) {
            for (int a = 0; a < 3; a++) spheres_h[4 * i + a] = acc[i].c[a];
            spheres_h[4 * i + 3] = acc[i].d;
        }
    }
    if (result != LBM_OK) {
        set_error("reconstruction stalled: %lld trials reached porosity %.4f of %.4f",
                  (long long)trials, stats_h->porosity, p->porosity);
        return result;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    LBM_TRY_HIP(hipMemcpyAsync(pore, mask.data(), (size_t)nvox, hipMemcpyHostToDevice, s));
    LBM_TRY_HIP(hipStreamSynchronize(s));
    return LBM_OK;
}
