/*
 * lbm_oracle.c -- plain, slow FP64 CPU oracle for the lattice Boltzmann
 * transport pipeline of Chen, Kang, Zhang & Tao, "Lattice Boltzmann prediction
 * of transport properties in reconstructed nanostructures of organic matters
 * in shales" (arXiv:1410.1921).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or constant with the HIP
 * library; every table below is written out here on its own.
 *
 * Everything works on the dense lattice (all N^3 voxels plus a mask), in
 * double precision, voxel linear index v = x + nx*(y + ny*z).  Loops follow the
 * paper's order of operations; there is no blocking or fusion.  OpenMP only
 * splits independent per-voxel loops over z; every sum is formed per z-plane
 * and then added plane by plane in order, so results do not depend on the
 * thread count.
 *
 * Readings of passages the paper leaves open are listed where they are used
 * and collected in the design notes of the repository.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.141592653589793

#define ORC_OK 0
#define ORC_W_NOT_CONVERGED 1
#define ORC_E_INVAL (-1)
#define ORC_E_NOMEM (-2)
#define ORC_E_STALL (-4)
#define ORC_E_DIVERGED (-5)

static int64_t vidx(int x, int y, int z, int nx, int ny) {
    return (int64_t)x + (int64_t)nx * ((int64_t)y + (int64_t)ny * z);
}
static int wrap(int a, int n) {
    a %= n;
    return a < 0 ? a + n : a;
}

/* ======================================================================
 * Section 2 (structure reconstruction), Steps 1-3.
 * The paper only says "random number generators"; the reading used here is
 * SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), written from its published
 * definition: the state advances by the golden gamma and each output is the
 * variant-13 finaliser of the new state.
 * ====================================================================== */
uint64_t orc_splitmix64_next(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform in [0,1): the top 53 bits scaled by 2^-53 */
double orc_uniform(uint64_t *state) {
    return (double)(orc_splitmix64_next(state) >> 11) * (1.0 / 9007199254740992.0);
}

/* standard normal by the Marsaglia polar method; the second normal of the
 * pair is discarded */
double orc_normal(uint64_t *state) {
    for (;;) {
        double a = 2.0 * orc_uniform(state) - 1.0;
        double b = 2.0 * orc_uniform(state) - 1.0;
        double q = a * a + b * b;
        if (q > 0.0 && q < 1.0) return a * sqrt(-2.0 * log(q) / q);
    }
}

/* a centre coordinate in 1/1024-voxel units: floor(u * 1024 * n) with the
 * product taken exactly in integers */
static int64_t draw_centre(uint64_t *state, int n) {
    uint64_t top = orc_splitmix64_next(state) >> 11; /* u = top / 2^53 */
    unsigned __int128 p = (unsigned __int128)top * (uint64_t)(1024LL * n);
    return (int64_t)(p >> 53);
}

/* volume of a sphere of radius r */
double orc_sphere_volume(double r) { return 4.0 * ORC_PI * r * r * r / 3.0; }

/* volume of the lens shared by spheres of radii r1, r2 with centres s apart */
double orc_lens_volume(double r1, double r2, double s) {
    if (s >= r1 + r2) return 0.0;
    double rmin = r1 < r2 ? r1 : r2;
    if (s <= fabs(r1 - r2)) return orc_sphere_volume(rmin);
    double t = r1 + r2 - s;
    double q = r1 - r2;
    return ORC_PI * t * t * (s * s + 2.0 * s * (r1 + r2) - 3.0 * q * q) / (12.0 * s);
}

/*
 * Reconstruction by random placement of pore spheres (Section 2, Steps 1-3).
 * Readings: diameters ~ N(d_mean, d_std) voxels redrawn below d_min; centres
 * uniform over the box, geometry not periodic; the overlap tolerance is
 * checked pairwise against both spheres' volumes; a trial that must overlap
 * (probability p0, disabled when xi == 0) needs at least one lens of positive
 * volume; stop at the first accepted sphere that brings the pore count to
 * ceil(eps * N^3).  Draw order per trial: overlap coin (not for the first
 * sphere), centre x, y, z, then the diameter.
 * Voxel (i,j,k) is pore iff 4*sum((1024*i + 512 - c)^2) <= d^2 in integers
 * (centres c and diameter d in 1/1024-voxel units).
 * spheres: cap rows of (cx, cy, cz, d) in 1/1024-voxel units.
 * info[0]=n_spheres, info[1]=n_trials, info[2]=n_pore.
 */
int orc_reconstruct(int nx, int ny, int nz, double eps, double d_mean, double d_std,
                    double d_min, double xi, double p0, uint64_t seed, int64_t max_trials,
                    uint8_t *pore, int64_t *spheres, int64_t cap, int64_t *info) {
    if (nx < 1 || ny < 1 || nz < 1 || !(eps > 0.0 && eps < 1.0) || !(xi >= 0.0 && xi <= 1.0) ||
        !(p0 >= 0.0 && p0 <= 1.0) || !(d_mean > 0.0) || !(d_std >= 0.0) || !pore)
        return ORC_E_INVAL;
    int64_t nvox = (int64_t)nx * ny * nz;
    memset(pore, 0, (size_t)nvox);
    int64_t target = (int64_t)ceil(eps * (double)nvox);
    int64_t nsph = 0, ncap = 64, npore = 0, trials = 0;
    int64_t *acc = (int64_t *)malloc((size_t)ncap * 4 * sizeof(int64_t));
    if (!acc) return ORC_E_NOMEM;
    uint64_t st = seed;
    while (npore < target) {
        if (trials >= max_trials) {
            free(acc);
            info[0] = nsph; info[1] = trials; info[2] = npore;
            return ORC_E_STALL;
        }
        trials++;
        int must = 0;
        if (nsph > 0) {
            double up = orc_uniform(&st);
            must = (xi > 0.0) && (up < p0);
        }
        int64_t cx = draw_centre(&st, nx);
        int64_t cy = draw_centre(&st, ny);
        int64_t cz = draw_centre(&st, nz);
        double d;
        do { d = d_mean + d_std * orc_normal(&st); } while (d < d_min);
        int64_t dq = llround(d * 1024.0);
        double r1 = (double)dq / 2048.0;
        int ok = 1, any = 0;
        for (int64_t j = 0; j < nsph && ok; j++) {
            double dx = (double)(cx - acc[4 * j + 0]) / 1024.0;
            double dy = (double)(cy - acc[4 * j + 1]) / 1024.0;
            double dz = (double)(cz - acc[4 * j + 2]) / 1024.0;
            double s = sqrt(dx * dx + dy * dy + dz * dz);
            double r2 = (double)acc[4 * j + 3] / 2048.0;
            double v = orc_lens_volume(r1, r2, s);
            if (v > 0.0) any = 1;
            if (v > xi * orc_sphere_volume(r1 < r2 ? r1 : r2)) ok = 0;
        }
        if (must && !any) ok = 0;
        if (!ok) continue;
        if (nsph == ncap) {
            ncap *= 2;
            int64_t *t = (int64_t *)realloc(acc, (size_t)ncap * 4 * sizeof(int64_t));
            if (!t) { free(acc); return ORC_E_NOMEM; }
            acc = t;
        }
        acc[4 * nsph + 0] = cx; acc[4 * nsph + 1] = cy;
        acc[4 * nsph + 2] = cz; acc[4 * nsph + 3] = dq;
        nsph++;
        /* voxelise: a box that surely contains the sphere, clipped to the domain */
        int64_t c[3] = {cx, cy, cz};
        int lo[3], hi[3], nn[3] = {nx, ny, nz};
        for (int a = 0; a < 3; a++) {
            int64_t l = (c[a] - dq / 2) / 1024 - 2, h = (c[a] + dq / 2) / 1024 + 2;
            lo[a] = l < 0 ? 0 : (int)l;
            hi[a] = h > nn[a] - 1 ? nn[a] - 1 : (int)h;
        }
        int64_t d2 = dq * dq;
        for (int k = lo[2]; k <= hi[2]; k++)
            for (int j = lo[1]; j <= hi[1]; j++)
                for (int i = lo[0]; i <= hi[0]; i++) {
                    int64_t ex = 1024LL * i + 512 - cx, ey = 1024LL * j + 512 - cy,
                            ez = 1024LL * k + 512 - cz;
                    if (4 * (ex * ex + ey * ey + ez * ez) <= d2) {
                        int64_t v = vidx(i, j, k, nx, ny);
                        if (!pore[v]) { pore[v] = 1; npore++; }
                    }
                }
    }
    if (spheres) {
        int64_t m = nsph < cap ? nsph : cap;
        memcpy(spheres, acc, (size_t)m * 4 * sizeof(int64_t));
    }
    info[0] = nsph; info[1] = trials; info[2] = npore;
    free(acc);
    return ORC_OK;
}

/* ======================================================================
 * Section 4.1: connected-phase labelling with the 18 neighbours (the 6 face
 * and 12 edge neighbours, as the D3Q19 links).  Readings: periodic in y and z,
 * open in x; a component is "transport" when it holds pore voxels on both
 * x = 0 and x = nx-1; each component's label is the smallest linear index in
 * it.  Breadth-first search from each unlabelled pore voxel in increasing
 * index order gives exactly that label.
 * info[0]=n_pore, info[1]=n_transport, info[2]=n_components.
 * ====================================================================== */
int orc_label18(int nx, int ny, int nz, const uint8_t *pore, int32_t *label,
                uint8_t *transport, int64_t *info) {
    int64_t nvox = (int64_t)nx * ny * nz;
    int64_t *queue = (int64_t *)malloc((size_t)nvox * sizeof(int64_t));
    if (!queue) return ORC_E_NOMEM;
    for (int64_t v = 0; v < nvox; v++) label[v] = -1;
    uint8_t *in_root = (uint8_t *)calloc((size_t)nvox, 1);
    uint8_t *out_root = (uint8_t *)calloc((size_t)nvox, 1);
    int64_t npore = 0, ncomp = 0, ntr = 0;
    for (int64_t s = 0; s < nvox; s++) {
        if (!pore[s] || label[s] >= 0) continue;
        ncomp++;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = (int32_t)s;
        while (head < tail) {
            int64_t v = queue[head++];
            int x = (int)(v % nx), y = (int)((v / nx) % ny), z = (int)(v / ((int64_t)nx * ny));
            if (x == 0) in_root[s] = 1;
            if (x == nx - 1) out_root[s] = 1;
            for (int dz = -1; dz <= 1; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        int m = abs(dx) + abs(dy) + abs(dz);
                        if (m < 1 || m > 2) continue;
                        int xx = x + dx;
                        if (xx < 0 || xx >= nx) continue;
                        int64_t u = vidx(xx, wrap(y + dy, ny), wrap(z + dz, nz), nx, ny);
                        if (pore[u] && label[u] < 0) {
                            label[u] = (int32_t)s;
                            queue[tail++] = u;
                        }
                    }
        }
    }
    for (int64_t v = 0; v < nvox; v++) {
        uint8_t t = 0;
        if (pore[v]) {
            npore++;
            t = in_root[label[v]] && out_root[label[v]];
            ntr += t;
        }
        if (transport) transport[v] = t;
    }
    free(queue); free(in_root); free(out_root);
    info[0] = npore; info[1] = ntr; info[2] = ncomp;
    return ORC_OK;
}

/* ======================================================================
 * Section 4.1: the 13-direction averaging pore size.  For each pore voxel and
 * each of the 13 directions (3 axes, 6 face diagonals, 4 body diagonals) the
 * chord is the run of consecutive pore voxels through it along that line,
 * stopping at the domain faces (reading); its length is the voxel count times
 * the direction's length (1, sqrt 2, sqrt 3).  The pore size is the mean of
 * the 13 chord lengths, formed from the integer class sums A, B, C as
 * ((A + sqrt2*B) + sqrt3*C) / 13.  Solid voxels get 0.
 * counts (nullable): 3 int64 per voxel (A, B, C).
 * ====================================================================== */
static const int DIR13[13][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1},
    {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {-1, 1, 1}};

void orc_chords13(int nx, int ny, int nz, const uint8_t *pore, double *diam, int64_t *counts) {
    const double s2 = sqrt(2.0), s3 = sqrt(3.0);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t v = vidx(x, y, z, nx, ny);
                int64_t cls[3] = {0, 0, 0};
                if (pore[v]) {
                    for (int d = 0; d < 13; d++) {
                        int64_t run = 1;
                        for (int sgn = -1; sgn <= 1; sgn += 2) {
                            int xx = x, yy = y, zz = z;
                            for (;;) {
                                xx += sgn * DIR13[d][0]; yy += sgn * DIR13[d][1]; zz += sgn * DIR13[d][2];
                                if (xx < 0 || xx >= nx || yy < 0 || yy >= ny || zz < 0 || zz >= nz) break;
                                if (!pore[vidx(xx, yy, zz, nx, ny)]) break;
                                run++;
                            }
                        }
                        cls[d < 3 ? 0 : (d < 9 ? 1 : 2)] += run;
                    }
                    diam[v] = ((double)cls[0] + s2 * (double)cls[1] + s3 * (double)cls[2]) / 13.0;
                } else {
                    diam[v] = 0.0;
                }
                if (counts) { counts[3 * v] = cls[0]; counts[3 * v + 1] = cls[1]; counts[3 * v + 2] = cls[2]; }
            }
}

/* ======================================================================
 * Maximum-inscribed-sphere pore diameter (the local-thickness map; not in the
 * paper, used for the 128^3 methane workload).
 * Squared Euclidean distance from each voxel centre to the nearest solid voxel
 * centre, no wrap, taken axis by axis: the squared distance separates into a
 * sum over axes, so three passes of the exact 1-D minimum
 * g_k(p) = min_t (g_{k-1}(p with axis k set to t) + (p_k - t)^2) give it.
 * Each 1-D minimum is taken by brute force over the whole line.
 * Returns ORC_E_INVAL when the domain holds no solid voxel.
 * ====================================================================== */
#define ORC_INF (INT64_C(1) << 60)
int orc_edt2(int nx, int ny, int nz, const uint8_t *pore, int64_t *e2) {
    int64_t nvox = (int64_t)nx * ny * nz;
    int any_solid = 0;
    for (int64_t v = 0; v < nvox; v++) if (!pore[v]) { any_solid = 1; break; }
    if (!any_solid) return ORC_E_INVAL;
    int64_t *g = (int64_t *)malloc((size_t)nvox * sizeof(int64_t));
    if (!g) return ORC_E_NOMEM;
    int n[3] = {nx, ny, nz};
    int64_t stride[3] = {1, nx, (int64_t)nx * ny};
    /* pass along x from the solid indicator */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t best = ORC_INF;
                for (int t = 0; t < nx; t++)
                    if (!pore[vidx(t, y, z, nx, ny)]) {
                        int64_t dd = (int64_t)(x - t) * (x - t);
                        if (dd < best) best = dd;
                    }
                g[vidx(x, y, z, nx, ny)] = best;
            }
    /* passes along y then z */
    int64_t *src = g, *dst = e2;
    for (int axis = 1; axis <= 2; axis++) {
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    int p[3] = {x, y, z};
                    int64_t base = vidx(x, y, z, nx, ny) - (int64_t)p[axis] * stride[axis];
                    int64_t best = ORC_INF;
                    for (int t = 0; t < n[axis]; t++) {
                        int64_t gv = src[base + (int64_t)t * stride[axis]];
                        if (gv >= ORC_INF) continue;
                        int64_t dd = gv + (int64_t)(p[axis] - t) * (p[axis] - t);
                        if (dd < best) best = dd;
                    }
                    dst[vidx(x, y, z, nx, ny)] = best;
                }
        int64_t *tmp = src; src = dst; dst = tmp;
    }
    /* after two swaps the result sits in g; copy it to e2 */
    if (src != e2) memcpy(e2, src, (size_t)nvox * sizeof(int64_t));
    free(g);
    return ORC_OK;
}

/* d_MIS(p) = 2*sqrt(max{ e2(c) : c pore, |p-c|^2 < e2(c) }) - 1 for pore p
 * (the widest inscribed ball covering p; the "-1" turns a centre-to-solid-
 * centre distance into a pore width).  Solid voxels get 0.
 * emax (out, nullable): the covering maximum of e2 per voxel. */
void orc_mis(int nx, int ny, int nz, const uint8_t *pore, const int64_t *e2, double *diam,
             int64_t *emax) {
    int64_t nvox = (int64_t)nx * ny * nz, mx = 0;
    for (int64_t v = 0; v < nvox; v++) if (pore[v] && e2[v] > mx) mx = e2[v];
    int R = (int)ceil(sqrt((double)mx));
#pragma omp parallel for schedule(dynamic, 1)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int64_t v = vidx(x, y, z, nx, ny), best = 0;
                if (pore[v]) {
                    for (int dz = -R; dz <= R; dz++) {
                        int zz = z + dz;
                        if (zz < 0 || zz >= nz) continue;
                        for (int dy = -R; dy <= R; dy++) {
                            int yy = y + dy;
                            if (yy < 0 || yy >= ny) continue;
                            for (int dx = -R; dx <= R; dx++) {
                                int xx = x + dx;
                                if (xx < 0 || xx >= nx) continue;
                                int64_t c = vidx(xx, yy, zz, nx, ny);
                                if (!pore[c]) continue;
                                int64_t dd = (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz;
                                if (dd < e2[c] && e2[c] > best) best = e2[c];
                            }
                        }
                    }
                    diam[v] = 2.0 * sqrt((double)best) - 1.0;
                } else {
                    diam[v] = 0.0;
                }
                if (emax) emax[v] = best;
            }
}

/* ======================================================================
 * Section 3.2, Eq. 12: local relaxation time from the local pore diameter,
 * tau_g = (d_p / d_ref) (tau_ref - 1/2) + 1/2 (d_p, d_ref in voxels).
 * ====================================================================== */
double orc_tau_g(double d_p, double d_ref, double tau_ref) {
    return d_p / d_ref * (tau_ref - 0.5) + 0.5;
}

/* ======================================================================
 * Section 3.1: D3Q19 lattice (Eq. 2, with the repeated (0,+-1,0) of the
 * printed equation read as (0,0,+-1)); velocity order follows the columns of
 * the transformation matrix in Appendix A; weights 1/3, 1/18, 1/36.
 * ====================================================================== */
static const int E19[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0},
    {1, 0, 1}, {-1, 0, 1}, {1, 0, -1}, {-1, 0, -1},
    {0, 1, 1}, {0, -1, 1}, {0, 1, -1}, {0, -1, -1}};

static double w19(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

/* the direction whose velocity is the negative of e_i */
static int opp19(int i) {
    for (int j = 0; j < 19; j++)
        if (E19[j][0] == -E19[i][0] && E19[j][1] == -E19[i][1] && E19[j][2] == -E19[i][2]) return j;
    return -1;
}

/*
 * One BGK collision at a node (Eq. 1 with S = 1/tau, equilibrium Eq. 3 with
 * c_s^2 = 1/3, density and momentum Eq. 9) with a constant body force F
 * (force density; the paper drives with pressure, the body force is the
 * reading for this workload) added by Guo, Zheng & Shi (2002): the velocity
 * carries half the force, u = (j + F/2)/rho, and the source is
 * (1 - 1/(2 tau)) w_i [3 (e_i - u) + 9 (e_i.u) e_i] . F.
 * mom (out, nullable): rho, then rho*u (= j + F/2).
 */
void orc_collide19(const double *fin, double tau, const double *F, double *fout, double *mom) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; i++) {
        rho += fin[i];
        for (int a = 0; a < 3; a++) j[a] += fin[i] * E19[i][a];
    }
    double u[3];
    for (int a = 0; a < 3; a++) u[a] = (j[a] + 0.5 * F[a]) / rho;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < 19; i++) {
        double eu = E19[i][0] * u[0] + E19[i][1] * u[1] + E19[i][2] * u[2];
        double feq = w19(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
        double eF = E19[i][0] * F[0] + E19[i][1] * F[1] + E19[i][2] * F[2];
        double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        double src = (1.0 - 0.5 / tau) * w19(i) * (3.0 * (eF - uF) + 9.0 * eu * eF);
        fout[i] = fin[i] - (fin[i] - feq) / tau + src;
    }
    if (mom) {
        mom[0] = rho;
        for (int a = 0; a < 3; a++) mom[1 + a] = rho * u[a];
    }
}

/*
 * Section 3.1, Eqs. 4-7 and Appendix A: the MRT collision.  Q is the
 * transformation matrix of Appendix A (rows: the 19 moments; columns: the
 * velocities in the order of E19).  Its inverse is not taken from the printed
 * table (row 6 of the printed inverse is garbled) but from the orthogonality of
 * Q's rows: Q^{-1}[i][k] = Q[k][i] / |Q_k|^2.
 */
static const double Q19[19][19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},
    {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, -4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1}};

/* q (19x19, row-major) and its inverse */
void orc_mrt_matrices(double *q, double *qinv) {
    for (int k = 0; k < 19; k++) {
        double n2 = 0.0;
        for (int i = 0; i < 19; i++) n2 += Q19[k][i] * Q19[k][i];
        for (int i = 0; i < 19; i++) {
            if (q) q[19 * k + i] = Q19[k][i];
            if (qinv) qinv[19 * i + k] = Q19[k][i] / n2;
        }
    }
}

/* Eq. 7: the relaxation rate of each moment (0 for the conserved ones) */
void orc_mrt_rates(double tau, double *s) {
    double sq = 8.0 * (2.0 * tau - 1.0) / (8.0 * tau - 1.0);
    for (int k = 0; k < 19; k++) s[k] = 1.0 / tau;
    s[0] = s[3] = s[5] = s[7] = 0.0;
    s[4] = s[6] = s[8] = s[16] = s[17] = s[18] = sq;
}

/*
 * One MRT collision (Eqs. 4-7) with the body force of the BGK collision: m = Q f;
 * equilibrium moments A1-A9 with rho0 = 1 (reading: the mean density of the
 * fluid at rest) and j = sum f e + F/2; m* = m - S (m - m_eq) + (I - S/2) Q F_src
 * with Guo's source F_src,i = w_i [3 (e_i - u) + 9 (e_i.u) e_i] . F, u = j / rho;
 * f* = Q^{-1} m*.  rates (nullable): the 19 relaxation rates, else Eq. 7.
 * mom (out, nullable): rho, then j (= rho u).
 */
void orc_collide19_mrt(const double *fin, double tau, const double *rates, const double *F,
                       double *fout, double *mom) {
    double q[361], qinv[361], s[19];
    orc_mrt_matrices(q, qinv);
    if (rates) memcpy(s, rates, sizeof(s));
    else orc_mrt_rates(tau, s);
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; i++) {
        rho += fin[i];
        for (int a = 0; a < 3; a++) j[a] += fin[i] * E19[i][a];
    }
    for (int a = 0; a < 3; a++) j[a] += 0.5 * F[a];
    double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    const double rho0 = 1.0;
    double jj = (j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / rho0;
    double meq[19];
    meq[0] = rho;
    meq[1] = -11.0 * rho + 19.0 * jj;
    meq[2] = 3.0 * rho - 5.5 * jj;
    meq[3] = j[0]; meq[4] = -2.0 / 3.0 * j[0];
    meq[5] = j[1]; meq[6] = -2.0 / 3.0 * j[1];
    meq[7] = j[2]; meq[8] = -2.0 / 3.0 * j[2];
    meq[9] = (3.0 * j[0] * j[0] / rho0 - jj);
    meq[10] = -0.5 * meq[9];
    meq[11] = (j[1] * j[1] - j[2] * j[2]) / rho0;
    meq[12] = -0.5 * meq[11];
    meq[13] = j[0] * j[1] / rho0;
    meq[14] = j[1] * j[2] / rho0;
    meq[15] = j[0] * j[2] / rho0;
    meq[16] = meq[17] = meq[18] = 0.0;
    double src[19];
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    for (int i = 0; i < 19; i++) {
        double eu = E19[i][0] * u[0] + E19[i][1] * u[1] + E19[i][2] * u[2];
        double eF = E19[i][0] * F[0] + E19[i][1] * F[1] + E19[i][2] * F[2];
        src[i] = w19(i) * (3.0 * (eF - uF) + 9.0 * eu * eF);
    }
    double mstar[19];
    for (int k = 0; k < 19; k++) {
        double m = 0.0, fm = 0.0;
        for (int i = 0; i < 19; i++) {
            m += q[19 * k + i] * fin[i];
            fm += q[19 * k + i] * src[i];
        }
        mstar[k] = m - s[k] * (m - meq[k]) + (1.0 - 0.5 * s[k]) * fm;
    }
    for (int i = 0; i < 19; i++) {
        double v = 0.0;
        for (int k = 0; k < 19; k++) v += qinv[19 * i + k] * mstar[k];
        fout[i] = v;
    }
    if (mom) {
        mom[0] = rho;
        for (int a = 0; a < 3; a++) mom[1 + a] = j[a];
    }
}

/*
 * Streaming (pull form) for one node: f_i arrives from x - e_i (periodic in
 * x, y and z); when that neighbour is solid, half-way bounce-back returns the
 * node's own post-collision f of the opposite direction (Section 3.3).
 * f is stored node-major: f[19*v + i].
 */
static void gather19(int nx, int ny, int nz, const uint8_t *fluid, const double *f, int x, int y,
                     int z, double *fin) {
    int64_t v = vidx(x, y, z, nx, ny);
    for (int i = 0; i < 19; i++) {
        int64_t s = vidx(wrap(x - E19[i][0], nx), wrap(y - E19[i][1], ny), wrap(z - E19[i][2], nz), nx, ny);
        fin[i] = fluid[s] ? f[19 * s + i] : f[19 * v + opp19(i)];
    }
}

/* The equilibrium of Eq. 3 (compressible form) of population i at rho, u. */
static double feq19(int i, double rho, const double *u) {
    double eu = E19[i][0] * u[0] + E19[i][1] * u[1] + E19[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return w19(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

/*
 * Pressure boundaries (Section 3.3) by Guo's non-equilibrium extrapolation: the ghost
 * node at x = -1 (x = nx) next to boundary node b = (0, y, z) ((nx - 1, y, z)) holds the
 * post-collision populations f_eq(rho_bc, u_b) + [f(b) - f_eq(rho_b, u_b)], with rho_b,
 * u_b the moments of b's post-collision state (u_b = (sum f e - F/2) / rho_b, the
 * velocity of b's collision) and f_eq that of Eq. 3.  The ghost planes continue the
 * boundary planes' geometry: a ghost beside a solid b is solid (links to it bounce
 * back), so walls that reach the x faces stay closed.  Population i of the ghost at
 * (y, z), b fluid.
 */
static double ghost19(int nx, int ny, const uint8_t *fluid, const double *f, int xb, int y, int z,
                      int i, double rho_bc, const double *F) {
    int64_t b = vidx(xb, y, z, nx, ny);
    (void)fluid;
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 19; k++) {
        rho += f[19 * b + k];
        for (int a = 0; a < 3; a++) j[a] += f[19 * b + k] * E19[k][a];
    }
    double u[3];
    for (int a = 0; a < 3; a++) u[a] = (j[a] - 0.5 * F[a]) / rho;
    return feq19(i, rho_bc, u) + (f[19 * b + i] - feq19(i, rho, u));
}

/* gather19 with x open: sources beyond an x face come from the ghost planes */
static void gather19_p(int nx, int ny, int nz, const uint8_t *fluid, const double *f, int x, int y,
                       int z, double rho_in, double rho_out, const double *F, double *fin) {
    int64_t v = vidx(x, y, z, nx, ny);
    for (int i = 0; i < 19; i++) {
        int sx = x - E19[i][0], sy = wrap(y - E19[i][1], ny), sz = wrap(z - E19[i][2], nz);
        if (sx < 0 || sx >= nx) {
            int xb = sx < 0 ? 0 : nx - 1;
            if (!fluid[vidx(xb, sy, sz, nx, ny)]) { fin[i] = f[19 * v + opp19(i)]; continue; }
            fin[i] = ghost19(nx, ny, fluid, f, xb, sy, sz, i, sx < 0 ? rho_in : rho_out, F);
            continue;
        }
        int64_t s = vidx(sx, sy, sz, nx, ny);
        fin[i] = fluid[s] ? f[19 * s + i] : f[19 * v + opp19(i)];
    }
}

/* initial populations: the D3Q19 equilibrium (Eq. 3) at rho = 1 + drho_init and u
 * (u_init planar [3][N^3], drho_init [N^3]; zero where null) */
void orc_flow_init(int nx, int ny, int nz, const uint8_t *fluid, const double *u_init,
                   const double *drho_init, double *f) {
    int64_t nvox = (int64_t)nx * ny * nz;
    for (int64_t v = 0; v < nvox; v++) {
        double u[3] = {0.0, 0.0, 0.0};
        double rho = 1.0;
        if (u_init && fluid[v]) for (int a = 0; a < 3; a++) u[a] = u_init[a * nvox + v];
        if (drho_init && fluid[v]) rho = 1.0 + drho_init[v];
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        for (int i = 0; i < 19; i++) {
            double eu = E19[i][0] * u[0] + E19[i][1] * u[1] + E19[i][2] * u[2];
            f[19 * v + i] = fluid[v] ? w19(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu) : 0.0;
        }
    }
}

/*
 * The two-relaxation-time form of the MRT collision above (Eq. 7 relaxes every even
 * non-conserved moment at 1/tau and every odd one at s_q, with the equilibrium moments
 * A1-A9 of the incompressible equilibrium, rho0 = 1): in velocity space, each pair of
 * opposite velocities (i, i') splits into its even part f+ = (f_i + f_i')/2, relaxed at
 * s+ = 1/tau towards the even part of f_eq,i = w_i [rho + 3 e.j + 9/2 (e.j)^2 - 3/2 j^2]
 * (j = sum f e + F/2), and its odd part f- = (f_i - f_i')/2, relaxed at s- = s_q towards
 * 3 w_i e.j; Guo's source splits alike, each part scaled by (1 - s/2).
 */
void orc_collide19_trt(const double *fin, double tau, const double *F, double *fout,
                       double *mom) {
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; i++) {
        rho += fin[i];
        for (int a = 0; a < 3; a++) j[a] += fin[i] * E19[i][a];
    }
    for (int a = 0; a < 3; a++) j[a] += 0.5 * F[a];
    const double u[3] = {j[0] / rho, j[1] / rho, j[2] / rho};
    const double sp = 1.0 / tau, sm = 8.0 * (2.0 * tau - 1.0) / (8.0 * tau - 1.0);
    const double jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
    const double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    for (int i = 0; i < 19; i++) {
        const int k = opp19(i);
        const double ej = E19[i][0] * j[0] + E19[i][1] * j[1] + E19[i][2] * j[2];
        const double eu = E19[i][0] * u[0] + E19[i][1] * u[1] + E19[i][2] * u[2];
        const double eF = E19[i][0] * F[0] + E19[i][1] * F[1] + E19[i][2] * F[2];
        const double w = w19(i);
        const double feq_even = w * (rho + 4.5 * ej * ej - 1.5 * jj);
        const double feq_odd = w * 3.0 * ej;
        const double src_even = w * (-3.0 * uF + 9.0 * eu * eF);
        const double src_odd = w * 3.0 * eF;
        const double f_even = 0.5 * (fin[i] + fin[k]), f_odd = 0.5 * (fin[i] - fin[k]);
        fout[i] = fin[i] - sp * (f_even - feq_even) - sm * (f_odd - feq_odd) +
                  (1.0 - 0.5 * sp) * src_even + (1.0 - 0.5 * sm) * src_odd;
    }
    if (mom) {
        mom[0] = rho;
        for (int a = 0; a < 3; a++) mom[1 + a] = j[a];
    }
}

/*
 * The flow solve: iterate stream + collide (collision 0: BGK, orc_collide19;
 * 1: MRT, orc_collide19_mrt; 2: its two-relaxation-time form, orc_collide19_trt)
 * from the state in f (node-major
 * 19*N^3, in/out).  Every check_every steps (and at the last step) the
 * moments of the incoming populations give u = rho*u / rho; the residual is
 * ||u(t) - u(t - n_c)||_2 / (n_c ||u(t)||_2) over fluid nodes (reading: the
 * paper only says "steady state"), the snapshot starting from u_prev0
 * (planar [3][N^3]; zero when null).  With fixed_steps > 0 exactly that many
 * steps run; otherwise the run stops at the first check with residual < tol
 * or at max_steps.  Darcy (Eq. 13) with the body force in place of the
 * pressure gradient: k = nu <rho u_x> / F_x, nu = (tau - 1/2)/3 (Eq. 8), the
 * average taken over the whole box (superficial velocity).
 * out: [0]=steps [1]=k_lattice [2]=residual [3..5]=<rho u> over the box
 *      [6]=sum of rho - n_fluid [7]=converged.
 * u_out (nullable): planar [3][N^3] velocity of the last step (0 at solids).
 */
static int flow_solve_impl(int nx, int ny, int nz, const uint8_t *fluid, double tau,
                           int collision, const double *F, int pressure, double rho_in,
                           double rho_out, int64_t max_steps, int64_t fixed_steps,
                           int check_every, double tol, const double *u_prev0, double *f,
                           double *u_out, double *out) {
    if (!(tau > 0.5) || check_every < 1) return ORC_E_INVAL;
    int64_t nvox = (int64_t)nx * ny * nz;
    double *f0 = f; /* the caller's buffer: holds the final state on return */
    double *g = (double *)malloc((size_t)nvox * 19 * sizeof(double));
    double *gbuf = g;
    double *uprev = (double *)calloc((size_t)nvox * 3, sizeof(double));
    double *ucur = (double *)calloc((size_t)nvox * 3, sizeof(double));
    double *pl = (double *)calloc((size_t)nz * 6, sizeof(double));
    if (!g || !uprev || !ucur || !pl) { free(g); free(uprev); free(ucur); free(pl); return ORC_E_NOMEM; }
    if (u_prev0) memcpy(uprev, u_prev0, (size_t)nvox * 3 * sizeof(double));
    int64_t nfl = 0;
    for (int64_t v = 0; v < nvox; v++) nfl += fluid[v] ? 1 : 0;
    int64_t limit = fixed_steps > 0 ? fixed_steps : max_steps;
    double resid = INFINITY, sums[6] = {0, 0, 0, 0, 0, 0};
    int status = ORC_W_NOT_CONVERGED, diverged = 0;
    int64_t t = 0;
    while (t < limit) {
        t++;
        int check = (t % check_every == 0) || (t == limit);
        memset(pl, 0, (size_t)nz * 6 * sizeof(double));
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    int64_t v = vidx(x, y, z, nx, ny);
                    if (!fluid[v]) {
                        for (int i = 0; i < 19; i++) g[19 * v + i] = 0.0;
                        continue;
                    }
                    double fin[19], mom[4];
                    if (pressure) gather19_p(nx, ny, nz, fluid, f, x, y, z, rho_in, rho_out, F, fin);
                    else gather19(nx, ny, nz, fluid, f, x, y, z, fin);
                    if (collision == 1) orc_collide19_mrt(fin, tau, NULL, F, g + 19 * v, mom);
                    else if (collision == 2) orc_collide19_trt(fin, tau, F, g + 19 * v, mom);
                    else orc_collide19(fin, tau, F, g + 19 * v, mom);
                    if (check) {
                        double du2 = 0.0, u2 = 0.0;
                        for (int a = 0; a < 3; a++) {
                            double ua = mom[1 + a] / mom[0];
                            ucur[a * nvox + v] = ua;
                            du2 += (ua - uprev[a * nvox + v]) * (ua - uprev[a * nvox + v]);
                            u2 += ua * ua;
                        }
                        pl[6 * z + 0] += du2;
                        pl[6 * z + 1] += u2;
                        pl[6 * z + 2] += mom[1];
                        pl[6 * z + 3] += mom[2];
                        pl[6 * z + 4] += mom[3];
                        pl[6 * z + 5] += mom[0] - 1.0;
                    }
                }
        double *tmp = f; f = g; g = tmp; /* f: the newest state */
        if (check) {
            for (int k = 0; k < 6; k++) sums[k] = 0.0;
            for (int z = 0; z < nz; z++) for (int k = 0; k < 6; k++) sums[k] += pl[6 * z + k];
            if (!isfinite(sums[0]) || !isfinite(sums[1]) || !isfinite(sums[2])) { diverged = 1; break; }
            if (t % check_every == 0) {
                resid = sqrt(sums[0]) / ((double)check_every * sqrt(sums[1]));
                memcpy(uprev, ucur, (size_t)nvox * 3 * sizeof(double));
                if (fixed_steps <= 0 && resid < tol) { status = ORC_OK; break; }
            }
        }
    }
    if (f != f0) memcpy(f0, f, (size_t)nvox * 19 * sizeof(double));
    if (fixed_steps > 0) status = ORC_OK;
    if (u_out) {
        for (int64_t v = 0; v < 3 * nvox; v++) u_out[v] = 0.0;
        for (int64_t v = 0; v < nvox; v++)
            if (fluid[v]) for (int a = 0; a < 3; a++) u_out[a * nvox + v] = ucur[a * nvox + v];
    }
    double nu = (tau - 0.5) / 3.0;
    /* the driving: F_x, plus c_s^2 (rho_in - rho_out) over the distance between the
       ghost planes (nx + 1) with pressure boundaries */
    double drive = F[0] + (pressure ? (rho_in - rho_out) / (3.0 * (nx + 1)) : 0.0);
    out[0] = (double)t;
    out[1] = nu * (sums[2] / (double)nvox) / drive;
    out[2] = resid;
    out[3] = sums[2] / (double)nvox;
    out[4] = sums[3] / (double)nvox;
    out[5] = sums[4] / (double)nvox;
    out[6] = sums[5];
    out[7] = status == ORC_OK ? 1.0 : 0.0;
    (void)nfl;
    free(gbuf); free(uprev); free(ucur); free(pl);
    if (diverged) return ORC_E_DIVERGED;
    return status;
}

int orc_flow_solve(int nx, int ny, int nz, const uint8_t *fluid, double tau, int collision,
                   const double *F, int64_t max_steps, int64_t fixed_steps, int check_every,
                   double tol, const double *u_prev0, double *f, double *u_out, double *out) {
    return flow_solve_impl(nx, ny, nz, fluid, tau, collision, F, 0, 1.0, 1.0, max_steps,
                           fixed_steps, check_every, tol, u_prev0, f, u_out, out);
}

/*
 * The flow solve with pressure boundaries at x = -1 (rho_in) and x = nx (rho_out)
 * instead of periodic x (ghost planes as in ghost19; F may still add a body force).
 * k = nu <rho u_x> / (F_x + c_s^2 (rho_in - rho_out) / (nx + 1)), the pressure drop taken
 * between the ghost planes.  Otherwise as orc_flow_solve.
 */
int orc_flow_solve_p(int nx, int ny, int nz, const uint8_t *fluid, double tau, int collision,
                     const double *F, double rho_in, double rho_out, int64_t max_steps,
                     int64_t fixed_steps, int check_every, double tol, const double *u_prev0,
                     double *f, double *u_out, double *out) {
    return flow_solve_impl(nx, ny, nz, fluid, tau, collision, F, 1, rho_in, rho_out, max_steps,
                           fixed_steps, check_every, tol, u_prev0, f, u_out, out);
}

/*
 * One node's update from its sampled neighbourhood: nb_fluid[i] says whether
 * x - e_i is fluid, nb_f[19*i + k] holds the post-collision population k of
 * that neighbour (row 0 is the node itself).  Gives the node's new
 * post-collision populations (same streaming and collision as the solve).
 */
void orc_flow_update_node(const uint8_t *nb_fluid, const double *nb_f, double tau, int collision,
                          const double *F, double *fout, double *mom) {
    double fin[19];
    for (int i = 0; i < 19; i++) fin[i] = nb_fluid[i] ? nb_f[19 * i + i] : nb_f[opp19(i)];
    if (collision == 1) orc_collide19_mrt(fin, tau, NULL, F, fout, mom);
    else if (collision == 2) orc_collide19_trt(fin, tau, F, fout, mom);
    else orc_collide19(fin, tau, F, fout, mom);
}

/* ======================================================================
 * Section 3.2 (Eq. 10) on the D3Q7 lattice: rest weight 1/4, face weights 1/8
 * (reading; the paper defines the equilibrium only for D3Q19), so
 * g_eq,i = w_i C (the printed "C/a_i" read as w_i C) and c_s^2 = 1/4.
 * Boundaries (Section 3.3): bounce-back at solid links (no flux), periodic in
 * y and z, and in x ghost planes at x = -1 and x = nx holding the equilibrium
 * w_i C_in and w_i C_out ("the unknown distribution is determined using the
 * equilibrium distribution functions").
 * ====================================================================== */
static const int E7[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static double w7(int i) { return i == 0 ? 0.25 : 0.125; }
static int opp7(int i) { return i == 0 ? 0 : (i % 2 == 1 ? i + 1 : i - 1); }

void orc_collide7(const double *gin, double tau, double *gout, double *conc) {
    double c = 0.0;
    for (int i = 0; i < 7; i++) c += gin[i];
    for (int i = 0; i < 7; i++) gout[i] = gin[i] - (gin[i] - w7(i) * c) / tau;
    if (conc) *conc = c;
}

/* initial g = w_i C (C_init planar [N^3], zero when null) */
void orc_knudsen_init(int nx, int ny, int nz, const uint8_t *fluid, const double *c_init, double *g) {
    int64_t nvox = (int64_t)nx * ny * nz;
    for (int64_t v = 0; v < nvox; v++)
        for (int i = 0; i < 7; i++) g[7 * v + i] = (fluid[v] && c_init) ? w7(i) * c_init[v] : 0.0;
}

/*
 * The Knudsen solve: iterate stream + collide with the local tau_g (planar
 * [N^3], used at fluid voxels).  Checks as in the flow solve with C as the
 * field.  Fluxes leave from the post-collision state of the check step: the
 * outlet plane x = nx - 1/2 carries sum(g*_{+x}(nx-1) - w C_out), the inlet
 * plane x = -1/2 carries sum(w C_in - g*_{-x}(0)).  Eq. 14 read on the
 * lattice: D_eff = Phi_out / (ny nz) * (nx + 1) / (C_in - C_out), the
 * distance being that between the two ghost planes.
 * out: [0]=steps [1]=D_eff_lattice [2]=residual [3]=Phi_out [4]=Phi_in
 *      [5]=sum C [6]=converged.
 * c_out (nullable): C of the last step (0 at solids).
 * plane_flux (nullable, nx + 1 entries): Phi(x - 1/2) for x = 0..nx from the
 * final state, links with both ends fluid (ghost planes count as fluid).
 */
int orc_knudsen_solve(int nx, int ny, int nz, const uint8_t *fluid, const double *tau_g,
                      double c_in, double c_outv, int64_t max_steps, int64_t fixed_steps,
                      int check_every, double tol, const double *c_prev0, double *g,
                      double *c_out, double *plane_flux, double *out) {
    if (check_every < 1) return ORC_E_INVAL;
    int64_t nvox = (int64_t)nx * ny * nz;
    for (int64_t v = 0; v < nvox; v++)
        if (fluid[v] && !(tau_g[v] > 0.5)) return ORC_E_INVAL;
    double *g0 = g; /* the caller's buffer: holds the final state on return */
    double *h = (double *)malloc((size_t)nvox * 7 * sizeof(double));
    double *hbuf = h;
    double *cprev = (double *)calloc((size_t)nvox, sizeof(double));
    double *ccur = (double *)calloc((size_t)nvox, sizeof(double));
    double *pl = (double *)calloc((size_t)nz * 5, sizeof(double));
    if (!h || !cprev || !ccur || !pl) { free(h); free(cprev); free(ccur); free(pl); return ORC_E_NOMEM; }
    if (c_prev0) memcpy(cprev, c_prev0, (size_t)nvox * sizeof(double));
    int64_t limit = fixed_steps > 0 ? fixed_steps : max_steps;
    double resid = INFINITY, sums[5] = {0, 0, 0, 0, 0};
    int status = ORC_W_NOT_CONVERGED, diverged = 0;
    int64_t t = 0;
    while (t < limit) {
        t++;
        int check = (t % check_every == 0) || (t == limit);
        memset(pl, 0, (size_t)nz * 5 * sizeof(double));
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    int64_t v = vidx(x, y, z, nx, ny);
                    if (!fluid[v]) {
                        for (int i = 0; i < 7; i++) h[7 * v + i] = 0.0;
                        continue;
                    }
                    double gin[7], conc;
                    for (int i = 0; i < 7; i++) {
                        int sx = x - E7[i][0];
                        if (sx < 0) { gin[i] = w7(i) * c_in; continue; }
                        if (sx >= nx) { gin[i] = w7(i) * c_outv; continue; }
                        int64_t s = vidx(sx, wrap(y - E7[i][1], ny), wrap(z - E7[i][2], nz), nx, ny);
                        gin[i] = fluid[s] ? g[7 * s + i] : g[7 * v + opp7(i)];
                    }
                    orc_collide7(gin, tau_g[v], h + 7 * v, &conc);
                    if (check) {
                        ccur[v] = conc;
                        pl[5 * z + 0] += (conc - cprev[v]) * (conc - cprev[v]);
                        pl[5 * z + 1] += conc * conc;
                        if (x == nx - 1) pl[5 * z + 2] += h[7 * v + 1] - w7(1) * c_outv;
                        if (x == 0) pl[5 * z + 3] += w7(2) * c_in - h[7 * v + 2];
                        pl[5 * z + 4] += conc;
                    }
                }
        double *tmp = g; g = h; h = tmp;
        if (check) {
            for (int k = 0; k < 5; k++) sums[k] = 0.0;
            for (int z = 0; z < nz; z++) for (int k = 0; k < 5; k++) sums[k] += pl[5 * z + k];
            if (!isfinite(sums[0]) || !isfinite(sums[1]) || !isfinite(sums[2])) { diverged = 1; break; }
            if (t % check_every == 0) {
                resid = sqrt(sums[0]) / ((double)check_every * sqrt(sums[1]));
                memcpy(cprev, ccur, (size_t)nvox * sizeof(double));
                if (fixed_steps <= 0 && resid < tol) { status = ORC_OK; break; }
            }
        }
    }
    if (g != g0) memcpy(g0, g, (size_t)nvox * 7 * sizeof(double));
    if (fixed_steps > 0) status = ORC_OK;
    if (c_out) for (int64_t v = 0; v < nvox; v++) c_out[v] = fluid[v] ? ccur[v] : 0.0;
    if (plane_flux) {
        for (int px = 0; px <= nx; px++) {
            double s = 0.0;
            for (int z = 0; z < nz; z++)
                for (int y = 0; y < ny; y++) {
                    int left = px - 1, right = px; /* link from x = left to x = right */
                    int lf = left < 0 ? 1 : fluid[vidx(left, y, z, nx, ny)];
                    int rf = right >= nx ? 1 : fluid[vidx(right, y, z, nx, ny)];
                    if (!lf || !rf) continue;
                    double fwd = left < 0 ? w7(1) * c_in : g[7 * vidx(left, y, z, nx, ny) + 1];
                    double bwd = right >= nx ? w7(2) * c_outv : g[7 * vidx(right, y, z, nx, ny) + 2];
                    s += fwd - bwd;
                }
            plane_flux[px] = s;
        }
    }
    out[0] = (double)t;
    out[1] = sums[2] / ((double)ny * nz) * (double)(nx + 1) / (c_in - c_outv);
    out[2] = resid;
    out[3] = sums[2];
    out[4] = sums[3];
    out[5] = sums[4];
    out[6] = status == ORC_OK ? 1.0 : 0.0;
    free(hbuf); free(cprev); free(ccur); free(pl);
    if (diverged) return ORC_E_DIVERGED;
    return status;
}

/* One node's D3Q7 update from its neighbourhood: nb_kind[i] for x - e_i is
 * 0 fluid, 1 solid, 2 inlet ghost, 3 outlet ghost; nb_g[7*i + k] the
 * post-collision g_k of that neighbour (row 0 the node itself). */
void orc_knudsen_update_node(const uint8_t *nb_kind, const double *nb_g, double tau, double c_in,
                             double c_outv, double *gout, double *conc) {
    double gin[7];
    for (int i = 0; i < 7; i++) {
        switch (nb_kind[i]) {
        case 0: gin[i] = nb_g[7 * i + i]; break;
        case 1: gin[i] = nb_g[opp7(i)]; break;
        case 2: gin[i] = w7(i) * c_in; break;
        default: gin[i] = w7(i) * c_outv; break;
        }
    }
    orc_collide7(gin, tau, gout, conc);
}

/* ======================================================================
 * Section 3.2 (Eq. 10) on the paper's own D3Q19 lattice: g_eq,i = a_i C with
 * a_0 = 1/3, a_1..6 = 1/18, a_7..18 = 1/36 (the printed "C/a_i" read as a_i C),
 * velocities as in the flow lattice, D = (tau_g - 1/2)/3 (c_s^2 = 1/3).  The
 * same boundaries as the D3Q7 solve: bounce-back at solid links, periodic in y
 * and z, ghost planes at x = -1 and x = nx holding a_i C_in and a_i C_out (a
 * population arriving from beyond an x face takes the ghost's value whatever
 * its y, z offset, the ghost planes being uniform).
 * ====================================================================== */
void orc_collide19_diff(const double *gin, double tau, double *gout, double *conc) {
    double c = 0.0;
    for (int i = 0; i < 19; i++) c += gin[i];
    for (int i = 0; i < 19; i++) gout[i] = gin[i] - (gin[i] - w19(i) * c) / tau;
    if (conc) *conc = c;
}

/* initial g = a_i C (C_init planar [N^3], zero when null) */
void orc_diffusion19_init(int nx, int ny, int nz, const uint8_t *fluid, const double *c_init,
                          double *g) {
    int64_t nvox = (int64_t)nx * ny * nz;
    for (int64_t v = 0; v < nvox; v++)
        for (int i = 0; i < 19; i++)
            g[19 * v + i] = (fluid[v] && c_init) ? w19(i) * c_init[v] : 0.0;
}

/*
 * The D3Q19 diffusion solve, as orc_knudsen_solve (same checks, outputs and
 * Eq. 14 reading).  The net flux into the outlet ghost plane is, over the
 * fluid nodes at x = nx - 1, the sum of their post-collision populations with
 * e_x = +1 less the ghost's populations with e_x = -1 arriving there (each
 * a_i C_out; the five of them weigh 1/6); the inlet likewise.  plane_flux:
 * over the links crossing x - 1/2 (the five directions with e_x = +1) whose
 * two ends are fluid (ghost planes count as fluid), g_i(left) - g_opp(i)(right).
 */
int orc_diffusion19_solve(int nx, int ny, int nz, const uint8_t *fluid, const double *tau_g,
                          double c_in, double c_outv, int64_t max_steps, int64_t fixed_steps,
                          int check_every, double tol, const double *c_prev0, double *g,
                          double *c_out, double *plane_flux, double *out) {
    if (check_every < 1) return ORC_E_INVAL;
    int64_t nvox = (int64_t)nx * ny * nz;
    for (int64_t v = 0; v < nvox; v++)
        if (fluid[v] && !(tau_g[v] > 0.5)) return ORC_E_INVAL;
    double *g0 = g;
    double *h = (double *)malloc((size_t)nvox * 19 * sizeof(double));
    double *hbuf = h;
    double *cprev = (double *)calloc((size_t)nvox, sizeof(double));
    double *ccur = (double *)calloc((size_t)nvox, sizeof(double));
    double *pl = (double *)calloc((size_t)nz * 5, sizeof(double));
    if (!h || !cprev || !ccur || !pl) { free(h); free(cprev); free(ccur); free(pl); return ORC_E_NOMEM; }
    if (c_prev0) memcpy(cprev, c_prev0, (size_t)nvox * sizeof(double));
    const double a_side = 1.0 / 6.0; /* the five populations with e_x = +1 (or -1) together */
    int64_t limit = fixed_steps > 0 ? fixed_steps : max_steps;
    double resid = INFINITY, sums[5] = {0, 0, 0, 0, 0};
    int status = ORC_W_NOT_CONVERGED, diverged = 0;
    int64_t t = 0;
    while (t < limit) {
        t++;
        int check = (t % check_every == 0) || (t == limit);
        memset(pl, 0, (size_t)nz * 5 * sizeof(double));
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    int64_t v = vidx(x, y, z, nx, ny);
                    if (!fluid[v]) {
                        for (int i = 0; i < 19; i++) h[19 * v + i] = 0.0;
                        continue;
                    }
                    double gin[19], conc;
                    for (int i = 0; i < 19; i++) {
                        int sx = x - E19[i][0];
                        if (sx < 0) { gin[i] = w19(i) * c_in; continue; }
                        if (sx >= nx) { gin[i] = w19(i) * c_outv; continue; }
                        int64_t s = vidx(sx, wrap(y - E19[i][1], ny), wrap(z - E19[i][2], nz), nx, ny);
                        gin[i] = fluid[s] ? g[19 * s + i] : g[19 * v + opp19(i)];
                    }
                    orc_collide19_diff(gin, tau_g[v], h + 19 * v, &conc);
                    if (check) {
                        ccur[v] = conc;
                        pl[5 * z + 0] += (conc - cprev[v]) * (conc - cprev[v]);
                        pl[5 * z + 1] += conc * conc;
                        double plus = 0.0, minus = 0.0;
                        for (int i = 1; i < 19; i++) {
                            if (E19[i][0] == 1) plus += h[19 * v + i];
                            if (E19[i][0] == -1) minus += h[19 * v + i];
                        }
                        if (x == nx - 1) pl[5 * z + 2] += plus - a_side * c_outv;
                        if (x == 0) pl[5 * z + 3] += a_side * c_in - minus;
                        pl[5 * z + 4] += conc;
                    }
                }
        double *tmp = g; g = h; h = tmp;
        if (check) {
            for (int k = 0; k < 5; k++) sums[k] = 0.0;
            for (int z = 0; z < nz; z++) for (int k = 0; k < 5; k++) sums[k] += pl[5 * z + k];
            if (!isfinite(sums[0]) || !isfinite(sums[1]) || !isfinite(sums[2])) { diverged = 1; break; }
            if (t % check_every == 0) {
                resid = sqrt(sums[0]) / ((double)check_every * sqrt(sums[1]));
                memcpy(cprev, ccur, (size_t)nvox * sizeof(double));
                if (fixed_steps <= 0 && resid < tol) { status = ORC_OK; break; }
            }
        }
    }
    if (g != g0) memcpy(g0, g, (size_t)nvox * 19 * sizeof(double));
    if (fixed_steps > 0) status = ORC_OK;
    if (c_out) for (int64_t v = 0; v < nvox; v++) c_out[v] = fluid[v] ? ccur[v] : 0.0;
    if (plane_flux) {
        for (int px = 0; px <= nx; px++) {
            double s = 0.0;
            for (int z = 0; z < nz; z++)
                for (int y = 0; y < ny; y++) {
                    int right = px; /* the right end at (px, y, z) */
                    int rf = right >= nx ? 1 : fluid[vidx(right, y, z, nx, ny)];
                    if (!rf) continue;
                    for (int i = 1; i < 19; i++) {
                        if (E19[i][0] != 1) continue;
                        int left = px - 1, ly = wrap(y - E19[i][1], ny), lz = wrap(z - E19[i][2], nz);
                        int lf = left < 0 ? 1 : fluid[vidx(left, ly, lz, nx, ny)];
                        if (!lf) continue;
                        double fwd = left < 0 ? w19(i) * c_in : g[19 * vidx(left, ly, lz, nx, ny) + i];
                        double bwd = right >= nx ? w19(opp19(i)) * c_outv
                                                 : g[19 * vidx(right, y, z, nx, ny) + opp19(i)];
                        s += fwd - bwd;
                    }
                }
            plane_flux[px] = s;
        }
    }
    out[0] = (double)t;
    out[1] = sums[2] / ((double)ny * nz) * (double)(nx + 1) / (c_in - c_outv);
    out[2] = resid;
    out[3] = sums[2];
    out[4] = sums[3];
    out[5] = sums[4];
    out[6] = status == ORC_OK ? 1.0 : 0.0;
    free(hbuf); free(cprev); free(ccur); free(pl);
    if (diverged) return ORC_E_DIVERGED;
    return status;
}

/* One node's D3Q19 diffusion update from its neighbourhood (nb_kind, nb_g as in
 * orc_knudsen_update_node with 19 rows of 19). */
void orc_diffusion19_update_node(const uint8_t *nb_kind, const double *nb_g, double tau,
                                 double c_in, double c_outv, double *gout, double *conc) {
    double gin[19];
    for (int i = 0; i < 19; i++) {
        switch (nb_kind[i]) {
        case 0: gin[i] = nb_g[19 * i + i]; break;
        case 1: gin[i] = nb_g[opp19(i)]; break;
        case 2: gin[i] = w19(i) * c_in; break;
        default: gin[i] = w19(i) * c_outv; break;
        }
    }
    orc_collide19_diff(gin, tau, gout, conc);
}

/* ======================================================================
 * Eq. 11: Knudsen diffusivity of a pore of diameter d (m), gas of molar mass
 * M (kg/mol) at temperature T (K); R = 8.314462618 J/(mol K).
 * ====================================================================== */
double orc_knudsen_diffusivity(double d, double T, double M) {
    return d / 3.0 * sqrt(8.0 * 8.314462618 * T / (ORC_PI * M));
}

/* Eq. 29: mean free path */
double orc_mean_free_path(double mu, double p, double T, double M) {
    return mu / p * sqrt(ORC_PI * 8.314462618 * T / (2.0 * M));
}

/* Eq. 26: correction factor between apparent and intrinsic permeability */
double orc_fc_dgm(double Deff, double mu, double k, double P) { return 1.0 + Deff * mu / (k * P); }

/* Eq. 17: Kozeny-Carman permeability with A = d^2/180 */
double orc_k_kozeny_carman(double d, double eps) {
    return d * d / 180.0 * eps * eps * eps / ((1.0 - eps) * (1.0 - eps));
}

/* ======================================================================
 * Section 3.2 and Eq. 15: the lattice diffusivity of a mass-transport
 * lattice, D_L = c_s^2 (tau - 1/2), with c_s^2 = 1/4 on D3Q7 (rest weight
 * 1/4, face weights 1/8) and 1/3 on D3Q19.  Eq. 15 ties the lattice to
 * physical units through the reference pore: a pore of diameter d_ref
 * relaxes at tau_ref and diffuses at D_K(d_ref) (Eq. 11), so one time step
 * lasts dt = D_L(tau_ref) dx^2 / D_K,ref and a lattice diffusivity D turns
 * into D dx^2 / dt = D D_K,ref / D_L(tau_ref).
 * ====================================================================== */
double orc_lattice_diffusivity(double cs2, double tau) { return cs2 * (tau - 0.5); }

double orc_time_step(double cs2, double tau_ref, double dx_m, double dk_ref) {
    return orc_lattice_diffusivity(cs2, tau_ref) * dx_m * dx_m / dk_ref;
}

double orc_deff_physical(double deff_lattice, double cs2, double tau_ref, double dk_ref) {
    return deff_lattice * dk_ref / orc_lattice_diffusivity(cs2, tau_ref);
}

/* Eq. 16 (Bruggeman form D_eff = (eps / tau) D): tortuosity from the effective
 * and the free diffusivity at the same reference, both in lattice units. */
double orc_tortuosity(double eps, double d_free, double deff) { return eps * d_free / deff; }

/* Section 4.2: the exponent of D_eff / D = eps^alpha */
double orc_bruggeman_alpha(double deff_over_d, double eps) { return log(deff_over_d) / log(eps); }

/* Eq. 15 for the flow lattice: lengths scale with dx, so k (an area) with dx^2;
 * one millidarcy is 9.869233e-16 m^2 */
double orc_k_physical(double k_lattice, double dx_m) { return k_lattice * dx_m * dx_m; }
double orc_m2_to_mD(double k_m2) { return k_m2 / 9.869233e-16; }

/* the number of OpenMP threads the per-voxel loops use */
#ifdef _OPENMP
#include <omp.h>
#endif
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
