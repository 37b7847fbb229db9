// Workspace sizing, the host-only property relations of Section 4, and the version.
#include <cmath>
#include <cstring>

#include "lbm_internal.h"

namespace lbm {
size_t label_ws_bytes_n(const int32_t n[3]);
size_t diam_ws_bytes_n(const int32_t n[3]);
size_t flow_ws_bytes_n(const int32_t n[3], int64_t nf, int32_t storage);
size_t knudsen_ws_bytes_n(const int32_t n[3], int64_t nf, int q);
}  // namespace lbm

using namespace lbm;

extern "C" lbm_status lbm_workspace_size(int32_t kind, const int32_t n[3], int64_t n_fluid,
                                         size_t *bytes_h) {
    LBM_REQUIRE(n && bytes_h, LBM_E_INVAL, "lbm_workspace_size: null argument");
    LBM_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1 && n[0] <= kMaxEdge && n[1] <= kMaxEdge &&
                    n[2] <= kMaxEdge,
                LBM_E_INVAL, "sizes must lie in [1, %d]", kMaxEdge);
    const int64_t nv = (int64_t)n[0] * n[1] * n[2];
    LBM_REQUIRE(n_fluid <= nv, LBM_E_INVAL, "more fluid nodes than voxels");
    switch (kind) {
    case LBM_WS_LABEL: *bytes_h = label_ws_bytes_n(n); return LBM_OK;
    case LBM_WS_PORE_DIAM: *bytes_h = diam_ws_bytes_n(n); return LBM_OK;
    case LBM_WS_FLOW: *bytes_h = flow_ws_bytes_n(n, n_fluid, LBM_STORE_FP32); return LBM_OK;
    case LBM_WS_FLOW_FP16: *bytes_h = flow_ws_bytes_n(n, n_fluid, LBM_STORE_FP16); return LBM_OK;
    case LBM_WS_FLOW_FP64: *bytes_h = flow_ws_bytes_n(n, n_fluid, LBM_STORE_FP64); return LBM_OK;
    case LBM_WS_KNUDSEN: *bytes_h = knudsen_ws_bytes_n(n, n_fluid, 7); return LBM_OK;
    case LBM_WS_KNUDSEN_D3Q19: *bytes_h = knudsen_ws_bytes_n(n, n_fluid, 19); return LBM_OK;
    default: break;
    }
    set_error("unknown workspace kind %d", kind);
    return LBM_E_INVAL;
}

// Section 4: Eq. 15 (units), Eq. 11 (D_K), Eq. 17 (Kozeny-Carman), the Bruggeman
// exponent of Section 4.2, Eq. 29 (mean free path) and Eq. 26 (f_c, apparent k).
extern "C" lbm_status lbm_props(const lbm_label_stats *g, const lbm_flow_result *f,
                                const lbm_knudsen_result *d, const lbm_props_params *p,
                                lbm_props_out *out) {
    LBM_REQUIRE(out && p, LBM_E_INVAL, "lbm_props: null argument");
    const double nan = std::nan("");
    const double R = 8.314462618, PI = 3.141592653589793;
    out->porosity = g ? g->porosity : nan;
    out->connectivity = g ? g->connectivity : nan;
    out->k_m2 = f ? f->k_m2 : nan;
    out->k_mD = f ? f->k_mD : nan;
    const double dm = p->d_mean_nm * 1e-9;
    const double eps = out->porosity;
    out->k_KC_m2 = g ? dm * dm / 180.0 * eps * eps * eps / ((1.0 - eps) * (1.0 - eps)) : nan;
    out->Deff_m2s = d ? d->Deff_m2s : nan;
    out->DK_ref_m2s = d ? d->DK_ref_m2s : nan;
    out->tortuosity = d ? d->tortuosity : nan;
    out->bruggeman_alpha = (d && g) ? std::log(d->Deff_over_DKref) / std::log(eps) : nan;
    out->mean_free_path_m = p->mu_Pa_s / p->P_Pa * std::sqrt(PI * R * p->T_K / (2.0 * p->M_kg_mol));
    out->fc_dgm = (d && f) ? 1.0 + d->Deff_m2s * p->mu_Pa_s / (f->k_m2 * p->P_Pa) : nan;
    out->k_apparent_m2 = (d && f) ? f->k_m2 * out->fc_dgm : nan;
    return LBM_OK;
}

extern "C" const char *lbm_version(void) { return "lbm-mi355x 0.1.0 (gfx950)"; }

// Streaming copy: one 16-byte element per thread, non-temporal load and store (the
// fastest of the plain copy shapes measured on MI355X; a grid-stride loop with four
// elements in flight per thread reached only two thirds of it).
typedef float lbm_f4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_probe(lbm_f4 *__restrict__ dst,
                                                    const lbm_f4 *__restrict__ src, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

extern "C" lbm_status lbm_copy_probe(void *dst, const void *src, size_t bytes, void *stream) {
    LBM_REQUIRE(dst && src, LBM_E_INVAL, "lbm_copy_probe: null buffer");
    LBM_REQUIRE(bytes % 16 == 0, LBM_E_INVAL, "lbm_copy_probe: size not a multiple of 16");
    const char *d = static_cast<const char *>(dst), *s = static_cast<const char *>(src);
    LBM_REQUIRE(d + bytes <= s || s + bytes <= d, LBM_E_INVAL, "lbm_copy_probe: buffers overlap");
    lbm_status st = check_device();
    if (st != LBM_OK) return st;
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return LBM_OK;
    LBM_REQUIRE((n + 255) / 256 <= (int64_t)0x7fffffff, LBM_E_INVAL, "lbm_copy_probe: too large");
    k_copy_probe<<<(unsigned)((n + 255) / 256), 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<lbm_f4 *>(dst), static_cast<const lbm_f4 *>(src), n);
    LBM_CHECK_LAUNCH();
    return LBM_OK;
}

extern "C" size_t lbm_sizeof(int32_t which) {
    switch (which) {
    case 0: return sizeof(lbm_recon_params);
    case 1: return sizeof(lbm_recon_stats);
    case 2: return sizeof(lbm_label_stats);
    case 3: return sizeof(lbm_flow_params);
    case 4: return sizeof(lbm_flow_result);
    case 5: return sizeof(lbm_knudsen_params);
    case 6: return sizeof(lbm_knudsen_result);
    case 7: return sizeof(lbm_props_params);
    case 8: return sizeof(lbm_props_out);
    case 9: return sizeof(lbm_batch_sched);
    default: return 0;
    }
}
