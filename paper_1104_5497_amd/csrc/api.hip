// api.hip -- argument checks, defaults and small utilities of the C ABI.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace nphc {

// Validates the host side of a batch.  mixed: more than one ring size.
int check_batch(const nphc_batch* b, bool* mixed, int* minN, int* maxN)
{
    if (!b || b->num_systems < 1 || !b->N_host || !b->path_off_host || !b->N || !b->path_off ||
        !b->J || !b->J_off || !b->gamma)
        return NPHC_EINVAL;
    int lo = 1 << 30, hi = 0;
    if (b->path_off_host[0] != 0) return NPHC_EINVAL;
    for (int s = 0; s < b->num_systems; ++s) {
        const int N = b->N_host[s];
        if (N < 2) return NPHC_EINVAL;
        if (N > NPHC_MAX_N) return NPHC_EUNSUPPORTED;
        if (s > 0 && N < b->N_host[s - 1]) return NPHC_EINVAL;  // sorted by ring size
        const int64_t paths = int64_t(1) << (2 * (N - 1));
        if (b->path_off_host[s + 1] - b->path_off_host[s] != paths) return NPHC_EINVAL;
        lo = N < lo ? N : lo;
        hi = N > hi ? N : hi;
    }
    *mixed = lo != hi;
    *minN = lo;
    *maxN = hi;
    return NPHC_OK;
}

}  // namespace nphc

extern "C" void nphc_default_track_opts(int precision, nphc_track_opts* o)
{
    if (!o) return;
    o->h0 = 0.01;
    o->hmax = 0.05;
    o->hmin = 1e-13;
    // tracking tolerance: float32 runs at its precision; float64 tracking
    // does not need more than 1e-8 since every endpoint is refined to 1e-15
    o->corr_tol = precision == NPHC_FP32 ? 1e-5 : 1e-8;
    o->R_inf = 1e5;
    o->t_stall = 1.0 - 1e-6;
    o->t_end = 1.0;
    // float32: two Newton iterations.  A wave runs as many iterations as its
    // slowest lane needs; a third one is rarely needed by any single path
    // (float64 residuals converge fast) but costs the whole wave a solve.
    // Measured on the N = 10 ring: launch 44 -> 39 ms, same solve and step
    // counts, same endpoints.  float64 tracking at its tighter tolerance
    // needs the third iteration.
    o->max_corr = precision == NPHC_FP32 ? 2 : 3;
    o->max_steps = 20000;
    o->predictor = 0;
    o->resume = 0;
    o->handoff_norm = 0.0;
    o->handoff_rejects = precision == NPHC_FP32 ? 8 : 0;
    o->pad = 0;
    o->t_endzone = 0.9;
    // float32: a step below 5% of 1 - t past the collapse norm means the
    // float32 Jacobian has run out of precision; the path goes on in float64
    o->hmin_rel = precision == NPHC_FP32 ? 0.05 : 1e-3;
    o->collapse_norm = 1e4;
    o->grow_ratio = 1.25;
    o->grow_cap = 0.5;
    o->grid_blocks = 0;
    o->handoff_steps = precision == NPHC_FP32 ? 200 : 0;
    o->pred_tol = 1e-3;
    o->step_ctrl = 0;
    o->lanes_per_path = 1;
    o->drain_steps = 0;
    o->pad3 = 0;
}

extern "C" void nphc_default_cert_opts(nphc_cert_opts* o)
{
    if (!o) return;
    o->max_iter = 20;
    o->lanes_per_item = 1;
    o->tol = 1e-15;
    o->res_tol = 1e-12;
    o->cond_max = 1e10;
    o->sing_res = 1e-8;
    o->div_norm = 1e4;
    o->real_tol = 1e-7;
}

extern "C" void nphc_default_class_opts(nphc_class_opts* o)
{
    if (!o) return;
    o->eig_rel = 1e-8;
    o->jacobi_sweeps = 30;
    o->pad = 0;
}

extern "C" const char* nphc_strerror(int code)
{
    switch (code) {
        case NPHC_OK: return "ok";
        case NPHC_EINVAL: return "invalid argument";
        case NPHC_EUNSUPPORTED: return "unsupported ring size or precision";
        case NPHC_EHIP: return "HIP error";
        case NPHC_EWORKSPACE: return "workspace too small or misaligned";
        default: return "unknown error";
    }
}

extern "C" const char* nphc_version(void) { return "nphc-mi355x 0.1 (gfx950)"; }
