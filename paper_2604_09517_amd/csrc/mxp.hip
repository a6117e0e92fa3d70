// Mixed-precision solve (Sec. III-A.2, Sec. II-B): options and workspace.
#include <hip/hip_runtime.h>

#include "common.h"

extern "C" void mxp_default_opts(mxp_opts *o) {
    if (!o) return;
    o->prec = MXLU_PREC_BF16;
    o->pivot = 0;
    o->nb = 512;
    o->refine = MXLU_IR_GMRES;
    o->restart = 30;
    o->max_outer = 20;
    o->max_inner_total = 300;
    o->inner_tol = 1e-6;
    o->resid_threshold = 16.0;
    o->scale_tile = 128;
    o->reuse_factors = 0;
    o->trans = 0;
    o->x_init = 0;
}

extern "C" size_t mxp_workspace_bytes(int64_t n, const mxp_opts *o) {
    if (n < 0 || !o) return 0;
    return (size_t)n * (size_t)n * 2 + 256;
}

extern "C" int mxp_solve(int64_t, int64_t, const double *, int64_t, const double *, int64_t,
                         double *, int64_t, void *, size_t, int32_t *, const mxp_opts *,
                         mxp_report *, void *) {
    mxlu::set_error_msg("mxp_solve: mixed-precision path not available in this build");
    return MXLU_E_HIP;
}
