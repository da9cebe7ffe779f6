// Projected solvers (Algorithms 1 and 2) and the IRLS step -- placeholder entry points.
#include "common.h"

using namespace ff;

extern "C" {

ff_status ff_workspace_size(ff_spectra h, int32_t which, int32_t solver, int32_t tp, size_t *bytes) {
  (void)h; (void)which; (void)solver; (void)tp; (void)bytes;
  return fail(FF_ENOTIMPL, "ff_workspace_size: not implemented yet");
}

ff_status gkb_project(ff_spectra h, const double *r_tilde, const double *wd, const double *winv, int32_t t,
                      int32_t tp, int32_t alpha_mode, double *y, double *alpha, double *sigma, void *workspace,
                      size_t ws_bytes, ff_stream stream) {
  return fail(FF_ENOTIMPL, "gkb_project: not implemented yet");
}

ff_status rsvd_project(ff_spectra h, const double *r_tilde, const double *wd, const double *winv, int32_t t,
                       int32_t tp, const double *omega, int32_t alpha_mode, double *y, double *alpha,
                       double *sigma, void *workspace, size_t ws_bytes, ff_stream stream) {
  return fail(FF_ENOTIMPL, "rsvd_project: not implemented yet");
}

ff_status irls_step(ff_spectra h, const ff_irls_params *p, const double *d_obs, const double *wd,
                    const double *m_prev, const double *m_prev2, const double *omega, double *m_new,
                    double *alpha, double *chi2_scaled, void *workspace, size_t ws_bytes, ff_stream stream) {
  return fail(FF_ENOTIMPL, "irls_step: not implemented yet");
}

}  // extern "C"
