// ctmhd_adjoint.hip -- reverse-mode derivative of one CT-MHD step (C ABI
// entry point ctmhd_step_adjoint).
#include "ctmhd_host.h"

extern "C" {

int ctmhd_step_adjoint(const ctmhd_params* p, const ctmhd_box* box, const double* const cons_n[5],
                       const double* const bface_n[3], const double* dt,
                       const double* const g_cons[5], const double* const g_bface[3],
                       double* const g_cons_out[5], double* const g_bface_out[3], void* workspace,
                       size_t ws_bytes, void* stream) {
  (void)p; (void)box; (void)cons_n; (void)bface_n; (void)dt; (void)g_cons; (void)g_bface;
  (void)g_cons_out; (void)g_bface_out; (void)workspace; (void)ws_bytes; (void)stream;
  return fail(CTMHD_EUNSUPPORTED, "ctmhd_step_adjoint is not built yet");
}

}  // extern "C"
