// Ragged batches of expansion problems (placeholder until the batched runner lands).
#include "fx_internal.h"

struct fx_batch {
    int n = 0;
};

extern "C" {
fx_status fx_batch_create(const fx_problem* probs, int32_t n, fx_batch** out) {
    (void)probs; (void)n; (void)out;
    fx::set_error("batches are not implemented yet");
    return FX_EUNSUPPORTED;
}
fx_status fx_batch_destroy(fx_batch* b) { delete b; return FX_OK; }
fx_status fx_batch_run(fx_batch* b, const void* const* psi0, void* const* psi_out, void* const* rho_out, void* stream) {
    (void)b; (void)psi0; (void)psi_out; (void)rho_out; (void)stream;
    fx::set_error("batches are not implemented yet");
    return FX_EUNSUPPORTED;
}
}
