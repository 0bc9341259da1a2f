// Link gradient (placeholder until the adjoint lands).
#include "abi_internal.h"
#include "kernels.h"

using namespace bri;

extern "C" {
size_t bri_grad_workspace_bytes(bri_dims) { return 0; }
bri_status bri_grad_links(bri_dims, const double *, const double *, const double *, int32_t,
                          double *, void *, size_t, void *) {
    g_last_error.clear();
    return fail(BRI_E_UNSUPPORTED, "gradient not built");
}
}
