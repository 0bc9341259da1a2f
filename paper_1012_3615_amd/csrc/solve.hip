// CG on the normal equations (placeholder until the solver lands).
#include "abi_internal.h"
#include "kernels.h"

using namespace bri;

extern "C" {
size_t bri_solve_workspace_bytes(bri_dims, const bri_solve_params *, int32_t) { return 0; }
bri_status bri_solve_cgne(bri_dims, const bri_solve_params *, const void *, const void *, double,
                          const double *, double *, int32_t, void *, size_t, bri_solve_stats *,
                          void *) {
    g_last_error.clear();
    return fail(BRI_E_UNSUPPORTED, "solver not built");
}
bri_status bri_dot(bri_dims, int32_t, const double *, const double *, double *, void *) {
    g_last_error.clear();
    return fail(BRI_E_UNSUPPORTED, "dot not built");
}
}
