// Stored-transporter apply instantiated for W storage __half2, spinor storage
// float2 and float accumulation.
#include "apply_launch.h"
#include "kernels.h"

namespace bri {

hipError_t apply_stored_f16(const Geom &g, int noff, int kernel, int rblk, const void *W,
                             const void *in, void *out, double diag, int nrhs, bool dag,
                             hipStream_t st, const double *table) {
    if (noff == 80)
        return launch::stored<80, __half2, float2, float>(g, kernel, rblk, W, in, out, diag, nrhs, dag, st, table);
    return launch::stored<40, __half2, float2, float>(g, kernel, rblk, W, in, out, diag, nrhs, dag, st, table);
}

}  // namespace bri
