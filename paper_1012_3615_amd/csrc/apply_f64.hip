// Stored-transporter apply instantiated for W storage double2, spinor storage
// double2 and double accumulation.
#include "apply_launch.h"
#include "kernels.h"

namespace bri {

hipError_t apply_stored_f64(const Geom &g, int noff, int kernel, int rblk, const void *W,
                             const void *in, void *out, double diag, int nrhs, bool dag,
                             hipStream_t st, const double *table) {
    if (noff == 80)
        return launch::stored<80, double2, double2, double>(g, kernel, rblk, W, in, out, diag, nrhs, dag, st, table);
    return launch::stored<40, double2, double2, double>(g, kernel, rblk, W, in, out, diag, nrhs, dag, st, table);
}

}  // namespace bri
