// Production-operator and generic-class forms of the stored apply (two-row SU(3) transporters,
// clover term, coefficient table) instantiated for W storage double2, spinor storage double2 and double accumulation.
#include "apply_launch.h"
#include "kernels.h"

namespace bri {

hipError_t apply_prod_f64(const Geom &g, int rows, int rblk, const void *W, const void *in, void *out,
                          double diag, int nrhs, bool dag, hipStream_t st, const void *clover,
                          const double *table) {
    return launch::stored_prod<double2, double2, double>(g, rows, rblk, W, in, out, diag, nrhs, dag, st, clover, table);
}

}  // namespace bri
