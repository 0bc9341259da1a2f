// Application of the Brillouin operator (Eq. def_pref, c_SW = 0):
//   (D psi)(x) = (lambda_0 + m) psi(x)
//              + sum_{n != 0} [lambda_k + rho_k sum_mu n_mu gamma_mu] W(x,x+n) psi(x+n)
// Two variants:
//  * STORED: W read from a precomputed store of 80 offsets, or of the 40
//    offsets with last non-zero component +1, the others via
//    W(x, x+n) = W(x+n, x)^dag (Sec. 5.1 paths reversed).
//  * RECOMPUTE: W rebuilt inside the kernel from the links, orthant by
//    orthant of the 3^4 neighbourhood (see k_apply_recompute).
// D^dag is the same stencil with rho_k -> -rho_k (gamma5-hermiticity, Sec. 1).
#include "common.h"
#include "kernels.h"
#include "apply_recompute.h"

namespace bri {

// ---------------------------------------------------------------- launchers
namespace {

template <typename LS, typename SS, typename A>
hipError_t launch_recompute(const Geom &g, const void *U, const void *in, void *out, double diag,
                            int nrhs, bool dag, hipStream_t st) {
    // element planes are addressed with 32-bit byte offsets
    if ((size_t)g.V * sizeof(LS) >= ((size_t)1 << 32) || (size_t)g.V * sizeof(SS) >= ((size_t)1 << 32))
        return hipErrorInvalidValue;
    dim3 grid((g.V + 15) / 16, nrhs);  // 16 sites per workgroup
    int gy, gz;
    strip_groups(g, gy, gz);
    if (dag)
        hipLaunchKernelGGL((k_apply_recompute<LS, SS, A, true>), grid, dim3(16 * recompute_tps<A>()), 0, st, g,
                           (const LS *)U, (const SS *)in, (SS *)out, (A)diag, gy, gz);
    else
        hipLaunchKernelGGL((k_apply_recompute<LS, SS, A, false>), grid, dim3(16 * recompute_tps<A>()), 0, st, g,
                           (const LS *)U, (const SS *)in, (SS *)out, (A)diag, gy, gz);
    return hipGetLastError();
}
}  // namespace

hipError_t apply_stored(const Geom &g, int noff, int wp, int sp, int kernel, int rblk, const void *W,
                        const void *in, void *out, double diag, int nrhs, bool dag, hipStream_t st,
                        const double *table) {
    if (wp == 0 && sp == 0) return apply_stored_f64(g, noff, kernel, rblk, W, in, out, diag, nrhs, dag, st, table);
    if (wp == 1 && sp == 1) return apply_stored_f32(g, noff, kernel, rblk, W, in, out, diag, nrhs, dag, st, table);
    if (wp == 2 && sp == 1) return apply_stored_f16(g, noff, kernel, rblk, W, in, out, diag, nrhs, dag, st, table);
    if (wp == 2 && sp == 2)
        return apply_stored_f16h(g, noff, kernel, rblk, W, in, out, diag, nrhs, dag, st, table);
    return hipErrorInvalidValue;
}

hipError_t apply_recompute(const Geom &g, int up, int sp, const void *U, const void *in, void *out,
                           double diag, int nrhs, bool dag, hipStream_t st) {
    if (up == 0 && sp == 0)
        return launch_recompute<double2, double2, double>(g, U, in, out, diag, nrhs, dag, st);
    if (up == 1 && sp == 1)
        return launch_recompute<float2, float2, float>(g, U, in, out, diag, nrhs, dag, st);
    return hipErrorInvalidValue;
}

}  // namespace bri
