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
#include "apply_kernels.h"

namespace bri {

// ---------------------------------------------------------------- launchers
namespace {
constexpr int kBlock = 256;

template <int NOFF, typename WS, typename SS, typename A, int R>
hipError_t launch_stored_r(const Geom &g, const void *W, const void *in, void *out, double diag,
                           int nrhs, bool dag, hipStream_t st) {
    dim3 grid((g.V + kBlock - 1) / kBlock, (nrhs + R - 1) / R);
    if (dag)
        hipLaunchKernelGGL((k_apply_stored<NOFF, WS, SS, A, true, R>), grid, dim3(kBlock), 0, st, g,
                           (const WS *)W, (const SS *)in, (SS *)out, (A)diag, nrhs);
    else
        hipLaunchKernelGGL((k_apply_stored<NOFF, WS, SS, A, false, R>), grid, dim3(kBlock), 0, st,
                           g, (const WS *)W, (const SS *)in, (SS *)out, (A)diag, nrhs);
    return hipGetLastError();
}

template <int NOFF, typename WS, typename SS, typename A, int TX, int TY>
hipError_t launch_tiled_t(const Geom &g, const void *W, const void *in, void *out, double diag,
                          int nrhs, bool dag, hipStream_t st) {
    const int ntx = (g.L[0] + TX - 1) / TX, nty = (g.L[1] + TY - 1) / TY;
    dim3 grid(ntx * nty * g.L[2] * g.L[3], nrhs);
    if (dag)
        hipLaunchKernelGGL((k_apply_tiled<NOFF, WS, SS, A, true, TX, TY>), grid, dim3(TX * TY), 0, st,
                           g, ntx, nty, (const WS *)W, (const SS *)in, (SS *)out, (A)diag);
    else
        hipLaunchKernelGGL((k_apply_tiled<NOFF, WS, SS, A, false, TX, TY>), grid, dim3(TX * TY), 0,
                           st, g, ntx, nty, (const WS *)W, (const SS *)in, (SS *)out, (A)diag);
    return hipGetLastError();
}

template <int NOFF, typename WS, typename SS, typename A>
hipError_t launch_stored(const Geom &g, const void *W, const void *in, void *out, double diag,
                         int nrhs, int rblk, bool dag, hipStream_t st) {
    if (rblk == 0) {  // LDS-tiled kernel, one right-hand side per thread
        if (g.L[0] <= 16)
            return launch_tiled_t<NOFF, WS, SS, A, 16, 16>(g, W, in, out, diag, nrhs, dag, st);
        return launch_tiled_t<NOFF, WS, SS, A, 32, 8>(g, W, in, out, diag, nrhs, dag, st);
    }
    switch (rblk) {
        case 1: return launch_stored_r<NOFF, WS, SS, A, 1>(g, W, in, out, diag, nrhs, dag, st);
        case 2: return launch_stored_r<NOFF, WS, SS, A, 2>(g, W, in, out, diag, nrhs, dag, st);
        case 3: return launch_stored_r<NOFF, WS, SS, A, 3>(g, W, in, out, diag, nrhs, dag, st);
        case 4: return launch_stored_r<NOFF, WS, SS, A, 4>(g, W, in, out, diag, nrhs, dag, st);
        case 6: return launch_stored_r<NOFF, WS, SS, A, 6>(g, W, in, out, diag, nrhs, dag, st);
        case 12: return launch_stored_r<NOFF, WS, SS, A, 12>(g, W, in, out, diag, nrhs, dag, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename WS, typename SS, typename A>
hipError_t launch_stored_any(const Geom &g, int noff, const void *W, const void *in, void *out,
                             double diag, int nrhs, int rblk, bool dag, hipStream_t st) {
    if (noff == 80) return launch_stored<80, WS, SS, A>(g, W, in, out, diag, nrhs, rblk, dag, st);
    return launch_stored<40, WS, SS, A>(g, W, in, out, diag, nrhs, rblk, dag, st);
}

template <typename LS, typename SS, typename A>
hipError_t launch_recompute(const Geom &g, const void *U, const void *in, void *out, double diag,
                            int nrhs, bool dag, hipStream_t st) {
    dim3 grid((g.V + kBlock - 1) / kBlock, nrhs);
    if (dag)
        hipLaunchKernelGGL((k_apply_recompute<LS, SS, A, true>), grid, dim3(kBlock), 0, st, g,
                           (const LS *)U, (const SS *)in, (SS *)out, (A)diag);
    else
        hipLaunchKernelGGL((k_apply_recompute<LS, SS, A, false>), grid, dim3(kBlock), 0, st, g,
                           (const LS *)U, (const SS *)in, (SS *)out, (A)diag);
    return hipGetLastError();
}
}  // namespace

hipError_t apply_stored(const Geom &g, int noff, int wp, int sp, const void *W, const void *in,
                        void *out, double diag, int nrhs, int rblk, bool dag, hipStream_t st) {
    if (wp == 0 && sp == 0)
        return launch_stored_any<double2, double2, double>(g, noff, W, in, out, diag, nrhs, rblk, dag, st);
    if (wp == 1 && sp == 1)
        return launch_stored_any<float2, float2, float>(g, noff, W, in, out, diag, nrhs, rblk, dag, st);
    if (wp == 2 && sp == 1)
        return launch_stored_any<__half2, float2, float>(g, noff, W, in, out, diag, nrhs, rblk, dag, st);
    if (wp == 2 && sp == 2)
        return launch_stored_any<__half2, __half2, float>(g, noff, W, in, out, diag, nrhs, rblk, dag, st);
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
