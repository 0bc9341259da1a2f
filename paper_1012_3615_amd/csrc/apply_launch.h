// Launchers of the stored-transporter apply for one precision triple
// (storage of W, storage of the spinors, accumulation); each apply_*.hip
// translation unit instantiates one triple.
#pragma once
#include <type_traits>
#include "apply_gather.h"
#include "apply_tiled.h"

namespace bri {
namespace launch {

constexpr int kGatherBlock = 256;

template <int NOFF, typename WS, typename SS, typename A, int TX, int TY, int R, bool PF = false,
          bool UN = false, int ROWS = 3, bool CLV = false>
hipError_t tiled(const Geom &g, const void *W, const void *in, void *out, double diag, int nrhs,
                 bool dag, hipStream_t st, const void *clover = nullptr, const double *table = nullptr) {
    // the LDS of a workgroup is at most 160 KiB on gfx950
    constexpr size_t lds = sizeof(SS) * 12 * R * (TX + 2) * (TY + 2);
    if constexpr (lds > 160 * 1024) {
        return hipErrorInvalidValue;
    } else {
        const int ntx = (g.L[0] + TX - 1) / TX, nty = (g.L[1] + TY - 1) / TY;
        // one-dimensional grid, right-hand-side group fastest (see k_apply_tiled)
        dim3 grid(ntx * nty * g.L[2] * g.L[3] * ((nrhs + R - 1) / R));
        const Coef<A> cf = make_coef<A>(table);
        if (dag)
            hipLaunchKernelGGL((k_apply_tiled<NOFF, WS, SS, A, true, TX, TY, R, PF, UN, ROWS, CLV>), grid,
                               dim3(TX * TY), 0, st, g, ntx, nty, (const WS *)W, (const SS *)in, (SS *)out,
                               (A)diag, nrhs, (const SS *)clover, cf);
        else
            hipLaunchKernelGGL((k_apply_tiled<NOFF, WS, SS, A, false, TX, TY, R, PF, UN, ROWS, CLV>), grid,
                               dim3(TX * TY), 0, st, g, ntx, nty, (const WS *)W, (const SS *)in, (SS *)out,
                               (A)diag, nrhs, (const SS *)clover, cf);
        return hipGetLastError();
    }
}

template <int NOFF, typename WS, typename SS, typename A, int R>
hipError_t gather(const Geom &g, const void *W, const void *in, void *out, double diag, int nrhs,
                  bool dag, hipStream_t st, const double *table) {
    dim3 grid((g.V + kGatherBlock - 1) / kGatherBlock, (nrhs + R - 1) / R);
    const Coef<A> cf = make_coef<A>(table);
    if (dag)
        hipLaunchKernelGGL((k_apply_stored<NOFF, WS, SS, A, true, R>), grid, dim3(kGatherBlock), 0, st,
                           g, (const WS *)W, (const SS *)in, (SS *)out, (A)diag, nrhs, cf);
    else
        hipLaunchKernelGGL((k_apply_stored<NOFF, WS, SS, A, false, R>), grid, dim3(kGatherBlock), 0,
                           st, g, (const WS *)W, (const SS *)in, (SS *)out, (A)diag, nrhs, cf);
    return hipGetLastError();
}

// kernel: 0 gather (rblk in 1,2,3,4,6,12); 2..5 tiles 32x8, 16x16, 64x4, 16x8; 6, 7 tiles 32x8 and 16x16 with the
// next transporter prefetched; 8 tile 32x8 with prefetch and the offsets of a
// layer unrolled at compile time (rblk 1, 2); 9, 10 tiles 32x8 (rblk 1-3) and
// 16x8 (rblk 2-4) with the offsets unrolled, no prefetch; 11, 12 tiles 24x8 and 48x4 with prefetch and
// unrolled offsets (rblk 1, 2); 13, 14 tiles 32x16 and 16x4 with prefetch and unrolled offsets (rblk 1).  Tiles hold rblk in 1..4 right-hand sides per thread (16x16 and 64x4: 1;
// 32x8, 24x8 and 48x4 with prefetch: 1, 2).  The built-in choice (code 1)
// is resolved to one of these on the host before the launch.
template <int NOFF, typename WS, typename SS, typename A>
hipError_t stored(const Geom &g, int kernel, int rblk, const void *W, const void *in, void *out,
                  double diag, int nrhs, bool dag, hipStream_t st, const double *table) {
    if (kernel == 0) {
        switch (rblk) {
            case 1: return gather<NOFF, WS, SS, A, 1>(g, W, in, out, diag, nrhs, dag, st, table);
            case 2: return gather<NOFF, WS, SS, A, 2>(g, W, in, out, diag, nrhs, dag, st, table);
            case 3: return gather<NOFF, WS, SS, A, 3>(g, W, in, out, diag, nrhs, dag, st, table);
            case 4: return gather<NOFF, WS, SS, A, 4>(g, W, in, out, diag, nrhs, dag, st, table);
            case 6: return gather<NOFF, WS, SS, A, 6>(g, W, in, out, diag, nrhs, dag, st, table);
            case 12: return gather<NOFF, WS, SS, A, 12>(g, W, in, out, diag, nrhs, dag, st, table);
            default: return hipErrorInvalidValue;
        }
    }
    switch (kernel * 16 + rblk) {
        case 2 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 8, 1>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 2 * 16 + 2: return tiled<NOFF, WS, SS, A, 32, 8, 2>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 2 * 16 + 3: return tiled<NOFF, WS, SS, A, 32, 8, 3>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 2 * 16 + 4: return tiled<NOFF, WS, SS, A, 32, 8, 4>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 3 * 16 + 1: return tiled<NOFF, WS, SS, A, 16, 16, 1>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 4 * 16 + 1: return tiled<NOFF, WS, SS, A, 64, 4, 1>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 5 * 16 + 1: return tiled<NOFF, WS, SS, A, 16, 8, 1>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 5 * 16 + 2: return tiled<NOFF, WS, SS, A, 16, 8, 2>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 5 * 16 + 3: return tiled<NOFF, WS, SS, A, 16, 8, 3>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 5 * 16 + 4: return tiled<NOFF, WS, SS, A, 16, 8, 4>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 6 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 8, 1, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 6 * 16 + 2: return tiled<NOFF, WS, SS, A, 32, 8, 2, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 7 * 16 + 1: return tiled<NOFF, WS, SS, A, 16, 16, 1, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 8 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 8, 1, true, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 8 * 16 + 2: return tiled<NOFF, WS, SS, A, 32, 8, 2, true, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 9 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 8, 1, false, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 9 * 16 + 2: return tiled<NOFF, WS, SS, A, 32, 8, 2, false, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 9 * 16 + 3: return tiled<NOFF, WS, SS, A, 32, 8, 3, false, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 10 * 16 + 2: return tiled<NOFF, WS, SS, A, 16, 8, 2, false, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 10 * 16 + 3: return tiled<NOFF, WS, SS, A, 16, 8, 3, false, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 10 * 16 + 4: return tiled<NOFF, WS, SS, A, 16, 8, 4, false, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 11 * 16 + 1: return tiled<NOFF, WS, SS, A, 24, 8, 1, true, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 11 * 16 + 2: return tiled<NOFF, WS, SS, A, 24, 8, 2, true, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 12 * 16 + 1: return tiled<NOFF, WS, SS, A, 48, 4, 1, true, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 12 * 16 + 2: return tiled<NOFF, WS, SS, A, 48, 4, 2, true, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 13 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 16, 1, true, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        case 14 * 16 + 1: return tiled<NOFF, WS, SS, A, 16, 4, 1, true, true>(g, W, in, out, diag, nrhs, dag, st, nullptr, table);
        default: return hipErrorInvalidValue;
    }
}

// Production-operator forms and the generic class (80-offset store only):
// ROWS = 2 for the two-row store of back-projected transporters, CLV for the
// clover term; the coefficients come from `table` (lambda_0..4, rho_1..4 of
// the generic class of Sec. 8; nullptr: the Brillouin column).  The tile is
// the default one for the extent Lx (32x8 with prefetch and unrolled offsets,
// 24x8 or 48x4 when Lx is a multiple of 24 or 48 but not of 32, or 16x16 /
// 16x8 for Lx <= 16; the 32x16 tile of the plain FP32 apply was slower
// here); rblk 1 or 2 right-hand sides per thread.
template <typename WS, typename SS, typename A, int ROWS, bool CLV>
hipError_t stored_ext(const Geom &g, int rblk, const void *W, const void *in, void *out, double diag,
                      int nrhs, bool dag, hipStream_t st, const void *clover, const double *table) {
#define BRI_EXT(TX, TY, R, PF, UN) \
    tiled<80, WS, SS, A, TX, TY, R, PF, UN, ROWS, CLV>(g, W, in, out, diag, nrhs, dag, st, clover, table)
    const int lx = g.L[0];
    const bool small = lx <= 16;
    if (rblk != 1 && rblk != 2) return hipErrorInvalidValue;
    if (!small && lx % 32 != 0 && lx % 48 == 0) return rblk == 1 ? BRI_EXT(48, 4, 1, true, true) : BRI_EXT(48, 4, 2, true, true);
    if (!small && lx % 32 != 0 && lx % 24 == 0) return rblk == 1 ? BRI_EXT(24, 8, 1, true, true) : BRI_EXT(24, 8, 2, true, true);
    if (rblk == 1) return small ? BRI_EXT(16, 16, 1, true, false) : BRI_EXT(32, 8, 1, true, true);
    return small ? BRI_EXT(16, 8, 2, false, true) : BRI_EXT(32, 8, 2, true, true);
#undef BRI_EXT
}

// rows: 3 or 2; clover: nullptr for c_SW = 0; table: nullptr for the Brillouin column
template <typename WS, typename SS, typename A>
hipError_t stored_prod(const Geom &g, int rows, int rblk, const void *W, const void *in, void *out, double diag,
                       int nrhs, bool dag, hipStream_t st, const void *clover, const double *table) {
    if (rows == 3 && clover)
        return stored_ext<WS, SS, A, 3, true>(g, rblk, W, in, out, diag, nrhs, dag, st, clover, table);
    if (rows == 2 && clover)
        return stored_ext<WS, SS, A, 2, true>(g, rblk, W, in, out, diag, nrhs, dag, st, clover, table);
    if (rows == 2)
        return stored_ext<WS, SS, A, 2, false>(g, rblk, W, in, out, diag, nrhs, dag, st, nullptr, table);
    return hipErrorInvalidValue;  // rows 3 without a clover term: stored()
}

}  // namespace launch
}  // namespace bri
