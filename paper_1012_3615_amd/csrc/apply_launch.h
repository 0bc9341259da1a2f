// Launchers of the stored-transporter apply for one precision triple
// (storage of W, storage of the spinors, accumulation); each apply_*.hip
// translation unit instantiates one triple.
#pragma once
#include "apply_gather.h"
#include "apply_tiled.h"

namespace bri {
namespace launch {

constexpr int kGatherBlock = 256;

template <int NOFF, typename WS, typename SS, typename A, int TX, int TY, int R, bool PF = false,
          bool UN = false>
hipError_t tiled(const Geom &g, const void *W, const void *in, void *out, double diag, int nrhs,
                 bool dag, hipStream_t st) {
    // the LDS of a workgroup is at most 160 KiB on gfx950
    constexpr size_t lds = sizeof(SS) * 12 * R * (TX + 2) * (TY + 2);
    if constexpr (lds > 160 * 1024) {
        return hipErrorInvalidValue;
    } else {
        const int ntx = (g.L[0] + TX - 1) / TX, nty = (g.L[1] + TY - 1) / TY;
        // one-dimensional grid, right-hand-side group fastest (see k_apply_tiled)
        dim3 grid(ntx * nty * g.L[2] * g.L[3] * ((nrhs + R - 1) / R));
        if (dag)
            hipLaunchKernelGGL((k_apply_tiled<NOFF, WS, SS, A, true, TX, TY, R, PF, UN>), grid, dim3(TX * TY),
                               0, st, g, ntx, nty, (const WS *)W, (const SS *)in, (SS *)out, (A)diag,
                               nrhs);
        else
            hipLaunchKernelGGL((k_apply_tiled<NOFF, WS, SS, A, false, TX, TY, R, PF, UN>), grid, dim3(TX * TY),
                               0, st, g, ntx, nty, (const WS *)W, (const SS *)in, (SS *)out, (A)diag,
                               nrhs);
        return hipGetLastError();
    }
}

template <int NOFF, typename WS, typename SS, typename A, int R>
hipError_t gather(const Geom &g, const void *W, const void *in, void *out, double diag, int nrhs,
                  bool dag, hipStream_t st) {
    dim3 grid((g.V + kGatherBlock - 1) / kGatherBlock, (nrhs + R - 1) / R);
    if (dag)
        hipLaunchKernelGGL((k_apply_stored<NOFF, WS, SS, A, true, R>), grid, dim3(kGatherBlock), 0, st,
                           g, (const WS *)W, (const SS *)in, (SS *)out, (A)diag, nrhs);
    else
        hipLaunchKernelGGL((k_apply_stored<NOFF, WS, SS, A, false, R>), grid, dim3(kGatherBlock), 0,
                           st, g, (const WS *)W, (const SS *)in, (SS *)out, (A)diag, nrhs);
    return hipGetLastError();
}

// kernel: 0 gather (rblk in 1,2,3,4,6,12); 1 tiles with the shape chosen from
// Lx; 2..5 tiles 32x8, 16x16, 64x4, 16x8; 6, 7 tiles 32x8 and 16x16 with the
// next transporter prefetched; 8 tile 32x8 with prefetch and the offsets of a
// layer unrolled at compile time (rblk 1, 2); 9, 10 tiles 32x8 (rblk 1-3) and
// 16x8 (rblk 2-4) with the offsets unrolled, no prefetch.  Tiles hold rblk in 1..4 right-hand sides per
// thread (16x16 and 64x4: 1; 32x8 with prefetch: 1, 2).
template <int NOFF, typename WS, typename SS, typename A>
hipError_t stored(const Geom &g, int kernel, int rblk, const void *W, const void *in, void *out,
                  double diag, int nrhs, bool dag, hipStream_t st) {
    if (kernel == 0) {
        switch (rblk) {
            case 1: return gather<NOFF, WS, SS, A, 1>(g, W, in, out, diag, nrhs, dag, st);
            case 2: return gather<NOFF, WS, SS, A, 2>(g, W, in, out, diag, nrhs, dag, st);
            case 3: return gather<NOFF, WS, SS, A, 3>(g, W, in, out, diag, nrhs, dag, st);
            case 4: return gather<NOFF, WS, SS, A, 4>(g, W, in, out, diag, nrhs, dag, st);
            case 6: return gather<NOFF, WS, SS, A, 6>(g, W, in, out, diag, nrhs, dag, st);
            case 12: return gather<NOFF, WS, SS, A, 12>(g, W, in, out, diag, nrhs, dag, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (kernel == 1) {
        // default shapes: transporter prefetch where it is instantiated
        if (g.L[0] <= 16)
            kernel = rblk == 1 ? 7 : 10;
        else
            kernel = rblk <= 2 ? 8 : rblk == 3 ? 9 : 2;
    }
    switch (kernel * 16 + rblk) {
        case 2 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 8, 1>(g, W, in, out, diag, nrhs, dag, st);
        case 2 * 16 + 2: return tiled<NOFF, WS, SS, A, 32, 8, 2>(g, W, in, out, diag, nrhs, dag, st);
        case 2 * 16 + 3: return tiled<NOFF, WS, SS, A, 32, 8, 3>(g, W, in, out, diag, nrhs, dag, st);
        case 2 * 16 + 4: return tiled<NOFF, WS, SS, A, 32, 8, 4>(g, W, in, out, diag, nrhs, dag, st);
        case 3 * 16 + 1: return tiled<NOFF, WS, SS, A, 16, 16, 1>(g, W, in, out, diag, nrhs, dag, st);
        case 4 * 16 + 1: return tiled<NOFF, WS, SS, A, 64, 4, 1>(g, W, in, out, diag, nrhs, dag, st);
        case 5 * 16 + 1: return tiled<NOFF, WS, SS, A, 16, 8, 1>(g, W, in, out, diag, nrhs, dag, st);
        case 5 * 16 + 2: return tiled<NOFF, WS, SS, A, 16, 8, 2>(g, W, in, out, diag, nrhs, dag, st);
        case 5 * 16 + 3: return tiled<NOFF, WS, SS, A, 16, 8, 3>(g, W, in, out, diag, nrhs, dag, st);
        case 5 * 16 + 4: return tiled<NOFF, WS, SS, A, 16, 8, 4>(g, W, in, out, diag, nrhs, dag, st);
        case 6 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 8, 1, true>(g, W, in, out, diag, nrhs, dag, st);
        case 6 * 16 + 2: return tiled<NOFF, WS, SS, A, 32, 8, 2, true>(g, W, in, out, diag, nrhs, dag, st);
        case 7 * 16 + 1: return tiled<NOFF, WS, SS, A, 16, 16, 1, true>(g, W, in, out, diag, nrhs, dag, st);
        case 8 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 8, 1, true, true>(g, W, in, out, diag, nrhs, dag, st);
        case 8 * 16 + 2: return tiled<NOFF, WS, SS, A, 32, 8, 2, true, true>(g, W, in, out, diag, nrhs, dag, st);
        case 9 * 16 + 1: return tiled<NOFF, WS, SS, A, 32, 8, 1, false, true>(g, W, in, out, diag, nrhs, dag, st);
        case 9 * 16 + 2: return tiled<NOFF, WS, SS, A, 32, 8, 2, false, true>(g, W, in, out, diag, nrhs, dag, st);
        case 9 * 16 + 3: return tiled<NOFF, WS, SS, A, 32, 8, 3, false, true>(g, W, in, out, diag, nrhs, dag, st);
        case 10 * 16 + 2: return tiled<NOFF, WS, SS, A, 16, 8, 2, false, true>(g, W, in, out, diag, nrhs, dag, st);
        case 10 * 16 + 3: return tiled<NOFF, WS, SS, A, 16, 8, 3, false, true>(g, W, in, out, diag, nrhs, dag, st);
        case 10 * 16 + 4: return tiled<NOFF, WS, SS, A, 16, 8, 4, false, true>(g, W, in, out, diag, nrhs, dag, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace launch
}  // namespace bri
