// Stored-transporter apply, neighbour gathers through the caches, several
// right-hand sides per thread (the fused multi-RHS form).
#pragma once
#include <type_traits>

#include "stencil.h"

namespace bri {
// ---------------------------------------------------------------- stored W
// One thread = one site x R right-hand sides (rhs r0 .. r0+R-1 of blockIdx.y).
// W of each offset is loaded once and applied to all R fields.
template <int NOFF, typename WS, typename SS, typename A, bool DAG, int R>
__global__ __launch_bounds__(256) void k_apply_stored(Geom g, const WS *__restrict__ W,
                                                      const SS *__restrict__ in,
                                                      SS *__restrict__ out, A diag, int nrhs, Coef<A> cf) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int site = blk * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const size_t V = (size_t)g.V;
    const int r0 = blockIdx.y * R;
    // FP16 transporters and spinors: the same packed FP16 colour products as
    // the LDS-tiled kernel (so that all configurations agree bit for bit)
    constexpr bool H2 = std::is_same<WS, __half2>::value && std::is_same<SS, __half2>::value &&
                        std::is_same<A, float>::value;
    int c[4];
    coords(g, site, c);
    const Nbr nb = make_nbr(g, c);

    cx<A> acc[R][4][3];
#pragma unroll
    for (int j = 0; j < R; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[j][s][a] = cmake<A>(0, 0);

#pragma unroll 1
    for (int i = 0; i < 81; ++i) {
        const int nx = i % 3 - 1, ny = (i / 3) % 3 - 1, nz = (i / 9) % 3 - 1, nt = i / 27 - 1;
        if (i == 40) {
            // the diagonal term, at its place in the offset order (as in the LDS-tiled kernel)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (R > 1 && r0 + r >= nrhs) break;
                const SS *q = in + (size_t)(r0 + r) * 12 * V + site;
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        acc[r][s][a] = caxpy(diag, ldc<A>(q + (3 * s + a) * V), acc[r][s][a]);
            }
            continue;
        }
        const int j = i < 40 ? i : i - 1;
        const int k = (nx != 0) + (ny != 0) + (nz != 0) + (nt != 0);
        const A lam = coef_pick(cf.lam, k);
        const A rho = DAG ? -coef_pick(cf.rho, k) : coef_pick(cf.rho, k);
        const int y = nbr_rt(nb, nx, ny, nz, nt);
        if constexpr (H2) {
            const uint32_t *W32 = reinterpret_cast<const uint32_t *>(W);
            uint32_t w[3][3];
            if (NOFF == 80 || i > 40) {
                const uint32_t *p = W32 + (size_t)(NOFF == 80 ? j : i - 41) * 9 * V + site;
#pragma unroll
                for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = p[e * V];
            } else {
                const uint32_t *p = W32 + (size_t)(39 - i) * 9 * V + y;
#pragma unroll
                for (int e = 0; e < 9; ++e) w[e % 3][e / 3] = p[e * V] ^ 0x80000000u;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (R > 1 && r0 + r >= nrhs) break;
                const uint32_t *q = reinterpret_cast<const uint32_t *>(in) + (size_t)(r0 + r) * 12 * V + y;
                uint32_t psi[4][3];
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int b = 0; b < 3; ++b) psi[s][b] = q[(3 * s + b) * V];
                colour_spin_accum_h2(acc[r], w, psi, lam, rho, nx, ny, nz, nt);
            }
            continue;
        }
        cx<A> w[3][3];
        if (NOFF == 80 || i > 40) {
            const WS *p = W + (size_t)(NOFF == 80 ? j : i - 41) * 9 * V + site;
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(p + e * V);
        } else {
            // W(x, x+n) = W(x+n, x)^dag, stored at x+n under offset -n (index 80-i)
            const WS *p = W + (size_t)(39 - i) * 9 * V + y;
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e % 3][e / 3] = cconj(ld<A>(p + e * V));
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (R > 1 && r0 + r >= nrhs) break;
            const SS *q = in + (size_t)(r0 + r) * 12 * V + y;
            cx<A> psi[4][3];
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int b = 0; b < 3; ++b) psi[s][b] = ldc<A>(q + (3 * s + b) * V);
            colour_spin_accum(acc[r], w, psi, lam, rho, nx, ny, nz, nt);
        }
    }

#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (R > 1 && r0 + r >= nrhs) break;
        SS *o = out + (size_t)(r0 + r) * 12 * V + site;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) stnt(o + (3 * s + a) * V, acc[r][s][a]);
    }
}


}  // namespace bri
