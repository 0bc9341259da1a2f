// Stored-transporter apply with LDS-staged spinor layers (one right-hand
// side per thread).
#pragma once
#include <type_traits>

#include "stencil.h"
#include "su3.h"

namespace bri {
// ---------------------------------------------------------------- stored W, LDS tiles
// One workgroup = a TX x TY tile of the (x, y) plane at fixed (z, t); one
// thread per site.  The 81-point neighbourhood is visited as 9 layers
// (n_z, n_t); for each layer the workgroup stages psi on the tile plus a
// one-site halo in x and y into LDS (every neighbour read of the layer then
// comes from LDS), and the 9 (n_x, n_y) offsets of the layer are applied.
// Transporters are streamed from HBM with non-temporal loads (80-offset
// store: every element is read exactly once per right-hand-side group).  With
// R > 1 each thread holds R right-hand sides: the LDS holds R layers and every
// transporter load serves all R.
//
// Options for the production operator: ROWS = 2 reads the two-row store of
// back-projected (SU(3)) transporters and rebuilds the third row; CLV adds
// the clover term, a Hermitian 6x6 block per chirality and site, at n = 0.
// lambda_k and rho_k come from the by-value argument cf (any member of the
// generic class of Sec. 8; the host fills in the Brillouin column by
// default).  In scalar registers they also cost no vector registers: with
// compile-time constants, which gfx9 VOP3 instructions cannot encode as
// literals, the FP32 32x8 kernel held them in VGPRs (137 instead of 123,
// three waves per SIMD instead of four).
template <int TX, int TY>
struct TileShape {
    static constexpr int HX = TX + 2, HY = TY + 2, NH = HX * HY, NT = TX * TY;
    static constexpr int LOADS = (NH + NT - 1) / NT;  // halo sites per thread
};

template <int NOFF, typename WS, typename SS, typename A, bool DAG, int TX, int TY, int R, bool PF = false,
          bool UN = false, int ROWS = 3, bool CLV = false>
__global__ __launch_bounds__(TX *TY) void k_apply_tiled(Geom g, int ntx, int nty,
                                                        const WS *__restrict__ W,
                                                        const SS *__restrict__ in,
                                                        SS *__restrict__ out, A diag, int nrhs,
                                                        const SS *__restrict__ clover, Coef<A> cf) {
    using TS = TileShape<TX, TY>;
    // FP16 transporters and spinors: colour products on packed FP16 pairs
    // with FP32 accumulation (the transporter words stay as loaded)
    constexpr bool H2 = std::is_same<WS, __half2>::value && std::is_same<SS, __half2>::value &&
                        std::is_same<A, float>::value && ROWS == 3;
    __shared__ SS lds[R][12][TS::NH];
    // one-dimensional grid: tile-major, right-hand-side group fastest, so the
    // groups of a tile run back to back on one XCD and share its transporters
    // through that XCD's L2
    const int ngrp = (nrhs + R - 1) / R;
    const int lin = xcd_block(blockIdx.x, gridDim.x);
    const int grp = lin % ngrp;
    const int blk = lin / ngrp;
    const size_t V = (size_t)g.V;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const int bx = blk % ntx;
    int r = blk / ntx;
    const int by = r % nty;
    r /= nty;
    const int z = r % Lz, t = r / Lz;
    const int r0 = grp * R;
    const int nr = nrhs - r0 < R ? nrhs - r0 : R;  // right-hand sides of this block
    in += (size_t)r0 * 12 * V;
    out += (size_t)r0 * 12 * V;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int x = bx * TX + tx, y = by * TY + ty;
    const bool valid = x < Lx && y < Ly;
    const int site = valid ? x + Lx * (y + Ly * (z + Lz * t)) : 0;

    // (x, y) part of the global index of the halo sites this thread stages
    int hxy[TS::LOADS];
#pragma unroll
    for (int k = 0; k < TS::LOADS; ++k) {
        const int q = threadIdx.x + k * TS::NT;
        const int hx = q % TS::HX - 1, hy = q / TS::HX - 1;
        const int gx = (bx * TX + hx + Lx) % Lx, gy = (by * TY + hy + Ly) % Ly;
        hxy[k] = q < TS::NH ? gx + Lx * gy : -1;
    }
    const int plane = Lx * Ly;

    cx<A> acc[R][4][3];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[r][s][a] = cmake<A>(0, 0);

    // clover term first, while few registers are live: one chirality block
    // (six spin-colour components) at a time, psi(x) read from global memory
    if constexpr (CLV) {
        if (valid) {
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cx<A> cl[18];
                clover_load_block(clover, V, site, b, cl);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (R > 1 && r >= nr) break;
                    cx<A> xb[6];
#pragma unroll
                    for (int i = 0; i < 6; ++i) xb[i] = ldc<A>(in + (size_t)r * 12 * V + (6 * b + i) * V + site);
                    clover_accum_block(cl, xb, b, acc[r]);
                }
            }
        }
    }

    // transporter of offset (nx, ny) of layer (lz, lt) = (layer % 3, layer / 3)
    auto load_w = [&](int layer, int nx, int ny, cx<A> (&w)[3][3]) {
        const int lnz = layer % 3 - 1, lnt = layer / 3 - 1;
        const int i = (nx + 1) + 3 * (ny + 1) + 9 * (lnz + 1) + 27 * (lnt + 1);
        constexpr int NE = 3 * ROWS;  // stored elements per transporter
        if (NOFF == 80) {
            const WS *p = W + (size_t)(i < 40 ? i : i - 1) * NE * V + site;
#pragma unroll
            for (int e = 0; e < NE; ++e) w[e / 3][e % 3] = ldnt<A>(p + e * V);
            if constexpr (ROWS == 2) su3_third_row(w);
        } else if (i > 40) {
            const WS *p = W + (size_t)(i - 41) * NE * V + site;
#pragma unroll
            for (int e = 0; e < NE; ++e) w[e / 3][e % 3] = ld<A>(p + e * V);
            if constexpr (ROWS == 2) su3_third_row(w);
        } else {
            // W(x, x+n) = W(x+n, x)^dag, stored at x+n under offset -n
            const int zn = (z + lnz + Lz) % Lz, tn = (t + lnt + Lt) % Lt;
            const int yn = ((x + nx + Lx) % Lx) + Lx * (((y + ny + Ly) % Ly) + Ly * (zn + Lz * tn));
            const WS *p = W + (size_t)(39 - i) * NE * V + yn;
            if constexpr (ROWS == 2) {
                cx<A> m[3][3];
#pragma unroll
                for (int e = 0; e < NE; ++e) m[e / 3][e % 3] = ld<A>(p + e * V);
                su3_third_row(m);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) w[a][b] = cconj(m[b][a]);
            } else {
#pragma unroll
                for (int e = 0; e < 9; ++e) w[e % 3][e / 3] = cconj(ld<A>(p + e * V));
            }
        }
    };
    // the same as raw FP16 words, the conjugate by the sign of the high half
    auto load_w_h2 = [&](int layer, int nx, int ny, uint32_t (&w)[3][3]) {
        const int lnz = layer % 3 - 1, lnt = layer / 3 - 1;
        const int i = (nx + 1) + 3 * (ny + 1) + 9 * (lnz + 1) + 27 * (lnt + 1);
        const uint32_t *W32 = reinterpret_cast<const uint32_t *>(W);
        if (NOFF == 80) {
            const uint32_t *p = W32 + (size_t)(i < 40 ? i : i - 1) * 9 * V + site;
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = __builtin_nontemporal_load(p + e * V);
        } else if (i > 40) {
            const uint32_t *p = W32 + (size_t)(i - 41) * 9 * V + site;
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = p[e * V];
        } else {
            const int zn = (z + lnz + Lz) % Lz, tn = (t + lnt + Lt) % Lt;
            const int yn = ((x + nx + Lx) % Lx) + Lx * (((y + ny + Ly) % Ly) + Ly * (zn + Lz * tn));
            const uint32_t *p = W32 + (size_t)(39 - i) * 9 * V + yn;
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e % 3][e / 3] = p[e * V] ^ 0x80000000u;
        }
    };
    // with PF the next transporter of the layer is in flight during the
    // arithmetic of the current one (not across layers: vector-memory loads
    // return in order, and an HBM load issued before the layer's LDS fill
    // would delay the fill's L2 hits)
    cx<A> wn[3][3];
    uint32_t wnh[3][3];

#pragma unroll 1
    for (int layer = 0; layer < 9; ++layer) {
        const int nz = layer % 3 - 1, nt = layer / 3 - 1;
        const int zz = (z + nz + Lz) % Lz, tt = (t + nt + Lt) % Lt;
        const int zt = plane * (zz + Lz * tt);
        __syncthreads();  // previous layer fully consumed
#pragma unroll
        for (int k = 0; k < TS::LOADS; ++k) {
            if (hxy[k] >= 0) {
                const int q = threadIdx.x + k * TS::NT;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (R > 1 && r >= nr) break;
                    const SS *src = in + (size_t)r * 12 * V + zt + hxy[k];
#pragma unroll
                    for (int p = 0; p < 12; ++p) lds[r][p][q] = src[p * V];
                }
            }
        }
        __syncthreads();
        const bool centre = (nz | nt) == 0;  // this layer holds n = 0 at o = 4
        if (valid) {
            if (PF) {
                if constexpr (H2)
                    load_w_h2(layer, -1, -1, wnh);
                else
                    load_w(layer, -1, -1, wn);
            }
            // one offset (nx, ny) = (o % 3 - 1, o / 3 - 1) of this layer
            auto offset = [&](const int o) __attribute__((always_inline)) {
                const int nx = o % 3 - 1, ny = o / 3 - 1;
                const int qn = (ty + 1 + ny) * TS::HX + tx + 1 + nx;
                if (centre && o == 4) {
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (R > 1 && r >= nr) break;
#pragma unroll
                        for (int s = 0; s < 4; ++s)
#pragma unroll
                            for (int a = 0; a < 3; ++a)
                                acc[r][s][a] = caxpy(diag, ldc<A>(&lds[r][3 * s + a][qn]), acc[r][s][a]);
                    }
                    return;
                }
                const int k = (nx != 0) + (ny != 0) + (nz != 0) + (nt != 0);
                const A lam = coef_pick(cf.lam, k);
                const A rho = DAG ? -coef_pick(cf.rho, k) : coef_pick(cf.rho, k);
                if constexpr (H2) {
                    uint32_t w[3][3];
                    if (PF) {
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int b = 0; b < 3; ++b) w[a][b] = wnh[a][b];
                        int o2 = o + 1;
                        if (centre && o2 == 4) ++o2;
                        if (o2 < 9) load_w_h2(layer, o2 % 3 - 1, o2 / 3 - 1, wnh);
                    } else {
                        load_w_h2(layer, nx, ny, w);
                    }
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        if (R > 1 && r >= nr) break;
                        uint32_t psi[4][3];
#pragma unroll
                        for (int s = 0; s < 4; ++s)
#pragma unroll
                            for (int b = 0; b < 3; ++b)
                                psi[s][b] = *reinterpret_cast<const uint32_t *>(&lds[r][3 * s + b][qn]);
                        colour_spin_accum_h2(acc[r], w, psi, lam, rho, nx, ny, nz, nt);
                    }
                    return;
                }
                cx<A> w[3][3];
                if (PF) {
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) w[a][b] = wn[a][b];
                    // issue the next transporter before this one's arithmetic
                    int o2 = o + 1;
                    if (centre && o2 == 4) ++o2;
                    if (o2 < 9) load_w(layer, o2 % 3 - 1, o2 / 3 - 1, wn);
                } else {
                    load_w(layer, nx, ny, w);
                }
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (R > 1 && r >= nr) break;
                    cx<A> psi[4][3];
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int b = 0; b < 3; ++b) psi[s][b] = ldc<A>(&lds[r][3 * s + b][qn]);
                    colour_spin_accum(acc[r], w, psi, lam, rho, nx, ny, nz, nt);
                }
            };
            if constexpr (UN) {
                // compile-time offsets: the spin structure and the prefetch
                // registers resolve statically
                static_for<0, 9>([&](auto O) { offset(decltype(O)::value); });
            } else {
#pragma unroll 1
                for (int o = 0; o < 9; ++o) offset(o);
            }
        }
    }
    if (valid) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (R > 1 && r >= nr) break;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int a = 0; a < 3; ++a) stnt(out + (size_t)r * 12 * V + (3 * s + a) * V + site, acc[r][s][a]);
        }
    }
}


}  // namespace bri
