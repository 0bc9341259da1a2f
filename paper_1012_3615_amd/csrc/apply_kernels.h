// Kernel templates of the operator application (Eq. def_pref, c_SW = 0);
// apply.hip instantiates them and holds the launchers.
//
//   (D psi)(x) = (lambda_0 + m) psi(x)
//              + sum_{n != 0} [lambda_k + rho_k sum_mu n_mu gamma_mu] W(x,x+n) psi(x+n)
//
// The loop over the 80 offsets runs at run time; the offset is the same for
// every lane of a wavefront, so the tests on its components are uniform
// (scalar) branches and the spin structure costs exactly the non-zero gamma
// terms.
#pragma once
#include "common.h"

namespace bri {

// Contribution of one offset, one colour:
//   out += lam * chi + sum_{mu: n_mu != 0} (rho n_mu) gamma_mu chi
// in the chiral basis
//   gamma_x chi = (-i chi3, -i chi2,  i chi1,  i chi0)
//   gamma_y chi = (  -chi3,    chi2,    chi1,  -chi0)
//   gamma_z chi = (-i chi2,  i chi3,  i chi0, -i chi1)
//   gamma_t chi = (   chi2,    chi3,    chi0,   chi1)
template <typename T>
__device__ __forceinline__ void spin_accum_rt(cx<T> o[4], const cx<T> c[4], T lam, T rho, int nx,
                                              int ny, int nz, int nt) {
#pragma unroll
    for (int s = 0; s < 4; ++s) o[s] = caxpy(lam, c[s], o[s]);
    if (nx != 0) {
        const T r = nx > 0 ? rho : -rho;  // (-i) z = (z.im, -z.re)
        o[0].re = fma(r, c[3].im, o[0].re); o[0].im = fma(-r, c[3].re, o[0].im);
        o[1].re = fma(r, c[2].im, o[1].re); o[1].im = fma(-r, c[2].re, o[1].im);
        o[2].re = fma(-r, c[1].im, o[2].re); o[2].im = fma(r, c[1].re, o[2].im);
        o[3].re = fma(-r, c[0].im, o[3].re); o[3].im = fma(r, c[0].re, o[3].im);
    }
    if (ny != 0) {
        const T r = ny > 0 ? rho : -rho;
        o[0].re = fma(-r, c[3].re, o[0].re); o[0].im = fma(-r, c[3].im, o[0].im);
        o[1].re = fma(r, c[2].re, o[1].re); o[1].im = fma(r, c[2].im, o[1].im);
        o[2].re = fma(r, c[1].re, o[2].re); o[2].im = fma(r, c[1].im, o[2].im);
        o[3].re = fma(-r, c[0].re, o[3].re); o[3].im = fma(-r, c[0].im, o[3].im);
    }
    if (nz != 0) {
        const T r = nz > 0 ? rho : -rho;
        o[0].re = fma(r, c[2].im, o[0].re); o[0].im = fma(-r, c[2].re, o[0].im);
        o[1].re = fma(-r, c[3].im, o[1].re); o[1].im = fma(r, c[3].re, o[1].im);
        o[2].re = fma(-r, c[0].im, o[2].re); o[2].im = fma(r, c[0].re, o[2].im);
        o[3].re = fma(r, c[1].im, o[3].re); o[3].im = fma(-r, c[1].re, o[3].im);
    }
    if (nt != 0) {
        const T r = nt > 0 ? rho : -rho;
        o[0] = caxpy(r, c[2], o[0]);
        o[1] = caxpy(r, c[3], o[1]);
        o[2] = caxpy(r, c[0], o[2]);
        o[3] = caxpy(r, c[1], o[3]);
    }
}

template <typename T>
__device__ __forceinline__ T lam_rt(int k) {
    return k == 1 ? (T)(-8.0 / 128.0) : k == 2 ? (T)(-4.0 / 128.0) : k == 3 ? (T)(-2.0 / 128.0) : (T)(-1.0 / 128.0);
}
template <typename T>
__device__ __forceinline__ T rho_rt(int k) {
    return k == 1 ? (T)(64.0 / 432.0) : k == 2 ? (T)(16.0 / 432.0) : k == 3 ? (T)(4.0 / 432.0) : (T)(1.0 / 432.0);
}

// neighbour site for a run-time offset (each n_mu in {-1,0,1})
__device__ __forceinline__ int nbr_rt(const Nbr &nb, int nx, int ny, int nz, int nt) {
    const int a = nx < 0 ? nb.part[0][0] : nx > 0 ? nb.part[0][2] : nb.part[0][1];
    const int b = ny < 0 ? nb.part[1][0] : ny > 0 ? nb.part[1][2] : nb.part[1][1];
    const int c = nz < 0 ? nb.part[2][0] : nz > 0 ? nb.part[2][2] : nb.part[2][1];
    const int d = nt < 0 ? nb.part[3][0] : nt > 0 ? nb.part[3][2] : nb.part[3][1];
    return a + b + c + d;
}

// chi[s] = w[a][.] psi[s][.] for colour row a, all spins, and accumulate
template <typename A>
__device__ __forceinline__ void colour_spin_accum(cx<A> acc[4][3], const cx<A> w[3][3],
                                                  const cx<A> psi[4][3], A lam, A rho, int nx,
                                                  int ny, int nz, int nt) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<A> chi[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            cx<A> t = cmul(w[a][0], psi[s][0]);
            t = cmac(t, w[a][1], psi[s][1]);
            chi[s] = cmac(t, w[a][2], psi[s][2]);
        }
        cx<A> o[4] = {acc[0][a], acc[1][a], acc[2][a], acc[3][a]};
        spin_accum_rt(o, chi, lam, rho, nx, ny, nz, nt);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s][a] = o[s];
    }
}

// ---------------------------------------------------------------- stored W
// One thread = one site x R right-hand sides (rhs r0 .. r0+R-1 of blockIdx.y).
// W of each offset is loaded once and applied to all R fields.
template <int NOFF, typename WS, typename SS, typename A, bool DAG, int R>
__global__ __launch_bounds__(256) void k_apply_stored(Geom g, const WS *__restrict__ W,
                                                      const SS *__restrict__ in,
                                                      SS *__restrict__ out, A diag, int nrhs) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int site = blk * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const size_t V = (size_t)g.V;
    const int r0 = blockIdx.y * R;
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
    for (int j = 0; j < 80; ++j) {
        const int i = j < 40 ? j : j + 1;
        const int nx = i % 3 - 1, ny = (i / 3) % 3 - 1, nz = (i / 9) % 3 - 1, nt = i / 27 - 1;
        const int k = (nx != 0) + (ny != 0) + (nz != 0) + (nt != 0);
        const A lam = lam_rt<A>(k);
        const A rho = DAG ? -rho_rt<A>(k) : rho_rt<A>(k);
        const int y = nbr_rt(nb, nx, ny, nz, nt);
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
        const SS *q = in + (size_t)(r0 + r) * 12 * V + site;
        SS *o = out + (size_t)(r0 + r) * 12 * V + site;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                cx<A> v = caxpy(diag, ldc<A>(q + (3 * s + a) * V), acc[r][s][a]);
                st(o + (3 * s + a) * V, v);
            }
    }
}

// ---------------------------------------------------------------- stored W, LDS tiles
// One workgroup = a TX x TY tile of the (x, y) plane at fixed (z, t); one
// thread per site.  The 81-point neighbourhood is visited as 9 layers
// (n_z, n_t); for each layer the workgroup stages psi on the tile plus a
// one-site halo in x and y into LDS (every neighbour read of the layer then
// comes from LDS), and the 9 (n_x, n_y) offsets of the layer are applied.
// Transporters are streamed from HBM with non-temporal loads (80-offset
// store: every element is read exactly once).
template <int TX, int TY>
struct TileShape {
    static constexpr int HX = TX + 2, HY = TY + 2, NH = HX * HY, NT = TX * TY;
    static constexpr int LOADS = (NH + NT - 1) / NT;  // halo sites per thread
};

template <int NOFF, typename WS, typename SS, typename A, bool DAG, int TX, int TY>
__global__ __launch_bounds__(TX *TY) void k_apply_tiled(Geom g, int ntx, int nty,
                                                        const WS *__restrict__ W,
                                                        const SS *__restrict__ in,
                                                        SS *__restrict__ out, A diag) {
    using TS = TileShape<TX, TY>;
    __shared__ SS lds[12][TS::NH];
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const size_t V = (size_t)g.V;
    const int Lx = g.L[0], Ly = g.L[1], Lz = g.L[2], Lt = g.L[3];
    const int bx = blk % ntx;
    int r = blk / ntx;
    const int by = r % nty;
    r /= nty;
    const int z = r % Lz, t = r / Lz;
    in += (size_t)blockIdx.y * 12 * V;
    out += (size_t)blockIdx.y * 12 * V;
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

    cx<A> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s][a] = cmake<A>(0, 0);

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
                const SS *src = in + zt + hxy[k];
#pragma unroll
                for (int p = 0; p < 12; ++p) lds[p][q] = src[p * V];
            }
        }
        __syncthreads();
        if (valid) {
#pragma unroll 1
            for (int o = 0; o < 9; ++o) {
                const int nx = o % 3 - 1, ny = o / 3 - 1;
                const int qn = (ty + 1 + ny) * TS::HX + tx + 1 + nx;
                cx<A> psi[4][3];
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int b = 0; b < 3; ++b) psi[s][b] = ldc<A>(&lds[3 * s + b][qn]);
                if ((nx | ny | nz | nt) == 0) {
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int a = 0; a < 3; ++a) acc[s][a] = caxpy(diag, psi[s][a], acc[s][a]);
                    continue;
                }
                const int i = (nx + 1) + 3 * (ny + 1) + 9 * (nz + 1) + 27 * (nt + 1);
                const int k = (nx != 0) + (ny != 0) + (nz != 0) + (nt != 0);
                const A lam = lam_rt<A>(k);
                const A rho = DAG ? -rho_rt<A>(k) : rho_rt<A>(k);
                cx<A> w[3][3];
                if (NOFF == 80) {
                    const WS *p = W + (size_t)(i < 40 ? i : i - 1) * 9 * V + site;
#pragma unroll
                    for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ldnt<A>(p + e * V);
                } else if (i > 40) {
                    const WS *p = W + (size_t)(i - 41) * 9 * V + site;
#pragma unroll
                    for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(p + e * V);
                } else {
                    // W(x, x+n) = W(x+n, x)^dag, stored at x+n under offset -n
                    const int yn = ((x + nx + Lx) % Lx) + Lx * (((y + ny + Ly) % Ly) + Ly * (zz + Lz * tt));
                    const WS *p = W + (size_t)(39 - i) * 9 * V + yn;
#pragma unroll
                    for (int e = 0; e < 9; ++e) w[e % 3][e / 3] = cconj(ld<A>(p + e * V));
                }
                colour_spin_accum(acc, w, psi, lam, rho, nx, ny, nz, nt);
            }
        }
    }
    if (valid) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) st(out + (3 * s + a) * V + site, acc[s][a]);
    }
}

// ---------------------------------------------------------------- recompute W
// W(x, x+n) rebuilt from the links.  The 3^4 neighbourhood is split into the
// 16 orthants s in {+1,-1}^4; orthant s holds the offsets n = s*b,
// b in {0,1}^4.  Inside an orthant the transporters follow the hop-order
// recursion (average over the k! paths, grouped by their last step)
//   W(b) = (1/|b|) sum_{mu in b} W(b - mu) L(b, mu),   W(0) = 1,
// where L(b, mu) is the link of the last step into x + s*b along s_mu mu:
//   U_mu(x + s*b - mu) if s_mu = +1,   U_mu(x + s*b)^dag if s_mu = -1.
// Each offset is applied by exactly one orthant: the one whose signs agree
// with n on supp(n) and are + elsewhere.  The orthant loop runs at run time
// (uniform signs); the 15 subsets b are unrolled at compile time.
template <typename LS, typename A>
__device__ __forceinline__ void load_link_rt(const LS *__restrict__ U, size_t V, int mu, int y,
                                             bool dagger, cx<A> m[3][3]) {
    const LS *p = U + (size_t)mu * 9 * V + y;
    cx<A> t[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) t[e] = ldc<A>(p + e * V);
    if (dagger) {
#pragma unroll
        for (int e = 0; e < 9; ++e) m[e % 3][e / 3] = cconj(t[e]);
    } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) m[e / 3][e % 3] = t[e];
    }
}

template <typename A>
__device__ __forceinline__ void mat_mul_acc(cx<A> c[3][3], const cx<A> a[3][3], const cx<A> b[3][3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<A> t = c[i][j];
            t = cmac(t, a[i][0], b[0][j]);
            t = cmac(t, a[i][1], b[1][j]);
            c[i][j] = cmac(t, a[i][2], b[2][j]);
        }
}

// the 15 non-empty subsets of {x,y,z,t} in hop order
__host__ __device__ constexpr int hop_subset(int q) {
    constexpr int t[15] = {1, 2, 4, 8, 3, 5, 6, 9, 10, 12, 7, 11, 13, 14, 15};
    return t[q];
}

template <typename LS, typename SS, typename A, bool DAG>
__global__ __launch_bounds__(256) void k_apply_recompute(Geom g, const LS *__restrict__ U,
                                                         const SS *__restrict__ in,
                                                         SS *__restrict__ out, A diag) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int site = blk * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const size_t V = (size_t)g.V;
    in += (size_t)blockIdx.y * 12 * V;
    out += (size_t)blockIdx.y * 12 * V;
    int c[4];
    coords(g, site, c);
    const Nbr nb = make_nbr(g, c);
    cx<A> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s][a] = cmake<A>(0, 0);

#pragma unroll 1
    for (int so = 0; so < 16; ++so) {
        const int sg[4] = {(so & 1) ? -1 : 1, (so & 2) ? -1 : 1, (so & 4) ? -1 : 1, (so & 8) ? -1 : 1};
        cx<A> w[16][3][3];
        static_for<0, 15>([&](auto Q) {
            constexpr int B = hop_subset(decltype(Q)::value);
            constexpr int pc = (B & 1) + ((B >> 1) & 1) + ((B >> 2) & 1) + ((B >> 3) & 1);
            const int n[4] = {(B & 1) ? sg[0] : 0, (B & 2) ? sg[1] : 0, (B & 4) ? sg[2] : 0,
                              (B & 8) ? sg[3] : 0};
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) w[B][a][b] = cmake<A>(0, 0);
            static_for<0, 4>([&](auto M) {
                constexpr int mu = decltype(M)::value;
                if constexpr ((B >> mu) & 1) {
                    int d[4] = {n[0], n[1], n[2], n[3]};
                    d[mu] = sg[mu] > 0 ? 0 : -1;
                    cx<A> l[3][3];
                    load_link_rt<LS, A>(U, V, mu, nbr_rt(nb, d[0], d[1], d[2], d[3]), sg[mu] < 0, l);
                    constexpr int P = B & ~(1 << mu);
                    if constexpr (P == 0) {
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int b = 0; b < 3; ++b) w[B][a][b] = l[a][b];
                    } else {
                        mat_mul_acc(w[B], w[P], l);
                    }
                }
            });
            if constexpr (pc > 1) {
                constexpr A inv = (A)1 / (A)pc;
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) w[B][a][b] = cscale(inv, w[B][a][b]);
            }
            // owned: every negative direction of this orthant lies in B
            if ((B & so) == so) {
                const A lam = (A)lam_k(pc);
                const A rho = DAG ? -(A)rho_k(pc) : (A)rho_k(pc);
                const int y = nbr_rt(nb, n[0], n[1], n[2], n[3]);
                cx<A> psi[4][3];
#pragma unroll
                for (int s = 0; s < 4; ++s)
#pragma unroll
                    for (int b = 0; b < 3; ++b) psi[s][b] = ldc<A>(in + (3 * s + b) * V + y);
                colour_spin_accum(acc, w[B], psi, lam, rho, n[0], n[1], n[2], n[3]);
            }
        });
    }

#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<A> v = caxpy(diag, ldc<A>(in + (3 * s + a) * V + site), acc[s][a]);
            st(out + (3 * s + a) * V + site, v);
        }
}

}  // namespace bri
