// Apply with the transporters rebuilt from the links inside the kernel.
#pragma once
#include "stencil.h"

namespace bri {
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

// The offsets owned by orthant `so` (signs s_mu = -1 where bit mu is set):
// its 15 sub-transporters by the recursion, and acc += their stencil terms.
template <typename LS, typename SS, typename A, bool DAG>
__device__ __forceinline__ void recompute_orthant(const LS *__restrict__ U, const SS *__restrict__ in, size_t V,
                                                  const Nbr &nb, int so, cx<A> (&acc)[4][3]) {
    const int sg[4] = {(so & 1) ? -1 : 1, (so & 2) ? -1 : 1, (so & 4) ? -1 : 1, (so & 8) ? -1 : 1};
    cx<A> w[16][3][3];
    static_for<0, 15>([&](auto Q) {
        constexpr int B = hop_subset(decltype(Q)::value);
        constexpr int pc = (B & 1) + ((B >> 1) & 1) + ((B >> 2) & 1) + ((B >> 3) & 1);
        const int n[4] = {(B & 1) ? sg[0] : 0, (B & 2) ? sg[1] : 0, (B & 4) ? sg[2] : 0, (B & 8) ? sg[3] : 0};
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

// One workgroup = 16 consecutive sites x the 16 orthants: a thread builds
// one orthant's transporters for one site, so the links and psi of those
// sites are read by 16 threads at once (from L1/L2) instead of by one thread
// over its whole loop.  The 16 partial sums of a site are added in orthant
// order through LDS, then the diagonal term.
template <typename LS, typename SS, typename A, bool DAG>
__global__ __launch_bounds__(256) void k_apply_recompute(Geom g, const LS *__restrict__ U,
                                                         const SS *__restrict__ in,
                                                         SS *__restrict__ out, A diag) {
    __shared__ A red[16][12][16][2];
    const int sl = threadIdx.x % 16, so = threadIdx.x / 16;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int s0 = blk * 16 + sl;
    const bool valid = s0 < g.V;
    const int site = valid ? s0 : 0;
    const size_t V = (size_t)g.V;
    in += (size_t)blockIdx.y * 12 * V;
    out += (size_t)blockIdx.y * 12 * V;
    cx<A> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s][a] = cmake<A>(0, 0);
    if (valid) {
        int c[4];
        coords(g, site, c);
        const Nbr nb = make_nbr(g, c);
        recompute_orthant<LS, SS, A, DAG>(U, in, V, nb, so, acc);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            red[so][3 * s + a][sl][0] = acc[s][a].re;
            red[so][3 * s + a][sl][1] = acc[s][a].im;
        }
    __syncthreads();
    if (threadIdx.x < 192) {
        const int ss = threadIdx.x % 16, comp = threadIdx.x / 16;
        const int st_site = blk * 16 + ss;
        if (st_site < g.V) {
            cx<A> sum = cmake<A>(red[0][comp][ss][0], red[0][comp][ss][1]);
#pragma unroll
            for (int o = 1; o < 16; ++o) sum = cadd(sum, cmake<A>(red[o][comp][ss][0], red[o][comp][ss][1]));
            st(out + comp * V + st_site, caxpy(diag, ldc<A>(in + comp * V + st_site), sum));
        }
    }
}


}  // namespace bri
