// The Wilson operator, the comparison operator of the paper (Sec. 1; the
// Wilson column of Tab. rholambda: lambda_0 = 4, lambda_1 = -1/2, rho_1 = 1/2,
// every other entry zero):
//   (D psi)(x) = (4 + m) psi(x)
//              - 1/2 sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
//                            + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)],
// D^dag the same with gamma_mu -> -gamma_mu.  It reads the links directly (no
// transporters), so it is the 9-point operator against which the 81-point
// Brillouin apply is priced.
//
// Each hop uses the half-spinor form.  In the chiral basis gamma_mu is
// [[0, B_mu], [B_mu^dag, 0]] on (upper spins 0,1 | lower spins 2,3) with
// B_mu^dag B_mu = 1, so (1 - s gamma_mu) chi has upper part
// h = chi_u - s B_mu chi_l and lower part -s B_mu^dag h: one colour
// multiplication of the two-spin h per hop instead of four.
//   B_x = [[0, -i], [-i, 0]]   B_y = [[0, -1], [1, 0]]
//   B_z = [[-i, 0], [0, i]]    B_t = [[1, 0], [0, 1]]
// (the gamma matrices are those of the Brillouin stencil's spin algebra).
#include "common.h"
#include "kernels.h"

namespace bri {
namespace {

template <typename A>
__device__ __forceinline__ cx<A> times_i(cx<A> z) { return {-z.im, z.re}; }
template <typename A>
__device__ __forceinline__ cx<A> times_mi(cx<A> z) { return {z.im, -z.re}; }

// (o0, o1) = B_mu (l0, l1)
template <int MU, typename A>
__device__ __forceinline__ void b_mul(cx<A> l0, cx<A> l1, cx<A> &o0, cx<A> &o1) {
    if (MU == 0) { o0 = times_mi(l1); o1 = times_mi(l0); }
    if (MU == 1) { o0 = {-l1.re, -l1.im}; o1 = l0; }
    if (MU == 2) { o0 = times_mi(l0); o1 = times_i(l1); }
    if (MU == 3) { o0 = l0; o1 = l1; }
}

// (o2, o3) = B_mu^dag (u0, u1)
template <int MU, typename A>
__device__ __forceinline__ void bdag_mul(cx<A> u0, cx<A> u1, cx<A> &o2, cx<A> &o3) {
    if (MU == 0) { o2 = times_i(u1); o3 = times_i(u0); }
    if (MU == 1) { o2 = u1; o3 = {-u0.re, -u0.im}; }
    if (MU == 2) { o2 = times_i(u0); o3 = times_mi(u1); }
    if (MU == 3) { o2 = u0; o3 = u1; }
}

// acc += -1/2 (1 - s gamma_mu) W psi(y), W = U_mu(x) for the forward hop
// (N = +1), U_mu(x-mu)^dag for the backward hop (N = -1); s = N, or -N for D^dag.
template <int MU, int N, bool DAG, typename T, typename A>
__device__ __forceinline__ void wilson_hop(const Geom &g, const int c[4], int site, size_t V,
                                           const T *__restrict__ U, const T *__restrict__ q,
                                           cx<A> (&acc)[4][3]) {
    const int L = g.L[MU], str = g.stride[MU];
    const int y = N > 0 ? (c[MU] == L - 1 ? site - (L - 1) * str : site + str)
                        : (c[MU] == 0 ? site + (L - 1) * str : site - str);
    const A s = (A)(DAG ? -N : N);
    cx<A> h[2][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const cx<A> u0 = ldc<A>(q + (size_t)(0 + b) * V + y), u1 = ldc<A>(q + (size_t)(3 + b) * V + y);
        const cx<A> l0 = ldc<A>(q + (size_t)(6 + b) * V + y), l1 = ldc<A>(q + (size_t)(9 + b) * V + y);
        cx<A> t0, t1;
        b_mul<MU>(l0, l1, t0, t1);
        h[0][b] = caxpy(-s, t0, u0);
        h[1][b] = caxpy(-s, t1, u1);
    }
    const T *p = U + (size_t)MU * 9 * V + (N > 0 ? site : y);
    cx<A> w[3][3];
#pragma unroll
    for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(p + (size_t)e * V);
    const A half = (A)0.5;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<A> y0, y1;
        if (N > 0) {
            y0 = cmul(w[a][0], h[0][0]);
            y1 = cmul(w[a][0], h[1][0]);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                y0 = cmac(y0, w[a][b], h[0][b]);
                y1 = cmac(y1, w[a][b], h[1][b]);
            }
        } else {
            y0 = cmul(cconj(w[0][a]), h[0][0]);
            y1 = cmul(cconj(w[0][a]), h[1][0]);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                y0 = cmacc(y0, w[b][a], h[0][b]);
                y1 = cmacc(y1, w[b][a], h[1][b]);
            }
        }
        acc[0][a] = caxpy(-half, y0, acc[0][a]);
        acc[1][a] = caxpy(-half, y1, acc[1][a]);
        cx<A> t2, t3;
        bdag_mul<MU>(y0, y1, t2, t3);
        acc[2][a] = caxpy(half * s, t2, acc[2][a]);
        acc[3][a] = caxpy(half * s, t3, acc[3][a]);
    }
}

// One thread = one site of one right-hand side (blockIdx.y).  Neighbour
// spinors and the backward links come through the caches; the site blocks
// of one XCD are consecutive, so a neighbour in y, z or t was read shortly
// before by a block of the same XCD.
template <typename T, typename A, bool DAG>
__global__ __launch_bounds__(256) void k_wilson(Geom g, const T *__restrict__ U, const T *__restrict__ in,
                                                T *__restrict__ out, A diag) {
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int site = blk * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const size_t V = (size_t)g.V;
    const T *q = in + (size_t)blockIdx.y * 12 * V;
    int c[4];
    coords(g, site, c);
    cx<A> acc[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s][a] = cscale(diag, ldc<A>(q + (size_t)(3 * s + a) * V + site));
    wilson_hop<0, +1, DAG>(g, c, site, V, U, q, acc);
    wilson_hop<0, -1, DAG>(g, c, site, V, U, q, acc);
    wilson_hop<1, +1, DAG>(g, c, site, V, U, q, acc);
    wilson_hop<1, -1, DAG>(g, c, site, V, U, q, acc);
    wilson_hop<2, +1, DAG>(g, c, site, V, U, q, acc);
    wilson_hop<2, -1, DAG>(g, c, site, V, U, q, acc);
    wilson_hop<3, +1, DAG>(g, c, site, V, U, q, acc);
    wilson_hop<3, -1, DAG>(g, c, site, V, U, q, acc);
    T *o = out + (size_t)blockIdx.y * 12 * V + site;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) st(o + (size_t)(3 * s + a) * V, acc[s][a]);
}

template <typename T, typename A>
hipError_t launch(const Geom &g, const void *U, const void *in, void *out, double diag, int nrhs, bool dag,
                  hipStream_t st) {
    const dim3 grid((g.V + 255) / 256, nrhs), block(256);
    if (dag)
        k_wilson<T, A, true><<<grid, block, 0, st>>>(g, (const T *)U, (const T *)in, (T *)out, (A)diag);
    else
        k_wilson<T, A, false><<<grid, block, 0, st>>>(g, (const T *)U, (const T *)in, (T *)out, (A)diag);
    return hipGetLastError();
}

}  // namespace

hipError_t apply_wilson(const Geom &g, int prec, const void *U, const void *in, void *out, double diag,
                        int nrhs, bool dag, hipStream_t st) {
    if (prec == 0) return launch<double2, double>(g, U, in, out, diag, nrhs, dag, st);
    return launch<float2, float>(g, U, in, out, diag, nrhs, dag, st);
}

}  // namespace bri
