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

// (o0, o1) = B_mu (l0, l1); mu is the same for every lane (uniform branches)
template <typename A>
__device__ __forceinline__ void b_mul(int mu, cx<A> l0, cx<A> l1, cx<A> &o0, cx<A> &o1) {
    if (mu == 0) { o0 = times_mi(l1); o1 = times_mi(l0); }
    else if (mu == 1) { o0 = {-l1.re, -l1.im}; o1 = l0; }
    else if (mu == 2) { o0 = times_mi(l0); o1 = times_i(l1); }
    else { o0 = l0; o1 = l1; }
}

// (o2, o3) = B_mu^dag (u0, u1)
template <typename A>
__device__ __forceinline__ void bdag_mul(int mu, cx<A> u0, cx<A> u1, cx<A> &o2, cx<A> &o3) {
    if (mu == 0) { o2 = times_i(u1); o3 = times_i(u0); }
    else if (mu == 1) { o2 = u1; o3 = {-u0.re, -u0.im}; }
    else if (mu == 2) { o2 = times_i(u0); o3 = times_mi(u1); }
    else { o2 = u0; o3 = u1; }
}

template <typename T, typename A>
__device__ __forceinline__ void load_spinor(const T *__restrict__ p, size_t V, cx<A> (&v)[4][3]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) v[s][a] = ldc<A>(p + (size_t)(3 * s + a) * V);
}

// acc += -1/2 (1 - s gamma_mu) W v with v the neighbour spinor and W the
// link (forward hop) or its adjoint taken here (backward hop), both in
// registers; s = +1 forward, -1 backward (negated for D^dag).
template <bool DAG, typename A>
__device__ __forceinline__ void hop_core(int mu, bool fwd, const cx<A> (&v)[4][3], const cx<A> (&w)[3][3],
                                         cx<A> (&acc)[4][3]) {
    const A s = (fwd != DAG) ? (A)1 : (A)-1;
    cx<A> h[2][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        cx<A> t0, t1;
        b_mul(mu, v[2][b], v[3][b], t0, t1);
        h[0][b] = caxpy(-s, t0, v[0][b]);
        h[1][b] = caxpy(-s, t1, v[1][b]);
    }
    const A half = (A)0.5;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<A> y0, y1;
        if (fwd) {
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
        bdag_mul(mu, y0, y1, t2, t3);
        acc[2][a] = caxpy(half * s, t2, acc[2][a]);
        acc[3][a] = caxpy(half * s, t3, acc[3][a]);
    }
}

// The hop 2 mu + (0: forward, 1: backward) of one site with its operands
// from memory: W = U_mu(x), y = x + mu forward, W = U_mu(x-mu)^dag, y = x - mu
// backward.  Everything lane-dependent is computed from the run-time hop, so
// the compiler cannot hoist the addresses of all the hops out of the loop.
template <bool DAG, typename T, typename A>
__device__ __forceinline__ void wilson_hop(int hop, const Geom &g, const int c[4], int site, size_t V,
                                           const T *__restrict__ U, const T *__restrict__ q,
                                           cx<A> (&acc)[4][3]) {
    const int mu = hop >> 1;
    const bool fwd = (hop & 1) == 0;
    const int L = g.L[mu], str = g.stride[mu];
    const int cm = mu == 0 ? c[0] : mu == 1 ? c[1] : mu == 2 ? c[2] : c[3];
    const int y = fwd ? (cm == L - 1 ? site - (L - 1) * str : site + str)
                      : (cm == 0 ? site + (L - 1) * str : site - str);
    cx<A> v[4][3], w[3][3];
    load_spinor(q + y, V, v);
    const T *p = U + (size_t)mu * 9 * V + (fwd ? site : y);
#pragma unroll
    for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(p + (size_t)e * V);
    hop_core<DAG>(mu, fwd, v, w, acc);
}

// The t hops from registers: U_mu(x - t)^dag h with h the backward projection
// of psi(x - t) is what the forward t hop of the site below has at hand (its
// link and its spinor), so a thread owns one (x, y, z) and walks a chunk of t
// values, carrying that product and the spinor it loaded for its forward hop
// to the next step.  The x, y and z hops read their neighbours through the
// caches (the threads of those neighbours read the same data at about the
// same step).

// (1 - s gamma_t) psi has upper part h = psi_u - s psi_l (B_t = 1)
template <typename A>
__device__ __forceinline__ void project_t(const cx<A> (&v)[4][3], A s, cx<A> (&h)[2][3]) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        h[0][b] = caxpy(-s, v[2][b], v[0][b]);
        h[1][b] = caxpy(-s, v[3][b], v[1][b]);
    }
}

// acc += -1/2 (1 - s gamma_t) applied to the colour-multiplied upper part y
template <typename A>
__device__ __forceinline__ void reconstruct_t(const cx<A> (&y)[2][3], A s, cx<A> (&acc)[4][3]) {
    const A half = (A)0.5;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[0][a] = caxpy(-half, y[0][a], acc[0][a]);
        acc[1][a] = caxpy(-half, y[1][a], acc[1][a]);
        acc[2][a] = caxpy(half * s, y[0][a], acc[2][a]);
        acc[3][a] = caxpy(half * s, y[1][a], acc[3][a]);
    }
}

// y = W^dag h
template <typename A>
__device__ __forceinline__ void mul_dag(const cx<A> (&w)[3][3], const cx<A> (&h)[2][3], cx<A> (&y)[2][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        y[0][a] = cmul(cconj(w[0][a]), h[0][0]);
        y[1][a] = cmul(cconj(w[0][a]), h[1][0]);
#pragma unroll
        for (int b = 1; b < 3; ++b) {
            y[0][a] = cmacc(y[0][a], w[b][a], h[0][b]);
            y[1][a] = cmacc(y[1][a], w[b][a], h[1][b]);
        }
    }
}

template <typename T, typename A, bool DAG>
__global__ __launch_bounds__(256) void k_wilson(Geom g, const T *__restrict__ U, const T *__restrict__ in,
                                                T *__restrict__ out, A diag, int tchunk) {
    const int v3 = g.stride[3];  // Lx Ly Lz
    const int s3 = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (s3 >= v3) return;
    const int lt = g.L[3];
    const int t0 = blockIdx.y * tchunk;
    const int t1 = min(t0 + tchunk, lt);
    const size_t V = (size_t)g.V;
    const T *q = in + (size_t)blockIdx.z * 12 * V;
    T *o = out + (size_t)blockIdx.z * 12 * V;
    const T *Ut = U + (size_t)3 * 9 * V;
    const A sf = DAG ? (A)-1 : (A)1;  // s of the forward hops; -sf for the backward ones

    // carry = U_t(x, t0-1)^dag (1 + sf gamma_t)-projection of psi(x, t0-1)
    cx<A> carry[2][3], nxt[4][3];
    {
        const int sb = s3 + (t0 == 0 ? lt - 1 : t0 - 1) * v3;
        cx<A> v[4][3], h[2][3], w[3][3];
        load_spinor(q + sb, V, v);
        project_t(v, -sf, h);
#pragma unroll
        for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(Ut + (size_t)e * V + sb);
        mul_dag(w, h, carry);
    }
    load_spinor(q + s3 + t0 * v3, V, nxt);

#pragma unroll 1
    for (int t = t0; t < t1; ++t) {
        const int site = s3 + t * v3;
        int c[4];
        coords(g, site, c);
        cx<A> acc[4][3], hb[2][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[s][a] = cscale(diag, nxt[s][a]);
        project_t(nxt, -sf, hb);  // for the backward t hop of the next step
#pragma unroll 1
        for (int hop = 0; hop < 6; ++hop) wilson_hop<DAG>(hop, g, c, site, V, U, q, acc);
        // loaded after the x, y, z hops: live across them it costs 24 (FP32)
        // or 48 (FP64) registers per lane
        const int sn = s3 + (t == lt - 1 ? 0 : t + 1) * v3;
        load_spinor(q + sn, V, nxt);
        // forward t hop from the spinor just loaded; its link also makes the carry
        cx<A> w[3][3], h[2][3], y[2][3];
#pragma unroll
        for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(Ut + (size_t)e * V + site);
        project_t(nxt, sf, h);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            y[0][a] = cmul(w[a][0], h[0][0]);
            y[1][a] = cmul(w[a][0], h[1][0]);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                y[0][a] = cmac(y[0][a], w[a][b], h[0][b]);
                y[1][a] = cmac(y[1][a], w[a][b], h[1][b]);
            }
        }
        reconstruct_t(y, sf, acc);
        reconstruct_t(carry, -sf, acc);  // backward t hop
        mul_dag(w, hb, carry);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) stnt(o + (size_t)(3 * s + a) * V + site, acc[s][a]);
    }
}

// The same walk over t for lattices with Lx a multiple of 32 and Ly of 8:
// a workgroup owns a 32 x 8 (x, y) tile at one z, and at every step stages
// the tile's spinors (from the registers of their threads) and its 80-site
// x/y halo (from memory) in LDS, so the x and y hops read their neighbours
// there instead of fetching them again through the caches.
constexpr int WTX = 32, WTY = 8, WHALO = 2 * WTX + 2 * WTY;

template <typename T, typename A, bool DAG, int WTZ>
__global__ __launch_bounds__(256 * WTZ) void k_wilson_tile(Geom g, const T *__restrict__ U,
                                                           const T *__restrict__ in, T *__restrict__ out, A diag,
                                                           int tchunk) {
    __shared__ cx<A> lds_all[WTZ][12][WTY + 2][WTX + 2];
    const int lx = g.L[0], ly = g.L[1], lt = g.L[3];
    const int ntx = lx / WTX, nty = ly / WTY;
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const int tz = threadIdx.x / 256, tid = threadIdx.x % 256;
    const int x0 = (tile % ntx) * WTX, y0 = ((tile / ntx) % nty) * WTY, z = (tile / (ntx * nty)) * WTZ + tz;
    const int tx = tid % WTX, ty = tid / WTX;
    auto &lds = lds_all[tz];
    const int v3 = g.stride[3];
    const int s3 = (x0 + tx) + lx * ((y0 + ty) + ly * z);
    const int t0 = blockIdx.y * tchunk;
    const int t1 = min(t0 + tchunk, lt);
    const size_t V = (size_t)g.V;
    const T *q = in + (size_t)blockIdx.z * 12 * V;
    T *o = out + (size_t)blockIdx.z * 12 * V;
    const T *Ut = U + (size_t)3 * 9 * V;
    const A sf = DAG ? (A)-1 : (A)1;

    cx<A> carry[2][3], cur[4][3];
    {
        const int sb = s3 + (t0 == 0 ? lt - 1 : t0 - 1) * v3;
        cx<A> v[4][3], h[2][3], w[3][3];
        load_spinor(q + sb, V, v);
        project_t(v, -sf, h);
#pragma unroll
        for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(Ut + (size_t)e * V + sb);
        mul_dag(w, h, carry);
    }
    load_spinor(q + s3 + t0 * v3, V, cur);

#pragma unroll 1
    for (int t = t0; t < t1; ++t) {
        const int site = s3 + t * v3;
        __syncthreads();  // the previous step's readers of the tile are done
#pragma unroll
        for (int c = 0; c < 12; ++c) lds[c][ty + 1][tx + 1] = cur[c / 3][c % 3];
        for (int i = tid; i < 12 * WHALO; i += 256) {
            const int c = i / WHALO, h = i % WHALO;
            int hx, hy;
            if (h < WTX) { hx = h + 1; hy = 0; }
            else if (h < 2 * WTX) { hx = h - WTX + 1; hy = WTY + 1; }
            else if (h < 2 * WTX + WTY) { hx = 0; hy = h - 2 * WTX + 1; }
            else { hx = WTX + 1; hy = h - 2 * WTX - WTY + 1; }
            const int gx = (x0 + hx - 1 + lx) % lx, gy = (y0 + hy - 1 + ly) % ly;
            lds[c][hy][hx] = ldc<A>(q + (size_t)c * V + gx + lx * (gy + ly * z) + (size_t)t * v3);
        }
        __syncthreads();
        int c4[4];
        coords(g, site, c4);
        cx<A> acc[4][3], hb[2][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[s][a] = cscale(diag, cur[s][a]);
        project_t(cur, -sf, hb);
#pragma unroll 1
        for (int hop = 0; hop < 4; ++hop) {
            const int mu = hop >> 1;
            const bool fwd = (hop & 1) == 0;
            const int d = fwd ? 1 : -1;
            const int hx = tx + 1 + (mu == 0 ? d : 0), hy = ty + 1 + (mu == 1 ? d : 0);
            cx<A> v[4][3], w[3][3];
#pragma unroll
            for (int c = 0; c < 12; ++c) v[c / 3][c % 3] = lds[c][hy][hx];
            int ls = site;
            if (!fwd) {
                const int L = g.L[mu], str = g.stride[mu];
                const int cm = mu == 0 ? c4[0] : c4[1];
                ls = cm == 0 ? site + (L - 1) * str : site - str;
            }
            const T *p = U + (size_t)mu * 9 * V + ls;
#pragma unroll
            for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(p + (size_t)e * V);
            hop_core<DAG>(mu, fwd, v, w, acc);
        }
        // z hops: with two slices per workgroup the neighbour inside it
        // comes from the other slice's LDS tile
#pragma unroll 1
        for (int hop = 4; hop < 6; ++hop) {
            const bool fwd = hop == 4;
            if (WTZ == 2 && (fwd ? tz == 0 : tz == 1)) {
                cx<A> v[4][3], w[3][3];
#pragma unroll
                for (int c = 0; c < 12; ++c) v[c / 3][c % 3] = lds_all[1 - tz][c][ty + 1][tx + 1];
                const T *p = U + (size_t)2 * 9 * V + (fwd ? site : site - g.stride[2]);
#pragma unroll
                for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(p + (size_t)e * V);
                hop_core<DAG>(2, fwd, v, w, acc);
            } else {
                wilson_hop<DAG>(hop, g, c4, site, V, U, q, acc);
            }
        }
        const int sn = s3 + (t == lt - 1 ? 0 : t + 1) * v3;
        load_spinor(q + sn, V, cur);
        cx<A> w[3][3], h[2][3], y[2][3];
#pragma unroll
        for (int e = 0; e < 9; ++e) w[e / 3][e % 3] = ld<A>(Ut + (size_t)e * V + site);
        project_t(cur, sf, h);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            y[0][a] = cmul(w[a][0], h[0][0]);
            y[1][a] = cmul(w[a][0], h[1][0]);
#pragma unroll
            for (int b = 1; b < 3; ++b) {
                y[0][a] = cmac(y[0][a], w[a][b], h[0][b]);
                y[1][a] = cmac(y[1][a], w[a][b], h[1][b]);
            }
        }
        reconstruct_t(y, sf, acc);
        reconstruct_t(carry, -sf, acc);
        mul_dag(w, hb, carry);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) stnt(o + (size_t)(3 * s + a) * V + site, acc[s][a]);
    }
}

template <typename T, typename A>
hipError_t launch(const Geom &g, const void *U, const void *in, void *out, double diag, int nrhs, bool dag,
                  hipStream_t st) {
    const int lt = g.L[3], v3 = g.stride[3];
    // chunks of 8 t values (one halo spinor and link per 8 sites) unless that
    // leaves fewer than four workgroups per CU
    int tchunk = 8;
    while (tchunk > 1 && (long long)((v3 + 255) / 256) * ((lt + tchunk - 1) / tchunk) * nrhs < 1024) tchunk /= 2;
    const dim3 grid((v3 + 255) / 256, (lt + tchunk - 1) / tchunk, nrhs), block(256);
    if (g.L[0] % WTX == 0 && g.L[1] % WTY == 0) {
        if (g.L[2] % 2 == 0) {
            // v3 / 512 workgroups of two 32 x 8 tiles at z and z + 1
            const dim3 grid2(v3 / 512, grid.y, grid.z), block2(512);
            if (dag)
                k_wilson_tile<T, A, true, 2><<<grid2, block2, 0, st>>>(g, (const T *)U, (const T *)in, (T *)out,
                                                                       (A)diag, tchunk);
            else
                k_wilson_tile<T, A, false, 2><<<grid2, block2, 0, st>>>(g, (const T *)U, (const T *)in, (T *)out,
                                                                        (A)diag, tchunk);
            return hipGetLastError();
        }
        // v3 / 256 tiles of 32 x 8 sites, the same grid
        if (dag)
            k_wilson_tile<T, A, true, 1><<<grid, block, 0, st>>>(g, (const T *)U, (const T *)in, (T *)out, (A)diag,
                                                                 tchunk);
        else
            k_wilson_tile<T, A, false, 1><<<grid, block, 0, st>>>(g, (const T *)U, (const T *)in, (T *)out, (A)diag,
                                                                  tchunk);
        return hipGetLastError();
    }
    if (dag)
        k_wilson<T, A, true><<<grid, block, 0, st>>>(g, (const T *)U, (const T *)in, (T *)out, (A)diag, tchunk);
    else
        k_wilson<T, A, false><<<grid, block, 0, st>>>(g, (const T *)U, (const T *)in, (T *)out, (A)diag, tchunk);
    return hipGetLastError();
}

}  // namespace

hipError_t apply_wilson(const Geom &g, int prec, const void *U, const void *in, void *out, double diag,
                        int nrhs, bool dag, hipStream_t st) {
    if (prec == 0) return launch<double2, double>(g, U, in, out, diag, nrhs, dag, st);
    return launch<float2, float>(g, U, in, out, diag, nrhs, dag, st);
}

}  // namespace bri
