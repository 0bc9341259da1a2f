// Gradient of S = Re sum_rhs <chi, D psi> with respect to the links, through
// the path averaging of the transporters (FP64).  g = dS/dRe U + i dS/dIm U.
// D is the Brillouin operator or, with a coefficient table, any member of
// the generic class of Sec. 8 (lambda_k, rho_k enter only the direct terms).
//
// 1. Per site x and offset n the transporter receives
//      G_n(x) = sum_rhs sum_s (C(n)^dag chi(x))_s psi_s(x+n)^dag,
//    C(n) = lambda_k + rho_k sum_mu n_mu gamma_mu (Hermitian, so C^dag = C).
// 2. Every transporter obeys the same-site recursion used to build it,
//      W(x,n) = (1/k) sum_{mu in supp n} W(x, n - s_mu mu) L(x,n,mu),
//      L = U_mu(x+n-mu) (s_mu = +1) or U_mu(x+n)^dag (s_mu = -1),
//    so G_{n - s_mu mu}(x) receives (1/k) G_n(x) L^dag.  Steps 1 and 2 run
//    together, one launch per hop count in reverse order (4 -> 1): each
//    lower-level gradient pulls these terms from its parents, which are
//    final by then.
// 3. Each link collects, without atomics, the product-rule terms of every
//    (x, n, mu) whose last step runs over it:
//      s_mu = +1: U_mu(y), y = x+n-mu:  += (1/k) W(x, n-mu)^dag G_n(x)
//      s_mu = -1: U_mu(y), y = x+n:     += (1/k) G_n(x)^dag W(x, n+mu)
//    with W(x, 0) = 1.
#include <cmath>

#include "abi_internal.h"
#include "apply_recompute.h"
#include "kernels.h"

namespace bri {
namespace {

constexpr int kB = 256;

__device__ __forceinline__ int plane80_rt(int i) { return i < 40 ? i : i - 1; }

__device__ __forceinline__ void ldm(const double2 *p, size_t V, cx<double> m[3][3]) {
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e / 3][e % 3] = ldc<double>(p + e * V);
}
__device__ __forceinline__ void stm(double2 *p, size_t V, const cx<double> m[3][3]) {
#pragma unroll
    for (int e = 0; e < 9; ++e) st(p + e * V, m[e / 3][e % 3]);
}

// site x + d (periodic) from the coordinates of x, by integer arithmetic (a
// table of neighbour indices would be indexed at run time, i.e. in scratch)
__device__ __forceinline__ int site_at(const Geom &g, const int c[4], int d0, int d1, int d2, int d3) {
    auto w = [](int v, int L) { return v < 0 ? v + L : (v >= L ? v - L : v); };
    return w(c[0] + d0, g.L[0]) +
           g.L[0] * (w(c[1] + d1, g.L[1]) + g.L[1] * (w(c[2] + d2, g.L[2]) + g.L[2] * w(c[3] + d3, g.L[3])));
}

// direct gradient of the transporter of offset n (K hops) at the site
// (y = x + n): G = sum_rhs sum_s (C(n) chi(x))_s psi_s(x+n)^dag
template <int K>
__device__ inline void grad_direct(int site, int y, size_t V, const double2 *__restrict__ chi,
                                   const double2 *__restrict__ psi, int nrhs, const int n[4], const Coef<double> &cf,
                                   cx<double> G[3][3]) {
    const double lam = cf.lam[K], rho = cf.rho[K];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) G[a][b] = cmake(0.0, 0.0);
    for (int r = 0; r < nrhs; ++r) {
        const double2 *xc = chi + (size_t)r * 12 * V + site;
        const double2 *ps = psi + (size_t)r * 12 * V + y;
        cx<double> ch[4][3], pp[4][3];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ch[s][a] = ldc<double>(xc + (3 * s + a) * V);
                pp[s][a] = ldc<double>(ps + (3 * s + a) * V);
            }
        // phi = C(n) chi, colour by colour
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<double> in4[4] = {ch[0][a], ch[1][a], ch[2][a], ch[3][a]};
            cx<double> o[4] = {cmake(0.0, 0.0), cmake(0.0, 0.0), cmake(0.0, 0.0), cmake(0.0, 0.0)};
            spin_accum_rt(o, in4, lam, rho, n[0], n[1], n[2], n[3]);
            // G[a][b] += sum_s phi_s[a] conj(psi_s[b])
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int s = 0; s < 4; ++s) G[a][b] = cmac(G[a][b], o[s], cconj(pp[s][b]));
        }
    }
}

// Offsets of each hop count k (index i = (nx+1) + 3(ny+1) + 9(nz+1) + 27(nt+1),
// increasing): 1, 8, 24, 32, 16 of them.
// Steps 1 and 2 in one kernel, through the hop levels 4 -> 1: the full
// gradient of the transporter of offset P (k hops) is its direct term plus
// what its parents p = P + s e_nu (nu outside the support of P, s = +-1; one
// hop more) pass down through their last link,
//   G_P += (1/|p|) G_p L^dag,  L = U_nu(x+P) (s = +1) or U_nu(x+P-nu)^dag (s = -1),
// the reverse of the same-site recursion that builds the transporters.  16
// consecutive sites x 32 threads per workgroup; every G of a level is written
// to G80 for the gather and kept in LDS, where the next level pulls it
// (levels 4 and 2 in one buffer, level 3 in the other: 129 KB, one
// workgroup per CU; one launch per level, with the parents read back from
// memory, took 1.1 ms at 16^3 x 32).  Each wavefront takes
// offsets of one support at a time, its four roles sign combinations, so the
// directions without a parent pull are the same across the wavefront:
//   four hops: wave w < 4, sign bits 4 w + role (bit mu: n_mu = -1);
//   three hops: wave w, the support without direction w / 2, sign bits
//     4 (w % 2) + role over the support in increasing order;
//   two hops: wave w < 6, the direction pair w (pair_lo, pair_hi), role the signs;
//   one hop: wave w < 4, direction w, role 0 / 1 the sign.
// LDS slots: level 4 its sign bits, level 3 8 Q + sign bits, level 2 4 P +
// sign bits (the slot layout of the recompute apply).
__device__ __forceinline__ int grad_slot(const int (&p)[4], int k) {
    if (k == 4) return (p[0] < 0) | ((p[1] < 0) << 1) | ((p[2] < 0) << 2) | ((p[3] < 0) << 3);
    if (k == 3) {
        const int q = p[0] == 0 ? 0 : p[1] == 0 ? 1 : p[2] == 0 ? 2 : 3;
        int b = 0, j = 0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu)
            if (mu != q) b |= (p[mu] < 0) << j++;
        return 8 * q + b;
    }
    // k == 2 (selects, not run-time indices, which would place p in scratch)
    const int lo = p[0] != 0 ? 0 : p[1] != 0 ? 1 : 2;
    const int hi = p[3] != 0 ? 3 : p[2] != 0 ? 2 : 1;
    const int plo = lo == 0 ? p[0] : lo == 1 ? p[1] : p[2];
    const int phi = hi == 3 ? p[3] : hi == 2 ? p[2] : p[1];
    return 4 * pair_index(lo, hi) + (plo < 0) + 2 * (phi < 0);
}

template <int K>
__device__ __forceinline__ void grad_level_task(const Geom &g, const int (&n)[4], const int (&c)[4], int site,
                                                bool valid, int sl, const double2 *__restrict__ U,
                                                const double2 *__restrict__ chi, const double2 *__restrict__ psi,
                                                int nrhs, double2 *__restrict__ G80, const Coef<double> &cf,
                                                cx<double> (*prev)[9][16], cx<double> (*cur)[9][16], int cslot) {
    const size_t V = (size_t)g.V;
    const int i = (n[0] + 1) + 3 * (n[1] + 1) + 9 * (n[2] + 1) + 27 * (n[3] + 1);
    const double inv = 1.0 / (K + 1);
    cx<double> G[3][3];
    grad_direct<K>(site, site_at(g, c, n[0], n[1], n[2], n[3]), V, chi, psi, nrhs, n, cf, G);
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        if (K == 4 || n[nu] != 0) continue;
#pragma unroll
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            int p[4] = {n[0], n[1], n[2], n[3]};
            p[nu] = sgn;
            cx<double> Gp[3][3];
            lds_get<double, 16>(prev, grad_slot(p, K + 1), sl, Gp);
            // the parent's last link: base site x+P (forward) or x+P-nu (backward)
            int d[4] = {n[0], n[1], n[2], n[3]};
            if (sgn < 0) d[nu] = -1;
            const int yl = site_at(g, c, d[0], d[1], d[2], d[3]);
            cx<double> l[3][3];
            const double2 *pu = U + (size_t)nu * 9 * V + yl;
#pragma unroll
            for (int e = 0; e < 9; ++e) {
                cx<double> v = ldc<double>(pu + e * V);
                if (sgn > 0) l[e / 3][e % 3] = v; else l[e % 3][e / 3] = cconj(v);
            }
            // G += inv * Gp * l^dag
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    cx<double> t = cmake(0.0, 0.0);
#pragma unroll
                    for (int q = 0; q < 3; ++q) t = cmac(t, Gp[a][q], cconj(l[b][q]));
                    G[a][b] = caxpy(inv, t, G[a][b]);
                }
        }
    }
    if (cur) lds_put<double, 16>(cur, cslot, sl, G);
    if (valid) stm(G80 + (size_t)plane80_rt(i) * 9 * V + site, V, G);
}

__global__ __launch_bounds__(512) void k_grad_fused(Geom g, const double2 *__restrict__ U,
                                                    const double2 *__restrict__ chi, const double2 *__restrict__ psi,
                                                    int nrhs, double2 *__restrict__ G80, Coef<double> cf, int gy,
                                                    int gz) {
    constexpr int S = 16;
    __shared__ cx<double> bufA[24][9][S];  // four hops, then two hops
    __shared__ cx<double> bufB[32][9][S];  // three hops
    const int sl = threadIdx.x % S;
    const int role = (threadIdx.x / S) % 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int s0 = strip_base(g, xcd_block(blockIdx.x, gridDim.x), gy, gz) + sl;
    const bool valid = s0 < g.V;
    const int site = valid ? s0 : 0;
    int c[4];
    coords(g, site, c);

    if (wave < 4) {  // four hops
        const int bits = 4 * wave + role;
        const int n[4] = {(bits & 1) ? -1 : 1, (bits & 2) ? -1 : 1, (bits & 4) ? -1 : 1, (bits & 8) ? -1 : 1};
        grad_level_task<4>(g, n, c, site, valid, sl, U, chi, psi, nrhs, G80, cf, nullptr, bufA, bits);
    }
    __syncthreads();
    {  // three hops
        const int q = wave >> 1, bits = 4 * (wave & 1) + role;
        int n[4], j = 0;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) n[mu] = mu == q ? 0 : (((bits >> j++) & 1) ? -1 : 1);
        grad_level_task<3>(g, n, c, site, valid, sl, U, chi, psi, nrhs, G80, cf, bufA, bufB, 8 * q + bits);
    }
    __syncthreads();
    if (wave < 6) {  // two hops (level 4 in bufA is no longer read)
        const int lo = pair_lo(wave), hi = pair_hi(wave);
        int n[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) n[mu] = mu == lo ? ((role & 1) ? -1 : 1) : mu == hi ? ((role & 2) ? -1 : 1) : 0;
        grad_level_task<2>(g, n, c, site, valid, sl, U, chi, psi, nrhs, G80, cf, bufB, bufA, 4 * wave + role);
    }
    __syncthreads();
    if (wave < 4 && role < 2) {  // one hop
        int n[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) n[mu] = mu == wave ? (role ? -1 : 1) : 0;
        grad_level_task<1>(g, n, c, site, valid, sl, U, chi, psi, nrhs, G80, cf, bufA, nullptr, 0);
    }
}

// step 3: gather onto the links; the lower-level transporter W(x, m) is read
// from the 40-offset FP64 store, at x when m is stored there, otherwise as
// W(x+m, x)^dag from x+m.  The four directions of a block of sites are
// consecutive blocks on one XCD: they read the same G and W planes around
// those sites, which then come from that XCD's L2.
__global__ __launch_bounds__(kB) void k_grad_gather(Geom g, const double2 *__restrict__ W40,
                                                    const double2 *__restrict__ G80,
                                                    double2 *__restrict__ gradU, double scale) {
    const int lin = xcd_block(blockIdx.x, gridDim.x);
    const int mu = lin % 4;
    const int site = (lin / 4) * kB + threadIdx.x;
    if (site >= g.V) return;
    const size_t V = (size_t)g.V;
    int c[4];
    coords(g, site, c);
    cx<double> acc[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[a][b] = cmake(0.0, 0.0);
#pragma unroll 1
    for (int i = 0; i < 81; ++i) {
        const int n[4] = {i % 3 - 1, (i / 3) % 3 - 1, (i / 9) % 3 - 1, i / 27 - 1};
        if (n[mu] == 0) continue;
        const int k = (n[0] != 0) + (n[1] != 0) + (n[2] != 0) + (n[3] != 0);
        // site x of the transporter: y = x+n-mu (forward) or y = x+n (backward)
        int xc[4];
        for (int nu = 0; nu < 4; ++nu) {
            int v = c[nu] - n[nu] + ((nu == mu && n[mu] > 0) ? 1 : 0);
            const int L = g.L[nu];
            v = (v % L + L) % L;
            xc[nu] = v;
        }
        const int x = xc[0] + g.L[0] * (xc[1] + g.L[1] * (xc[2] + g.L[2] * xc[3]));
        cx<double> G[3][3], P[3][3];
        ldm(G80 + (size_t)plane80_rt(i) * 9 * V + x, V, G);
        int m[4] = {n[0], n[1], n[2], n[3]};
        m[mu] = 0;
        const int im = (m[0] + 1) + 3 * (m[1] + 1) + 9 * (m[2] + 1) + 27 * (m[3] + 1);
        if (im == 40) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) P[a][b] = cmake(a == b ? 1.0 : 0.0, 0.0);
        } else if (im > 40) {
            ldm(W40 + (size_t)(im - 41) * 9 * V + x, V, P);
        } else {
            int yc[4];
            for (int nu = 0; nu < 4; ++nu) {
                const int L = g.L[nu];
                yc[nu] = (xc[nu] + m[nu] + L) % L;
            }
            const int y = yc[0] + g.L[0] * (yc[1] + g.L[1] * (yc[2] + g.L[2] * yc[3]));
            cx<double> Q[3][3];
            ldm(W40 + (size_t)(80 - im - 41) * 9 * V + y, V, Q);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) P[a][b] = cconj(Q[b][a]);
        }
        const double inv = 1.0 / k;
        if (n[mu] > 0) {
            // acc += inv * P^dag G
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    cx<double> t = cmake(0.0, 0.0);
#pragma unroll
                    for (int q = 0; q < 3; ++q) t = cmac(t, cconj(P[q][a]), G[q][b]);
                    acc[a][b] = caxpy(inv, t, acc[a][b]);
                }
        } else {
            // acc += inv * G^dag P
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    cx<double> t = cmake(0.0, 0.0);
#pragma unroll
                    for (int q = 0; q < 3; ++q) t = cmac(t, cconj(G[q][a]), P[q][b]);
                    acc[a][b] = caxpy(inv, t, acc[a][b]);
                }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[a][b] = cscale(scale, acc[a][b]);
    stm(gradU + (size_t)mu * 9 * V + site, V, acc);
}

}  // namespace
}  // namespace bri

using namespace bri;

extern "C" {

size_t bri_grad_workspace_bytes(bri_dims d) {
    Geom g;
    if (!dims_ok(d, &g)) return 0;
    return (size_t)g.V * 9 * 16 * (40 + 80);
}

size_t bri_grad_workspace_bytes_w(bri_dims d) {
    Geom g;
    if (!dims_ok(d, &g)) return 0;
    return (size_t)g.V * 9 * 16 * 80;
}

}  // extern "C"

namespace bri {
namespace {

// the three gradient steps with given FP64 40-offset transporters W40 and the
// transporter-gradient store G80
bri_status grad_steps(const Geom &g, const double *U, const double2 *W40, const double *chi, const double *psi,
                      int nrhs, double scale, const double *coef, double *gradU, double2 *G80, hipStream_t st) {
    dim3 grid((g.V + kB - 1) / kB);
    const Coef<double> cf = make_coef<double>(coef);
    int gy, gz;
    strip_groups(g, gy, gz);
    hipLaunchKernelGGL(k_grad_fused, dim3((g.V + 15) / 16), dim3(512), 0, st, g, (const double2 *)U,
                       (const double2 *)chi, (const double2 *)psi, nrhs, G80, cf, gy, gz);
    hipLaunchKernelGGL(k_grad_gather, dim3(grid.x * 4), dim3(kB), 0, st, g, W40, (const double2 *)G80,
                       (double2 *)gradU, scale);
    return hip_check(hipGetLastError(), "gradient kernels");
}

bri_status grad_check(bri_dims d, Geom *g, const double *U, const double *chi, const double *psi, int32_t nrhs,
                      const double *coef, double *gradU) {
    if (!dims_ok(d, g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (coef)
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(coef[i])) return fail(BRI_E_ARG, "coefficient %d of the table is not finite", i);
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!aligned(U) || !aligned(chi) || !aligned(psi) || !aligned(gradU))
        return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t lb = (size_t)g->V * 36 * 16;
    if (overlap(gradU, lb, U, lb)) return fail(BRI_E_ARG, "gradU overlaps the links");
    return BRI_OK;
}

}  // namespace
}  // namespace bri

extern "C" {

bri_status bri_grad_links(bri_dims d, const double *U, const double *chi, const double *psi,
                          int32_t nrhs, double scale, const double *coef, double *gradU, void *work,
                          size_t work_bytes, void *stream) {
    g_last_error.clear();
    Geom g;
    bri_status s = grad_check(d, &g, U, chi, psi, nrhs, coef, gradU);
    if (s != BRI_OK) return s;
    const size_t need = bri_grad_workspace_bytes(d);
    if (!aligned(work) || work_bytes < need)
        return fail(BRI_E_WORKSPACE, "workspace too small: need %zu bytes", need);
    if (overlap(work, need, gradU, (size_t)g.V * 36 * 16))
        return fail(BRI_E_ARG, "gradU overlaps the workspace");
    hipStream_t st = (hipStream_t)stream;
    double2 *W40 = (double2 *)work;
    double2 *G80 = W40 + (size_t)40 * 9 * g.V;
    // transporters rebuilt from the links (not kept from the forward pass)
    s = hip_check(build_w40_f64(g, (const double2 *)U, W40, st), "build transporters");
    if (s != BRI_OK) return s;
    return grad_steps(g, U, W40, chi, psi, nrhs, scale, coef, gradU, G80, st);
}

bri_status bri_grad_links_w(bri_dims d, const double *U, const double *W40, const double *chi, const double *psi,
                            int32_t nrhs, double scale, const double *coef, double *gradU, void *work,
                            size_t work_bytes, void *stream) {
    g_last_error.clear();
    Geom g;
    bri_status s = grad_check(d, &g, U, chi, psi, nrhs, coef, gradU);
    if (s != BRI_OK) return s;
    if (!aligned(W40)) return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t need = bri_grad_workspace_bytes_w(d);
    if (!aligned(work) || work_bytes < need)
        return fail(BRI_E_WORKSPACE, "workspace too small: need %zu bytes", need);
    if (overlap(work, need, gradU, (size_t)g.V * 36 * 16) || overlap(work, need, W40, (size_t)g.V * 40 * 9 * 16))
        return fail(BRI_E_ARG, "the workspace overlaps gradU or the transporters");
    return grad_steps(g, U, (const double2 *)W40, chi, psi, nrhs, scale, coef, gradU, (double2 *)work,
                      (hipStream_t)stream);
}

}  // extern "C"
