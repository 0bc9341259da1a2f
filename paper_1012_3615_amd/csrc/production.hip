// The ingredients of the paper's production operator (Sec. 5): projection to
// SU(3) (Sec. 5.2), one APE smearing step (Eq. def_ape), back-projection of
// the path-averaged transporters (Sec. 5.1) and the clover term of
// Eq. def_pref.  All arithmetic is FP64.
#include "kernels.h"
#include "stencil.h"
#include "su3.h"

namespace bri {

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_project_soa(const double2 *__restrict__ A, double2 *__restrict__ Y,
                                                        int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const M3 a = mload(A + i, (size_t)n);
    mstore(Y + i, (size_t)n, project_su3(a));
}

// in place on the FP64 40-offset stage [40][9][V]; the 1-hop planes hold the
// links themselves, which are already in SU(3), and are left alone
__global__ __launch_bounds__(kBlock) void k_project_w40(double2 *W40, int V) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= V) return;
    const int i = 41 + (int)blockIdx.y;
    if (off_k(i) < 2) return;
    double2 *p = W40 + (size_t)blockIdx.y * 9 * V + site;
    mstore(p, (size_t)V, project_su3(mload(p, (size_t)V)));
}

__device__ __forceinline__ M3 link(const double2 *U, size_t V, int mu, int site) {
    return mload(U + (size_t)mu * 9 * V + site, V);
}

// V_mu(x) = P_SU(3){(1-alpha) 1 + (alpha/6) sum_{+-nu != mu} loop} U_mu(x), the loop for
// +nu being U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag U_mu(x)^dag and for -nu
// U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^dag.
__global__ __launch_bounds__(kBlock) void k_ape(Geom g, const double2 *__restrict__ U, double2 *__restrict__ Vout,
                                                double alpha) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const int mu = blockIdx.y;
    const size_t V = (size_t)g.V;
    int c[4];
    coords(g, site, c);
    const Nbr nb = make_nbr(g, c);
    auto at = [&](int dmu, int smu, int dnu, int snu) {
        int d[4] = {0, 0, 0, 0};
        d[dmu] += smu;
        d[dnu] += snu;
        return nb.at(d[0], d[1], d[2], d[3]);
    };
    const M3 umu = link(U, V, mu, site);
    M3 st = mzero();
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        // U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
        const M3 up = mmuld(mmul(link(U, V, nu, site), link(U, V, mu, at(nu, 1, mu, 0))),
                            link(U, V, nu, at(mu, 1, nu, 0)));
        // U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu)
        const M3 dn = mmul(mdmul(link(U, V, nu, at(nu, -1, mu, 0)), link(U, V, mu, at(nu, -1, mu, 0))),
                           link(U, V, nu, at(nu, -1, mu, 1)));
        st = madd(st, madd(up, dn));
    }
    M3 m = mmuld(st, umu);
    const double a6 = alpha / 6.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m.m[i][j] = cscale(a6, m.m[i][j]);
#pragma unroll
    for (int i = 0; i < 3; ++i) m.m[i][i].re += 1.0 - alpha;
    mstore(Vout + (size_t)mu * 9 * V + site, V, mmul(project_su3(m), umu));
}

// Hermitian traceless clover-leaf field strength F_{mu nu}(x) = (Q - Q^dag)/(8i) - tr/3,
// Q the sum of the four plaquettes at x in the (mu, nu) plane.
__device__ inline M3 field_strength(const double2 *U, size_t V, const Nbr &nb, int site, int mu, int nu) {
    auto at = [&](int smu, int snu) {
        int d[4] = {0, 0, 0, 0};
        d[mu] += smu;
        d[nu] += snu;
        return nb.at(d[0], d[1], d[2], d[3]);
    };
    // x -> x+mu -> x+mu+nu -> x+nu -> x
    M3 q = mmuld(mmuld(mmul(link(U, V, mu, site), link(U, V, nu, at(1, 0))), link(U, V, mu, at(0, 1))),
                 link(U, V, nu, site));
    // x -> x+nu -> x+nu-mu -> x-mu -> x
    q = madd(q, mmul(mmuld(mmuld(link(U, V, nu, site), link(U, V, mu, at(-1, 1))), link(U, V, nu, at(-1, 0))),
                     link(U, V, mu, at(-1, 0))));
    // x -> x-mu -> x-mu-nu -> x-nu -> x
    q = madd(q, mmul(mmul(mdmul(link(U, V, mu, at(-1, 0)), mdag(link(U, V, nu, at(-1, -1)))),
                          link(U, V, mu, at(-1, -1))),
                     link(U, V, nu, at(0, -1))));
    // x -> x-nu -> x-nu+mu -> x+mu -> x
    q = madd(q, mmuld(mmul(mdmul(link(U, V, nu, at(0, -1)), link(U, V, mu, at(0, -1))), link(U, V, nu, at(1, -1))),
                      link(U, V, mu, site)));
    // (Q - Q^dag)/(8i): element (a,b) = (q_ab - conj(q_ba)) * (-i/8)
    M3 f;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cd d = csub(q.m[a][b], cconj(q.m[b][a]));
            f.m[a][b] = cmake(d.im / 8.0, -d.re / 8.0);
        }
    const double tr = (f.m[0][0].re + f.m[1][1].re + f.m[2][2].re) / 3.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) f.m[a][a].re -= tr;
    return f;
}

// -(c_SW/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu} in the chiral basis is block
// diagonal: on spins (0,1) and on (2,3) it is sum_m sigma_m (x) G_m with the
// Pauli matrices sigma_m and
//   G_x = (c/2)(F_yz -+ F_xt),  G_y = (c/2)(-F_xz -+ F_yt),  G_z = (c/2)(F_xy -+ F_zt)
// (upper sign on spins 0,1).  Block entry [(s,a),(s',b)], local index 3s+a:
//   [0,0] = G_z, [1,1] = -G_z, [0,1] = G_x - i G_y, [1,0] = G_x + i G_y.
// Stored per block as 18 complex planes: three planes holding the real
// diagonal in pairs (M_00, M_11), (M_22, M_33), (M_44, M_55), then the 15
// entries M_ij, i < j, row by row.  Layout [2][18][V].
template <typename CS>
__global__ __launch_bounds__(kBlock) void k_clover(Geom g, const double2 *__restrict__ U, CS *__restrict__ C,
                                                   double csw) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const size_t V = (size_t)g.V;
    int c[4];
    coords(g, site, c);
    const Nbr nb = make_nbr(g, c);
    const double h = 0.5 * csw;
    // one chirality block at a time (the field strengths are recomputed for the second)
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const double sg = blk == 0 ? -1.0 : 1.0;
        M3 gx = mzero(), gy = mzero(), gz = mzero();
        auto add = [&](M3 &gm, int mu, int nu, double w) {
            const M3 f = field_strength(U, V, nb, site, mu, nu);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) gm.m[a][b] = caxpy(w * h, f.m[a][b], gm.m[a][b]);
        };
        add(gx, 1, 2, 1.0);   // G_x: F_yz
        add(gx, 0, 3, sg);    //      -+ F_xt
        add(gy, 0, 2, -1.0);  // G_y: -F_xz
        add(gy, 1, 3, sg);    //      -+ F_yt
        add(gz, 0, 1, 1.0);   // G_z: F_xy
        add(gz, 2, 3, sg);    //      -+ F_zt
        // entry (i, j) of the 6x6 block, i = 3s + a, j = 3s' + b
        auto entry = [&](int i, int j) -> cd {
            const int s1 = i / 3, a = i % 3, s2 = j / 3, b = j % 3;
            const cd ex = gx.m[a][b], ey = gy.m[a][b], ez = gz.m[a][b];
            if (s1 == 0 && s2 == 0) return ez;
            if (s1 == 1 && s2 == 1) return cscale(-1.0, ez);
            if (s1 == 0) return cmake(ex.re + ey.im, ex.im - ey.re);  // G_x - i G_y
            return cmake(ex.re - ey.im, ex.im + ey.re);               // G_x + i G_y
        };
        CS *o = C + (size_t)blk * 18 * V + site;
#pragma unroll
        for (int p = 0; p < 3; ++p) st(o + p * V, cmake(entry(2 * p, 2 * p).re, entry(2 * p + 1, 2 * p + 1).re));
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i + 1; j < 6; ++j) st(o + clover_plane(i, j) * V, entry(i, j));
    }
}

// W40 (FP64) -> two-row store: rows 0 and 1 of every transporter (the third
// row of an SU(3) matrix follows from them).  One thread per (site x,
// canonical offset n), as in the full conversion: rows 0, 1 of W(x, x+n) at
// x and, for 80 offsets, rows 0, 1 of W(x, x+n)^dag at x+n under -n.
template <typename WT>
__global__ __launch_bounds__(kBlock) void k_convert_rows2(Geom g, const double2 *__restrict__ W40,
                                                          WT *__restrict__ W, int noff) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const int c = blockIdx.y;
    const int i = 41 + c;
    const size_t V = (size_t)g.V;
    const double2 *p = W40 + (size_t)c * 9 * V + site;
    cd m[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = ldc<double>(p + e * V);
    WT *o = W + (size_t)(noff == 80 ? i - 1 : c) * 6 * V + site;
#pragma unroll
    for (int e = 0; e < 6; ++e) st(o + e * V, m[e]);
    if (noff == 80) {
        int cc[4];
        coords(g, site, cc);
        const Nbr nb = make_nbr(g, cc);
        const int y = nb.at(off_n(i, 0), off_n(i, 1), off_n(i, 2), off_n(i, 3));
        WT *ob = W + (size_t)(80 - i) * 6 * V + y;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int a = e / 3, b = e % 3;
            st(ob + e * V, cconj(m[3 * b + a]));
        }
    }
}

}  // namespace

hipError_t project_su3_soa(const double2 *A, double2 *Y, int64_t n, hipStream_t st) {
    const int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_project_soa, dim3((unsigned)nb), dim3(kBlock), 0, st, A, Y, n);
    return hipGetLastError();
}

hipError_t project_w40(const Geom &g, double2 *W40, hipStream_t st) {
    hipLaunchKernelGGL(k_project_w40, dim3((g.V + kBlock - 1) / kBlock, 40), dim3(kBlock), 0, st, W40, g.V);
    return hipGetLastError();
}

hipError_t ape_smear(const Geom &g, const double2 *U, double2 *Vout, double alpha, hipStream_t st) {
    hipLaunchKernelGGL(k_ape, dim3((g.V + kBlock - 1) / kBlock, 4), dim3(kBlock), 0, st, g, U, Vout, alpha);
    return hipGetLastError();
}

hipError_t build_clover(const Geom &g, const double2 *U, void *C, int cp, double csw, hipStream_t st) {
    dim3 grid((g.V + kBlock - 1) / kBlock);
    if (cp == 0)
        hipLaunchKernelGGL(k_clover<double2>, grid, dim3(kBlock), 0, st, g, U, (double2 *)C, csw);
    else if (cp == 1)
        hipLaunchKernelGGL(k_clover<float2>, grid, dim3(kBlock), 0, st, g, U, (float2 *)C, csw);
    else if (cp == 2)
        hipLaunchKernelGGL(k_clover<__half2>, grid, dim3(kBlock), 0, st, g, U, (__half2 *)C, csw);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t convert_w40_rows2(const Geom &g, const double2 *W40, void *W, int wp, int noff, hipStream_t st) {
    dim3 grid((g.V + kBlock - 1) / kBlock, 40);
    if (wp == 0)
        hipLaunchKernelGGL(k_convert_rows2<double2>, grid, dim3(kBlock), 0, st, g, W40, (double2 *)W, noff);
    else if (wp == 1)
        hipLaunchKernelGGL(k_convert_rows2<float2>, grid, dim3(kBlock), 0, st, g, W40, (float2 *)W, noff);
    else if (wp == 2)
        hipLaunchKernelGGL(k_convert_rows2<__half2>, grid, dim3(kBlock), 0, st, g, W40, (__half2 *)W, noff);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace bri
