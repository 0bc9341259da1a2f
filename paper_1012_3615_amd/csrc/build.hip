// Construction of the gauge transporters W(x, x+n) (Sec. 5.1): the average of
// the link products over all k! shortest paths from x to x+n.
//
// The k-hop transporters follow from the (k-1)-hop ones at the same site by
// splitting off the last step of every path:
//   W(x, x+n) = (1/k) sum_{mu in supp n} W(x, x+n-s_mu mu) L(n, mu),
//   L(n, mu) = U_mu(x+n-mu)      if s_mu = +1,
//            = U_mu(x+n)^dag     if s_mu = -1,
// (grouping the k! paths by their last direction gives k groups of (k-1)!
// paths, each of which is the (k-1)-hop average times the last link).
// Levels are built in separate launches (1, 2, 3, 4 hops), one thread per
// (site, offset), in FP64, into the 40-offset store (offsets whose last non-zero component is +1); the other
// orientation of a lower-level transporter is read through
// W(x, x+m) = W(x+m, x)^dag.
#include "common.h"
#include "kernels.h"

namespace bri {

namespace {

__device__ __forceinline__ void load_mat(const double2 *p, size_t V, bool dagger, cx<double> m[3][3]) {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        cx<double> v = ldc<double>(p + e * V);
        if (dagger)
            m[e % 3][e / 3] = cconj(v);
        else
            m[e / 3][e % 3] = v;
    }
}

// The canonical offsets (i > 40) of each hop count: 4, 12, 16, 8 of them.
struct CanonLevels {
    signed char idx[5][16];
    int count[5];
};
constexpr CanonLevels make_canon() {
    CanonLevels t{};
    for (int i = 41; i < 81; ++i) {
        const int k = off_k(i);
        t.idx[k][t.count[k]++] = (signed char)i;
    }
    return t;
}
constexpr CanonLevels kCanon = make_canon();
__constant__ CanonLevels c_canon = make_canon();

// One thread per (site, canonical offset of the level): the offsets of a
// block of sites are consecutive blocks on one XCD, so the lower-level
// transporters and links they share are read through its L2.  The offset
// is uniform in a block; its code is selected by a uniform branch, so the
// offset arithmetic stays compile-time.
// Wout (optional): the target store (precision WT, 40 or 80 offsets), written
// as soon as a transporter is final (the cast fused into the build: own plane
// at x and, for 80 offsets, the adjoint at x+n under -n).  keep_stage = false
// skips the FP64 stage write (the last level, whose stage nothing reads).
template <int K, typename WT>
__global__ __launch_bounds__(256) void k_build_level(Geom g, const double2 *__restrict__ U,
                                                     double2 *__restrict__ W40, WT *__restrict__ Wout, int noff,
                                                     bool keep_stage) {
    constexpr int cnt = kCanon.count[K];
    const int lin = xcd_block(blockIdx.x, gridDim.x);
    const int site = (lin / cnt) * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const int target = c_canon.idx[K][lin % cnt];
    const size_t V = (size_t)g.V;
    int c[4];
    coords(g, site, c);
    const Nbr nb = make_nbr(g, c);

    static_for<41, 81>([&](auto I) {
        constexpr int i = decltype(I)::value;
        if constexpr (off_k(i) == K) {
            if (i != target) return;
            constexpr int n[4] = {off_n(i, 0), off_n(i, 1), off_n(i, 2), off_n(i, 3)};
            cx<double> acc[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) acc[a][b] = cmake(0.0, 0.0);
            static_for<0, 4>([&](auto M) {
                constexpr int mu = decltype(M)::value;
                if constexpr (n[mu] != 0) {
                    // last link L(n, mu)
                    constexpr int sm = n[mu];
                    int dl[4] = {n[0], n[1], n[2], n[3]};
                    if (sm > 0) dl[mu] -= 1;
                    const int yl = nb.at(dl[0], dl[1], dl[2], dl[3]);
                    cx<double> l[3][3];
                    load_mat(U + (size_t)mu * 9 * V + yl, V, sm < 0, l);
                    if constexpr (K == 1) {
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int b = 0; b < 3; ++b) acc[a][b] = cadd(acc[a][b], l[a][b]);
                    } else {
                        // predecessor m = n - s_mu mu
                        constexpr int m0 = mu == 0 ? 0 : n[0], m1 = mu == 1 ? 0 : n[1],
                                      m2 = mu == 2 ? 0 : n[2], m3 = mu == 3 ? 0 : n[3];
                        constexpr int im = off_index(m0, m1, m2, m3);
                        cx<double> p[3][3];
                        if constexpr (is_canonical(im)) {
                            load_mat(W40 + (size_t)plane40(im) * 9 * V + site, V, false, p);
                        } else {
                            const int ym = nb.at(m0, m1, m2, m3);
                            load_mat(W40 + (size_t)plane40(80 - im) * 9 * V + ym, V, true, p);
                        }
#pragma unroll
                        for (int a = 0; a < 3; ++a)
#pragma unroll
                            for (int b = 0; b < 3; ++b) {
                                cx<double> t = acc[a][b];
                                t = cmac(t, p[a][0], l[0][b]);
                                t = cmac(t, p[a][1], l[1][b]);
                                acc[a][b] = cmac(t, p[a][2], l[2][b]);
                            }
                    }
                }
            });
            constexpr double inv = 1.0 / K;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) acc[a][b] = cscale(inv, acc[a][b]);
            if (keep_stage) {
                double2 *o = W40 + (size_t)plane40(i) * 9 * V + site;
#pragma unroll
                for (int e = 0; e < 9; ++e) st(o + e * V, acc[e / 3][e % 3]);
            }
            if (Wout) {
                WT *o = Wout + (size_t)(noff == 80 ? i - 1 : plane40(i)) * 9 * V + site;
#pragma unroll
                for (int e = 0; e < 9; ++e) st(o + e * V, acc[e / 3][e % 3]);
                if (noff == 80) {
                    const int y = nb.at(n[0], n[1], n[2], n[3]);
                    WT *ob = Wout + (size_t)(80 - i) * 9 * V + y;  // plane of offset 80 - i (< 40)
#pragma unroll
                    for (int e = 0; e < 9; ++e) st(ob + e * V, cconj(acc[e % 3][e / 3]));
                }
            }
        }
    });
}

// W40 (FP64) -> target store (precision WT, 40 or 80 offsets).  One thread
// per (site x, canonical offset n): it reads W(x, x+n) once and writes it to
// the plane of n at x and, in the 80-offset store, its adjoint to the plane
// of -n at x+n (W(x+n, x) = W(x, x+n)^dag); every output element is written
// by exactly one thread.
template <typename WT>
__global__ __launch_bounds__(256) void k_convert(Geom g, const double2 *__restrict__ W40,
                                                 WT *__restrict__ W, int noff) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= g.V) return;
    const int c = blockIdx.y;  // canonical plane, offset i = 41 + c
    const int i = 41 + c;
    const size_t V = (size_t)g.V;
    const double2 *p = W40 + (size_t)c * 9 * V + site;
    cx<double> m[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = ldc<double>(p + e * V);
    WT *o = W + (size_t)(noff == 80 ? i - 1 : c) * 9 * V + site;
#pragma unroll
    for (int e = 0; e < 9; ++e) st(o + e * V, m[e]);
    if (noff == 80) {
        int cc[4];
        coords(g, site, cc);
        const Nbr nb = make_nbr(g, cc);
        const int y = nb.at(off_n(i, 0), off_n(i, 1), off_n(i, 2), off_n(i, 3));
        WT *ob = W + (size_t)(80 - i) * 9 * V + y;  // plane of offset 80 - i (< 40)
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            // element (a,b) of the adjoint = conj of element (b,a)
            const int a = e / 3, b = e % 3;
            st(ob + e * V, cconj(m[3 * b + a]));
        }
    }
}

constexpr int kBlock = 256;
}  // namespace

namespace {
template <typename WT>
hipError_t build_levels(const Geom &g, const double2 *U, double2 *W40, WT *Wout, int noff, hipStream_t st) {
    const unsigned nb = (g.V + kBlock - 1) / kBlock;
    const bool last_stage = Wout == nullptr;  // the 4-hop stage is read only when it is the output
    hipLaunchKernelGGL((k_build_level<1, WT>), dim3(nb * kCanon.count[1]), dim3(kBlock), 0, st, g, U, W40, Wout,
                       noff, true);
    hipLaunchKernelGGL((k_build_level<2, WT>), dim3(nb * kCanon.count[2]), dim3(kBlock), 0, st, g, U, W40, Wout,
                       noff, true);
    hipLaunchKernelGGL((k_build_level<3, WT>), dim3(nb * kCanon.count[3]), dim3(kBlock), 0, st, g, U, W40, Wout,
                       noff, true);
    hipLaunchKernelGGL((k_build_level<4, WT>), dim3(nb * kCanon.count[4]), dim3(kBlock), 0, st, g, U, W40, Wout,
                       noff, last_stage);
    return hipGetLastError();
}
}  // namespace

hipError_t build_w40_f64(const Geom &g, const double2 *U, double2 *W40, hipStream_t st) {
    return build_levels<double2>(g, U, W40, nullptr, 40, st);
}

hipError_t build_cast(const Geom &g, const double2 *U, double2 *stage, void *W, int wp, int noff, hipStream_t st) {
    if (wp == 0) return build_levels<double2>(g, U, stage, (double2 *)W, noff, st);
    if (wp == 1) return build_levels<float2>(g, U, stage, (float2 *)W, noff, st);
    if (wp == 2) return build_levels<__half2>(g, U, stage, (__half2 *)W, noff, st);
    return hipErrorInvalidValue;
}

hipError_t convert_w40(const Geom &g, const double2 *W40, void *W, int wp, int noff, hipStream_t st) {
    dim3 grid((g.V + kBlock - 1) / kBlock, 40);
    if (wp == 0)
        hipLaunchKernelGGL(k_convert<double2>, grid, dim3(kBlock), 0, st, g, W40, (double2 *)W, noff);
    else if (wp == 1)
        hipLaunchKernelGGL(k_convert<float2>, grid, dim3(kBlock), 0, st, g, W40, (float2 *)W, noff);
    else if (wp == 2)
        hipLaunchKernelGGL(k_convert<__half2>, grid, dim3(kBlock), 0, st, g, W40, (__half2 *)W, noff);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace bri
