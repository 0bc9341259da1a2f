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
// k_build_fused builds all 80 transporters of a site in one kernel, each
// once, in FP64, with the lower levels kept on chip; k_convert turns the
// FP64 40-offset store into another store (the SU(3) forms project that
// store first).
#include "apply_recompute.h"
#include "common.h"
#include "kernels.h"

namespace bri {

namespace {

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

// ---------------------------------------------------------------- fused build
// All transporters of a site in one kernel, the way k_apply_recompute builds
// them: 16 consecutive sites x 32 threads per workgroup, every one of the 80
// transporters of a site built once by the hop-order recursion (k! W
// carried, two- and three-hop ones shared through LDS, one support per wave),
// in FP64, and written to the store as soon as it is built (the 40-offset
// store keeps the offsets whose last non-zero component is +1).  No FP64
// stage goes through HBM: the kernel reads the links (through the caches)
// and writes the store.
namespace {
template <typename WT, int NOFF>
__device__ __forceinline__ void store_w(WT *__restrict__ W, size_t V, int site, bool valid, const int (&n)[4],
                                        double inv_fact, const cx<double> s[3][3]) {
    const int i = (n[0] + 1) + 3 * (n[1] + 1) + 9 * (n[2] + 1) + 27 * (n[3] + 1);
    if (!valid || (NOFF == 40 && i < 41)) return;
    const int plane = NOFF == 80 ? (i < 40 ? i : i - 1) : i - 41;
    WT *o = W + (size_t)plane * 9 * V + site;
#pragma unroll
    for (int e = 0; e < 9; ++e) stnt(o + e * V, cscale(inv_fact, s[e / 3][e % 3]));
}

template <int P, typename WT, int NOFF>
__device__ __forceinline__ void build_l2(const double2 *U, WT *W, size_t V, const NbrParts &q, int bits, int sl,
                                         int site, bool valid, cx<double> (*w2)[9][16]) {
    constexpr int MU = pair_lo(P), NU = pair_hi(P);
    int n[4] = {0, 0, 0, 0};
    n[MU] = (bits & 1) ? -1 : 1;
    n[NU] = (bits & 2) ? -1 : 1;
    cx<double> w[3][3], p[3][3], l[3][3];
    zero33(w);
    {
        int m[4] = {0, 0, 0, 0};
        m[NU] = n[NU];
        last_link<NU, double2, double>(U, V, q, m, p);
        last_link<MU, double2, double>(U, V, q, n, l);
        mat_mul_acc(w, p, l);
    }
    {
        int m[4] = {0, 0, 0, 0};
        m[MU] = n[MU];
        last_link<MU, double2, double>(U, V, q, m, p);
        last_link<NU, double2, double>(U, V, q, n, l);
        mat_mul_acc(w, p, l);
    }
    lds_put<double, 16>(w2, 4 * P + bits, sl, w);
    store_w<WT, NOFF>(W, V, site, valid, n, 0.5, w);
}

template <int Q, typename WT, int NOFF>
__device__ __forceinline__ void build_l3(const double2 *U, WT *W, size_t V, const NbrParts &q, int bits, int sl,
                                         int site, bool valid, cx<double> (*w2)[9][16], cx<double> (*w3)[9][16]) {
    constexpr int D0 = Q == 0 ? 1 : 0, D1 = Q <= 1 ? 2 : 1, D2 = Q <= 2 ? 3 : 2;
    int n[4] = {0, 0, 0, 0};
    n[D0] = (bits & 1) ? -1 : 1;
    n[D1] = (bits & 2) ? -1 : 1;
    n[D2] = (bits & 4) ? -1 : 1;
    const int b0 = bits & 1, b1 = (bits >> 1) & 1, b2 = (bits >> 2) & 1;
    cx<double> w[3][3], p[3][3], l[3][3];
    zero33(w);
    lds_get<double, 16>(w2, 4 * pair_index(D1, D2) + b1 + 2 * b2, sl, p);
    last_link<D0, double2, double>(U, V, q, n, l);
    mat_mul_acc(w, p, l);
    lds_get<double, 16>(w2, 4 * pair_index(D0, D2) + b0 + 2 * b2, sl, p);
    last_link<D1, double2, double>(U, V, q, n, l);
    mat_mul_acc(w, p, l);
    lds_get<double, 16>(w2, 4 * pair_index(D0, D1) + b0 + 2 * b1, sl, p);
    last_link<D2, double2, double>(U, V, q, n, l);
    mat_mul_acc(w, p, l);
    lds_put<double, 16>(w3, 8 * Q + bits, sl, w);
    store_w<WT, NOFF>(W, V, site, valid, n, 1.0 / 6.0, w);
}

template <typename WT, int NOFF>
__global__ __launch_bounds__(512) void k_build_fused(Geom g, const double2 *__restrict__ U, WT *__restrict__ W, int gy,
                                                    int gz) {
    // 16 sites x 32 threads: eight waves, each of 16 sites x 4 roles; the
    // FP64 levels in LDS (129 KB) allow one workgroup per CU, i.e. two waves
    // per SIMD
    constexpr int S = 16;
    __shared__ cx<double> w2[24][9][S];
    __shared__ cx<double> w3[32][9][S];
    const int sl = threadIdx.x % S;
    const int role = (threadIdx.x / S) % 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int s0 = strip_base(g, xcd_block(blockIdx.x, gridDim.x), gy, gz) + sl;
    const bool valid = s0 < g.V;
    const int site = valid ? s0 : 0;
    const size_t V = (size_t)g.V;
    int c[4];
    coords(g, site, c);
    const NbrParts q = make_parts(g, c);

    // two hops: waves 0-5, one direction pair each, role = the two signs;
    // links: wave 6 the x and y directions, wave 7 z and t, role bit 0 the sign
    static_for<0, 6>([&](auto P) {
        if (wave == decltype(P)::value) build_l2<decltype(P)::value, WT, NOFF>(U, W, V, q, role, sl, site, valid, w2);
    });
    if (wave >= 6) {
        const int sgn = (role & 1) ? -1 : 1;
        static_for<0, 4>([&](auto M) {
            constexpr int MU = decltype(M)::value;
            if (wave == 6 + MU / 2 && (role >> 1) == MU % 2) {
                int n[4] = {0, 0, 0, 0};
                n[MU] = sgn;
                cx<double> w[3][3];
                last_link<MU, double2, double>(U, V, q, n, w);
                store_w<WT, NOFF>(W, V, site, valid, n, 1.0, w);
            }
        });
    }
    __syncthreads();
    // three hops: support = all directions but Q = wave / 2, signs 4 (wave % 2) + role
    static_for<0, 4>([&](auto Q) {
        if ((wave >> 1) == decltype(Q)::value)
            build_l3<decltype(Q)::value, WT, NOFF>(U, W, V, q, 4 * (wave & 1) + role, sl, site, valid, w2, w3);
    });
    __syncthreads();
    // four hops, signs 4 (wave % 4) + role: waves 0-3 sum the paths whose last
    // step is along x or y, waves 4-7 those along z or t; the first half goes
    // through LDS (the two-hop slots are free by now) to the second, which
    // adds it and stores
    {
        const int h = wave >> 2;
        const int bits = 4 * (wave & 3) + role;
        int n[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) n[mu] = ((bits >> mu) & 1) ? -1 : 1;
        cx<double> w[3][3], p[3][3], l[3][3];
        zero33(w);
        static_for<0, 4>([&](auto M) {
            constexpr int MU = decltype(M)::value;
            if (h == MU / 2) {
                const int low = bits & ((1 << MU) - 1), high = bits >> (MU + 1);
                lds_get<double, 16>(w3, 8 * MU + (low | (high << MU)), sl, p);
                last_link<MU, double2, double>(U, V, q, n, l);
                mat_mul_acc(w, p, l);
            }
        });
        if (h == 0) lds_put<double, 16>(w2, bits, sl, w);
        __syncthreads();
        if (h == 1) {
            lds_get<double, 16>(w2, bits, sl, p);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) w[a][b] = cmake<double>(w[a][b].re + p[a][b].re, w[a][b].im + p[a][b].im);
            store_w<WT, NOFF>(W, V, site, valid, n, 1.0 / 24.0, w);
        }
    }
}

template <typename WT>
hipError_t build_fused_t(const Geom &g, const double2 *U, void *W, int noff, hipStream_t st) {
    // the link planes are addressed with 32-bit byte offsets
    if ((size_t)g.V * sizeof(double2) >= ((size_t)1 << 32)) return hipErrorInvalidValue;
    dim3 grid((g.V + 15) / 16);
    // strip groups of Lx/16 x 4 x 4 (32 workgroups at Lx = 32, what an XCD
    // holds at a time); 32^3 x 64 FP32 W80: 7.43 ms in site order, 7.02 ms
    // with 4 x 4, 7.11-7.18 ms with 8 x 4, 4 x 8 or 8 x 8, 7.75 ms with 2 x 2
    int gy, gz;
    strip_groups(g, gy, gz);
    if (noff == 80)
        hipLaunchKernelGGL((k_build_fused<WT, 80>), grid, dim3(512), 0, st, g, U, (WT *)W, gy, gz);
    else
        hipLaunchKernelGGL((k_build_fused<WT, 40>), grid, dim3(512), 0, st, g, U, (WT *)W, gy, gz);
    return hipGetLastError();
}
}  // namespace

hipError_t build_fused(const Geom &g, const double2 *U, void *W, int wp, int noff, hipStream_t st) {
    if (wp == 0) return build_fused_t<double2>(g, U, W, noff, st);
    if (wp == 1) return build_fused_t<float2>(g, U, W, noff, st);
    if (wp == 2) return build_fused_t<__half2>(g, U, W, noff, st);
    return hipErrorInvalidValue;
}

hipError_t build_w40_f64(const Geom &g, const double2 *U, double2 *W40, hipStream_t st) {
    return build_fused(g, U, W40, 0, 40, st);
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
