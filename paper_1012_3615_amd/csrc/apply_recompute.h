// Apply with the transporters rebuilt from the links inside the kernel.
#pragma once
#include "stencil.h"

namespace bri {
// ---------------------------------------------------------------- recompute W
// W(x, x+n) rebuilt from the links inside the apply (see k_apply_recompute).
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

// Linear-index parts of x + d for one site, per direction and d in
// {-1, 0, +1}, held as named scalars (no array: a run-time index into an
// array would send it to scratch memory).
struct NbrParts {
    int m[4], z[4], p[4];
};
__device__ __forceinline__ NbrParts make_parts(const Geom &g, const int c[4]) {
    NbrParts q;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int L = g.L[mu];
        q.m[mu] = (c[mu] == 0 ? L - 1 : c[mu] - 1) * g.stride[mu];
        q.z[mu] = c[mu] * g.stride[mu];
        q.p[mu] = (c[mu] == L - 1 ? 0 : c[mu] + 1) * g.stride[mu];
    }
    return q;
}
// part of direction MU (compile-time) for a per-lane displacement d
template <int MU>
__device__ __forceinline__ int part_of(const NbrParts &q, int d) {
    return d < 0 ? q.m[MU] : d > 0 ? q.p[MU] : q.z[MU];
}
__device__ __forceinline__ int site_of(const NbrParts &q, const int (&d)[4]) {
    return part_of<0>(q, d[0]) + part_of<1>(q, d[1]) + part_of<2>(q, d[2]) + part_of<3>(q, d[3]);
}

// element e of the SoA plane `plane` at site y: a uniform base pointer and a
// 32-bit byte offset (the launcher checks that every plane is below 4 GiB)
template <typename A, typename T>
__device__ __forceinline__ cx<A> ld_plane(const T *__restrict__ plane, int y) {
    const char *p = reinterpret_cast<const char *>(plane) + (unsigned)y * (unsigned)sizeof(T);
    return ldc<A>(reinterpret_cast<const T *>(p));
}

// the link of the last step into x + n along MU (n_MU != 0):
//   U_MU(x + n - MU) if n_MU = +1,   U_MU(x + n)^dag if n_MU = -1
// (the adjoint taken per lane by selecting transposed elements)
template <int MU, typename LS, typename A>
__device__ __forceinline__ void last_link(const LS *__restrict__ U, size_t V, const NbrParts &q, const int (&n)[4],
                                          cx<A> m[3][3]) {
    int d[4] = {n[0], n[1], n[2], n[3]};
    d[MU] = n[MU] > 0 ? 0 : -1;
    const int y = site_of(q, d);
    const bool dg = n[MU] < 0;
    cx<A> t[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) t[e] = ld_plane<A>(U + ((size_t)MU * 9 + e) * V, y);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cx<A> u = t[3 * a + b], v = t[3 * b + a];
            m[a][b] = a == b ? cmake<A>(u.re, dg ? -u.im : u.im) : cmake<A>(dg ? v.re : u.re, dg ? -v.im : u.im);
        }
}

// acc += C W psi(x+n) for an offset whose support is SUPP (bit mu = direction
// mu): lam, rho are the class coefficients of Tab. rholambda divided by k!
// (the kernel carries k! W), the gamma terms of the support directions with
// the lane's signs (gamma matrices as in spin_accum_rt)
template <int SUPP, typename SS, typename A>
__device__ __forceinline__ void stencil_term(const SS *__restrict__ in, size_t V, const NbrParts &q, const int (&n)[4],
                                             A lam, A rho, const cx<A> w[3][3], cx<A> (&acc)[4][3]) {
    const int y = site_of(q, n);
    cx<A> psi[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b) psi[s][b] = ld_plane<A>(in + (size_t)(3 * s + b) * V, y);
    const A rx = n[0] < 0 ? -rho : rho, ry = n[1] < 0 ? -rho : rho;
    const A rz = n[2] < 0 ? -rho : rho, rt = n[3] < 0 ? -rho : rho;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cx<A> c[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            cx<A> t = cmul(w[a][0], psi[s][0]);
            t = cmac(t, w[a][1], psi[s][1]);
            c[s] = cmac(t, w[a][2], psi[s][2]);
        }
        cx<A> o[4] = {acc[0][a], acc[1][a], acc[2][a], acc[3][a]};
#pragma unroll
        for (int s = 0; s < 4; ++s) o[s] = caxpy(lam, c[s], o[s]);
        if constexpr ((SUPP & 1) != 0) {
            o[0].re = fma(rx, c[3].im, o[0].re); o[0].im = fma(-rx, c[3].re, o[0].im);
            o[1].re = fma(rx, c[2].im, o[1].re); o[1].im = fma(-rx, c[2].re, o[1].im);
            o[2].re = fma(-rx, c[1].im, o[2].re); o[2].im = fma(rx, c[1].re, o[2].im);
            o[3].re = fma(-rx, c[0].im, o[3].re); o[3].im = fma(rx, c[0].re, o[3].im);
        }
        if constexpr ((SUPP & 2) != 0) {
            o[0].re = fma(-ry, c[3].re, o[0].re); o[0].im = fma(-ry, c[3].im, o[0].im);
            o[1].re = fma(ry, c[2].re, o[1].re); o[1].im = fma(ry, c[2].im, o[1].im);
            o[2].re = fma(ry, c[1].re, o[2].re); o[2].im = fma(ry, c[1].im, o[2].im);
            o[3].re = fma(-ry, c[0].re, o[3].re); o[3].im = fma(-ry, c[0].im, o[3].im);
        }
        if constexpr ((SUPP & 4) != 0) {
            o[0].re = fma(rz, c[2].im, o[0].re); o[0].im = fma(-rz, c[2].re, o[0].im);
            o[1].re = fma(-rz, c[3].im, o[1].re); o[1].im = fma(rz, c[3].re, o[1].im);
            o[2].re = fma(-rz, c[0].im, o[2].re); o[2].im = fma(rz, c[0].re, o[2].im);
            o[3].re = fma(rz, c[1].im, o[3].re); o[3].im = fma(-rz, c[1].re, o[3].im);
        }
        if constexpr ((SUPP & 8) != 0) {
            o[0] = caxpy(rt, c[2], o[0]);
            o[1] = caxpy(rt, c[3], o[1]);
            o[2] = caxpy(rt, c[0], o[2]);
            o[3] = caxpy(rt, c[1], o[3]);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s][a] = o[s];
    }
}

// LDS slots: the 24 two-hop offsets at 4 p + sign bits (p enumerating the
// pairs (0,1) (0,2) (0,3) (1,2) (1,3) (2,3); bit 0 set when the lower
// direction is negative, bit 1 for the higher); the 32 three-hop offsets at
// 8 q + sign bits (q the direction outside the support; bit j for the j-th
// support direction in increasing order).
__host__ __device__ constexpr int pair_index(int mu, int nu) { return mu == 0 ? nu - 1 : mu == 1 ? nu + 1 : 5; }
__host__ __device__ constexpr int pair_lo(int p) { return p < 3 ? 0 : p < 5 ? 1 : 2; }
__host__ __device__ constexpr int pair_hi(int p) { return p < 3 ? p + 1 : p < 5 ? p - 1 : 3; }

// W[slot][e][site] <-> a 3x3 matrix of one site (LDS)
template <typename A, int S>
__device__ __forceinline__ void lds_put(cx<A> (*buf)[9][S], int slot, int sl, const cx<A> m[3][3]) {
#pragma unroll
    for (int e = 0; e < 9; ++e) buf[slot][e][sl] = m[e / 3][e % 3];
}
template <typename A, int S>
__device__ __forceinline__ void lds_get(cx<A> (*buf)[9][S], int slot, int sl, cx<A> m[3][3]) {
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e / 3][e % 3] = buf[slot][e][sl];
}

template <typename A>
__device__ __forceinline__ void zero33(cx<A> m[3][3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) m[a][b] = cmake<A>(0, 0);
}

// coefficients of Tab. rholambda for k hops, divided by k! (k! W is carried)
__host__ __device__ constexpr double fact(int k) { return k <= 1 ? 1.0 : k * fact(k - 1); }

// Each task builds one transporter (k! times it) of a compile-time support
// with the lane's signs, applies it and, for two and three hops, leaves it in
// LDS for the next level.
template <int MU, typename LS, typename SS, typename A, bool DAG>
__device__ __forceinline__ void task_l1(const LS *U, const SS *in, size_t V, const NbrParts &nb, int sgn,
                                        cx<A> (&acc)[4][3]) {
    int n[4] = {0, 0, 0, 0};
    n[MU] = sgn;
    cx<A> w[3][3];
    last_link<MU, LS, A>(U, V, nb, n, w);
    stencil_term<1 << MU, SS, A>(in, V, nb, n, (A)lam_k(1), DAG ? -(A)rho_k(1) : (A)rho_k(1), w, acc);
}

template <int P, typename LS, typename SS, typename A, bool DAG, int S>
__device__ __forceinline__ void task_l2(const LS *U, const SS *in, size_t V, const NbrParts &nb, int bits, int sl,
                                        cx<A> (*w2)[9][S], cx<A> (&acc)[4][3]) {
    constexpr int MU = pair_lo(P), NU = pair_hi(P);
    int n[4] = {0, 0, 0, 0};
    n[MU] = (bits & 1) ? -1 : 1;
    n[NU] = (bits & 2) ? -1 : 1;
    cx<A> w[3][3], p[3][3], l[3][3];
    zero33(w);
    {  // last step along MU: predecessor n_NU NU, a link
        int m[4] = {0, 0, 0, 0};
        m[NU] = n[NU];
        last_link<NU, LS, A>(U, V, nb, m, p);
        last_link<MU, LS, A>(U, V, nb, n, l);
        mat_mul_acc(w, p, l);
    }
    {  // last step along NU
        int m[4] = {0, 0, 0, 0};
        m[MU] = n[MU];
        last_link<MU, LS, A>(U, V, nb, m, p);
        last_link<NU, LS, A>(U, V, nb, n, l);
        mat_mul_acc(w, p, l);
    }
    lds_put<A, S>(w2, 4 * P + bits, sl, w);
    constexpr double f = 2.0;
    stencil_term<(1 << MU) | (1 << NU), SS, A>(in, V, nb, n, (A)(lam_k(2) / f),
                                               (A)(DAG ? -rho_k(2) / f : rho_k(2) / f), w, acc);
}

template <int Q, typename LS, typename SS, typename A, bool DAG, int S>
__device__ __forceinline__ void task_l3(const LS *U, const SS *in, size_t V, const NbrParts &nb, int bits, int sl,
                                        cx<A> (*w2)[9][S], cx<A> (*w3)[9][S], cx<A> (&acc)[4][3]) {
    // support directions D0 < D1 < D2 (all but Q)
    constexpr int D0 = Q == 0 ? 1 : 0, D1 = Q <= 1 ? 2 : 1, D2 = Q <= 2 ? 3 : 2;
    int n[4] = {0, 0, 0, 0};
    n[D0] = (bits & 1) ? -1 : 1;
    n[D1] = (bits & 2) ? -1 : 1;
    n[D2] = (bits & 4) ? -1 : 1;
    const int b0 = bits & 1, b1 = (bits >> 1) & 1, b2 = (bits >> 2) & 1;
    cx<A> w[3][3], p[3][3], l[3][3];
    zero33(w);
    // last step along D0: predecessor on the pair (D1, D2)
    lds_get<A, S>(w2, 4 * pair_index(D1, D2) + b1 + 2 * b2, sl, p);
    last_link<D0, LS, A>(U, V, nb, n, l);
    mat_mul_acc(w, p, l);
    lds_get<A, S>(w2, 4 * pair_index(D0, D2) + b0 + 2 * b2, sl, p);
    last_link<D1, LS, A>(U, V, nb, n, l);
    mat_mul_acc(w, p, l);
    lds_get<A, S>(w2, 4 * pair_index(D0, D1) + b0 + 2 * b1, sl, p);
    last_link<D2, LS, A>(U, V, nb, n, l);
    mat_mul_acc(w, p, l);
    lds_put<A, S>(w3, 8 * Q + bits, sl, w);
    constexpr double f = 6.0;
    stencil_term<15 & ~(1 << Q), SS, A>(in, V, nb, n, (A)(lam_k(3) / f), (A)(DAG ? -rho_k(3) / f : rho_k(3) / f),
                                        w, acc);
}

template <typename LS, typename SS, typename A, bool DAG, int S>
__device__ __forceinline__ void task_l4(const LS *U, const SS *in, size_t V, const NbrParts &nb, int bits, int sl,
                                        cx<A> (*w3)[9][S], cx<A> (&acc)[4][3]) {
    int n[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) n[mu] = ((bits >> mu) & 1) ? -1 : 1;
    cx<A> w[3][3], p[3][3], l[3][3];
    zero33(w);
    // last step along MU: predecessor has support all but MU; its sign bits
    // are those of the other three directions in increasing order
    static_for<0, 4>([&](auto M) {
        constexpr int MU = decltype(M)::value;
        const int low = bits & ((1 << MU) - 1), high = bits >> (MU + 1);
        lds_get<A, S>(w3, 8 * MU + (low | (high << MU)), sl, p);
        last_link<MU, LS, A>(U, V, nb, n, l);
        mat_mul_acc(w, p, l);
    });
    constexpr double f = 24.0;
    stencil_term<15, SS, A>(in, V, nb, n, (A)(lam_k(4) / f), (A)(DAG ? -rho_k(4) / f : rho_k(4) / f), w, acc);
}

// First site of the 16-site x strip that a workgroup takes.  With gy > 0
// (Lx a multiple of 16, gy | Ly, gz | Lz) the strips are ordered in groups of
// Lx/16 x gy x gz strips at one t, a group walking t before the next group
// (y blocks fastest): the workgroups an XCD runs at a time then cover a
// compact (x, y, z) block, and its next t step re-reads the links of this one
// from L2.  With gy = 0 the strips follow the site order.
__device__ __forceinline__ int strip_base(const Geom &g, int blk, int gy, int gz) {
    if (gy == 0) return blk * 16;
    const int nxs = g.L[0] / 16;
    int r = blk;
    const int xs = r % nxs;
    r /= nxs;
    const int yy = r % gy;
    r /= gy;
    const int zz = r % gz;
    r /= gz;
    const int t = r % g.L[3];
    r /= g.L[3];
    const int nyb = g.L[1] / gy;
    const int y = (r % nyb) * gy + yy, z = (r / nyb) * gz + zz;
    return 16 * xs + y * g.stride[1] + z * g.stride[2] + t * g.stride[3];
}

// the strip groups used with strip_base: Lx/16 x 4 x 4 where the extents allow
inline void strip_groups(const Geom &g, int &gy, int &gz) {
    gy = gz = 0;
    if (g.L[0] % 16 != 0) return;
    gy = g.L[1] % 4 == 0 ? 4 : g.L[1] % 2 == 0 ? 2 : 1;
    gz = g.L[2] % 4 == 0 ? 4 : g.L[2] % 2 == 0 ? 2 : 1;
}

// One workgroup = 16 consecutive sites x TPS threads per site (TPS = 16 for
// FP32, 32 for FP64), TPS / 4 waves of 16 sites x 4 "roles".  The 80
// transporters of each site are built exactly once, by the hop-order
// recursion of the path average (Sec. 5.1),
//   W(n) = (1/k) sum_{mu in supp n} W(n - n_mu mu) L(n, mu),
// carried as k! W (no scaling; the stencil coefficients take the 1/k!),
// level by level; the two- and three-hop ones stay in LDS, where the next
// level reads them as predecessors: 208 3x3 products per site (48 + 96 + 64),
// none repeated.  Each wave takes offsets of one support at a time, its four
// roles the sign combinations, so directions are compile-time and only the
// signs vary across lanes.  With 16 threads per site:
//   two hops: wave w the pair w, then waves 0, 1 the pairs 4, 5 and wave 2
//   the links +-x, +-y, wave 3 +-z, +-t;
//   three hops: wave w the offsets without direction w (signs 0-3, then 4-7);
//   four hops: wave w the offsets with sign bits 4 w + role.
// With 32 threads per site (FP64: the levels take 129 KB of LDS, one
// workgroup per CU, so the eight waves give two per SIMD instead of one):
//   two hops: wave w < 6 the pair w; wave 6 the links +-x, +-y, wave 7 +-z, +-t;
//   three hops: wave w the offsets without direction w / 2, signs 4 (w % 2) + role;
//   four hops: signs 4 (w % 4) + role; waves 0-3 sum the paths whose last
//   step is along x or y, waves 4-7 those along z or t, and the first half
//   reaches the second through LDS.
// The x strips run in groups (strip_base).  Each transporter is applied to
// psi(x+n) as soon as it is complete; the TPS partial sums of a site are
// added in a fixed order through LDS, then the diagonal term.
// 32^3 x 64: FP32 4.53 ms in site order, 4.34 ms with 4 x 4 strip groups
// (4.82 ms with 32 threads per site); FP64 7.96 ms (16 threads per site,
// site order) -> 7.01 ms.
template <typename A>
constexpr int recompute_tps() { return sizeof(A) == 8 ? 32 : 16; }

template <typename LS, typename SS, typename A, bool DAG>
__global__ __launch_bounds__(16 * recompute_tps<A>())
void k_apply_recompute(Geom g, const LS *__restrict__ U, const SS *__restrict__ in, SS *__restrict__ out, A diag,
                       int gy, int gz) {
    constexpr int S = 16;
    constexpr int TPS = recompute_tps<A>();
    __shared__ cx<A> lds[56][9][S];
    cx<A>(*w2)[9][S] = lds;       // 24 two-hop slots
    cx<A>(*w3)[9][S] = lds + 24;  // 32 three-hop slots
    static_assert(sizeof(lds) >= sizeof(A) * 2 * TPS * 12 * S, "the reduction reuses the level buffers");
    const int sl = threadIdx.x % S;
    const int role = (threadIdx.x / S) % 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    const int base = strip_base(g, xcd_block(blockIdx.x, gridDim.x), gy, gz);
    const int s0 = base + sl;
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
    int c[4];
    coords(g, site, c);
    const NbrParts nb = make_parts(g, c);
    const int sgn = (role & 1) ? -1 : 1;  // sign of a link task

    if constexpr (TPS == 32) {
        // two hops and the links
        static_for<0, 6>([&](auto P) {
            if (wave == decltype(P)::value)
                task_l2<decltype(P)::value, LS, SS, A, DAG, S>(U, in, V, nb, role, sl, w2, acc);
        });
        static_for<0, 4>([&](auto M) {
            constexpr int MU = decltype(M)::value;
            if (wave == 6 + MU / 2 && (role >> 1) == MU % 2) task_l1<MU, LS, SS, A, DAG>(U, in, V, nb, sgn, acc);
        });
        __syncthreads();
        // three hops
        static_for<0, 4>([&](auto Q) {
            if ((wave >> 1) == decltype(Q)::value)
                task_l3<decltype(Q)::value, LS, SS, A, DAG, S>(U, in, V, nb, 4 * (wave & 1) + role, sl, w2, w3, acc);
        });
        __syncthreads();
        // four hops: the half sums of the paths by the direction of their last
        // step, the first half through the (now free) two-hop slots
        const int h = wave >> 2;
        const int bits = 4 * (wave & 3) + role;
        int n[4];
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) n[mu] = ((bits >> mu) & 1) ? -1 : 1;
        cx<A> w[3][3], p[3][3], l[3][3];
        zero33(w);
        static_for<0, 4>([&](auto M) {
            constexpr int MU = decltype(M)::value;
            if (h == MU / 2) {
                // predecessor: support all but MU, sign bits of the other three
                // directions in increasing order
                const int low = bits & ((1 << MU) - 1), high = bits >> (MU + 1);
                lds_get<A, S>(w3, 8 * MU + (low | (high << MU)), sl, p);
                last_link<MU, LS, A>(U, V, nb, n, l);
                mat_mul_acc(w, p, l);
            }
        });
        if (h == 0) lds_put<A, S>(w2, bits, sl, w);
        __syncthreads();
        if (h == 1) {
            lds_get<A, S>(w2, bits, sl, p);
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) w[a][b] = cadd(w[a][b], p[a][b]);
            constexpr double f = 24.0;
            stencil_term<15, SS, A>(in, V, nb, n, (A)(lam_k(4) / f), (A)(DAG ? -rho_k(4) / f : rho_k(4) / f), w,
                                    acc);
        }
    } else {
        // two hops and the links
        static_for<0, 4>([&](auto P) {
            if (wave == decltype(P)::value)
                task_l2<decltype(P)::value, LS, SS, A, DAG, S>(U, in, V, nb, role, sl, w2, acc);
        });
        if (wave == 0) task_l2<4, LS, SS, A, DAG, S>(U, in, V, nb, role, sl, w2, acc);
        if (wave == 1) task_l2<5, LS, SS, A, DAG, S>(U, in, V, nb, role, sl, w2, acc);
        static_for<0, 4>([&](auto M) {
            constexpr int MU = decltype(M)::value;
            if (wave == 2 + MU / 2 && (role >> 1) == MU % 2) task_l1<MU, LS, SS, A, DAG>(U, in, V, nb, sgn, acc);
        });
        __syncthreads();
        // three hops
#pragma unroll 1
        for (int half = 0; half < 2; ++half) {
            const int bits = 4 * half + role;
            static_for<0, 4>([&](auto Q) {
                if (wave == decltype(Q)::value)
                    task_l3<decltype(Q)::value, LS, SS, A, DAG, S>(U, in, V, nb, bits, sl, w2, w3, acc);
            });
        }
        __syncthreads();
        // four hops
        task_l4<LS, SS, A, DAG, S>(U, in, V, nb, 4 * wave + role, sl, w3, acc);
    }
    __syncthreads();

    // the TPS partial sums of each site in a fixed order (level buffers reused)
    A(*red)[12][S][2] = reinterpret_cast<A(*)[12][S][2]>(&lds[0][0][0]);
    const int slot = 4 * wave + role;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            red[slot][3 * s + a][sl][0] = acc[s][a].re;
            red[slot][3 * s + a][sl][1] = acc[s][a].im;
        }
    __syncthreads();
    if (threadIdx.x < 12 * S) {
        const int ss = threadIdx.x % S, comp = threadIdx.x / S;
        const int st_site = base + ss;
        if (st_site < g.V) {
            cx<A> sum = cmake<A>(red[0][comp][ss][0], red[0][comp][ss][1]);
#pragma unroll
            for (int o = 1; o < TPS; ++o) sum = cadd(sum, cmake<A>(red[o][comp][ss][0], red[o][comp][ss][1]));
            stnt(out + comp * V + st_site, caxpy(diag, ld_plane<A>(in + (size_t)comp * V, st_site), sum));
        }
    }
}

}  // namespace bri
