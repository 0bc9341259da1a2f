// Device-side building blocks shared by the HIP kernels of the Brillouin
// operator library: complex arithmetic, storage <-> compute conversion,
// lattice geometry, the offset numbering and the stencil coefficients.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstddef>
#include <cstdint>
#include <utility>

namespace bri {

// ------------------------------------------------------------------ complex
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmake(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
// a*b (explicit fused multiply-adds: the library is built with
// -ffp-contract=off so every kernel configuration rounds identically)
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
// acc + a*b
template <typename T>
__device__ __forceinline__ cx<T> cmac(cx<T> acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
    return acc;
}
// acc + conj(a)*b
template <typename T>
__device__ __forceinline__ cx<T> cmacc(cx<T> acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
    return acc;
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(T s, cx<T> a) { return {s * a.re, s * a.im}; }
// acc + s*a (s real)
template <typename T>
__device__ __forceinline__ cx<T> caxpy(T s, cx<T> a, cx<T> acc) {
    return {fma(s, a.re, acc.re), fma(s, a.im, acc.im)};
}

// ------------------------------------------------------------------ storage
// Storage element types: double2 (F64), float2 (F32), __half2 (F16).
template <typename S> struct storage_traits;
template <> struct storage_traits<double2> { using real = double; };
template <> struct storage_traits<float2> { using real = float; };
template <> struct storage_traits<__half2> { using real = float; };

template <typename A>
__device__ __forceinline__ cx<A> ld(const double2 *p) {
    double2 v = *p;
    return {(A)v.x, (A)v.y};
}
template <typename A>
__device__ __forceinline__ cx<A> ld(const float2 *p) {
    float2 v = *p;
    return {(A)v.x, (A)v.y};
}
template <typename A>
__device__ __forceinline__ cx<A> ld(const __half2 *p) {
    float2 v = __half22float2(*p);
    return {(A)v.x, (A)v.y};
}
// streaming loads (data read exactly once per launch: the 80-offset store)
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename A>
__device__ __forceinline__ cx<A> ldnt(const double2 *p) {
    f64x2 v = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p));
    return {(A)v.x, (A)v.y};
}
template <typename A>
__device__ __forceinline__ cx<A> ldnt(const float2 *p) {
    f32x2 v = __builtin_nontemporal_load(reinterpret_cast<const f32x2 *>(p));
    return {(A)v.x, (A)v.y};
}
template <typename A>
__device__ __forceinline__ cx<A> ldnt(const __half2 *p) {
    unsigned int u = __builtin_nontemporal_load(reinterpret_cast<const unsigned int *>(p));
    __half2 h = *reinterpret_cast<__half2 *>(&u);
    float2 v = __half22float2(h);
    return {(A)v.x, (A)v.y};
}
// cached (reused) loads: spinor neighbours
template <typename A>
__device__ __forceinline__ cx<A> ldc(const double2 *p) {
    double2 v = *p;
    return {(A)v.x, (A)v.y};
}
template <typename A>
__device__ __forceinline__ cx<A> ldc(const float2 *p) { return ld<A>(p); }
template <typename A>
__device__ __forceinline__ cx<A> ldc(const __half2 *p) { return ld<A>(p); }

template <typename A>
__device__ __forceinline__ void st(double2 *p, cx<A> v) { *p = make_double2((double)v.re, (double)v.im); }
template <typename A>
__device__ __forceinline__ void st(float2 *p, cx<A> v) { *p = make_float2((float)v.re, (float)v.im); }
template <typename A>
__device__ __forceinline__ void st(__half2 *p, cx<A> v) {
    *p = __floats2half2_rn((float)v.re, (float)v.im);
}
// streaming stores (data written once per launch and not read again by it:
// operator outputs), so the output stream does not take L2 capacity from
// the spinor halos the tile kernels re-read
template <typename A>
__device__ __forceinline__ void stnt(double2 *p, cx<A> v) {
    const f64x2 t = {(double)v.re, (double)v.im};
    __builtin_nontemporal_store(t, reinterpret_cast<f64x2 *>(p));
}
template <typename A>
__device__ __forceinline__ void stnt(float2 *p, cx<A> v) {
    const f32x2 t = {(float)v.re, (float)v.im};
    __builtin_nontemporal_store(t, reinterpret_cast<f32x2 *>(p));
}
template <typename A>
__device__ __forceinline__ void stnt(__half2 *p, cx<A> v) {
    __half2 h = __floats2half2_rn((float)v.re, (float)v.im);
    __builtin_nontemporal_store(*reinterpret_cast<unsigned int *>(&h), reinterpret_cast<unsigned int *>(p));
}

// ------------------------------------------------------------------ geometry
struct Geom {
    int L[4];        // Lx, Ly, Lz, Lt
    int stride[4];   // 1, Lx, Lx*Ly, Lx*Ly*Lz
    int V;
};

__host__ __device__ inline Geom make_geom(const int32_t L[4]) {
    Geom g;
    int s = 1;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = L[mu];
        g.stride[mu] = s;
        s *= L[mu];
    }
    g.V = s;
    return g;
}

// coordinates of a site
__device__ __forceinline__ void coords(const Geom &g, int site, int c[4]) {
    c[0] = site % g.L[0];
    int r = site / g.L[0];
    c[1] = r % g.L[1];
    r /= g.L[1];
    c[2] = r % g.L[2];
    c[3] = r / g.L[2];
}

// For one site: the linear-index contribution of coordinate c_mu + d for d in
// {-1, 0, +1} (periodic), per direction.  nb(n) = sum_mu part[mu][n_mu + 1].
struct Nbr {
    int part[4][3];
    __device__ __forceinline__ int at(int nx, int ny, int nz, int nt) const {
        return part[0][nx + 1] + part[1][ny + 1] + part[2][nz + 1] + part[3][nt + 1];
    }
};

__device__ __forceinline__ Nbr make_nbr(const Geom &g, const int c[4]) {
    Nbr n;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int L = g.L[mu];
        const int cm = c[mu] == 0 ? L - 1 : c[mu] - 1;
        const int cp = c[mu] == L - 1 ? 0 : c[mu] + 1;
        n.part[mu][0] = cm * g.stride[mu];
        n.part[mu][1] = c[mu] * g.stride[mu];
        n.part[mu][2] = cp * g.stride[mu];
    }
    return n;
}

// ------------------------------------------------------------------ offsets
// Offset i in 0..80 <-> n = (i%3-1, (i/3)%3-1, (i/9)%3-1, i/27-1); i = 40 is 0.
__host__ __device__ constexpr int off_n(int i, int mu) {
    return mu == 0 ? i % 3 - 1 : mu == 1 ? (i / 3) % 3 - 1 : mu == 2 ? (i / 9) % 3 - 1 : i / 27 - 1;
}
__host__ __device__ constexpr int off_k(int i) {
    return (off_n(i, 0) != 0) + (off_n(i, 1) != 0) + (off_n(i, 2) != 0) + (off_n(i, 3) != 0);
}
__host__ __device__ constexpr int off_index(int nx, int ny, int nz, int nt) {
    return (nx + 1) + 3 * (ny + 1) + 9 * (nz + 1) + 27 * (nt + 1);
}
// plane of offset i in the 80-offset store
__host__ __device__ constexpr int plane80(int i) { return i < 40 ? i : i - 1; }
// offsets stored in the 40-offset (hermitian) store: i in 41..80
__host__ __device__ constexpr bool is_canonical(int i) { return i > 40; }
__host__ __device__ constexpr int plane40(int i) { return i - 41; }

// ------------------------------------------------------------------ coefficients
// lambda_k and rho_k of Tab. rholambda (Brillouin column); lambda_0 = 240/128.
__host__ __device__ constexpr double lam_k(int k) {
    return k == 0 ? 240.0 / 128.0 : k == 1 ? -8.0 / 128.0 : k == 2 ? -4.0 / 128.0 : k == 3 ? -2.0 / 128.0 : -1.0 / 128.0;
}
__host__ __device__ constexpr double rho_k(int k) {
    return k == 1 ? 64.0 / 432.0 : k == 2 ? 16.0 / 432.0 : k == 3 ? 4.0 / 432.0 : k == 4 ? 1.0 / 432.0 : 0.0;
}

// out += lam * chi + rho * (sum_mu n_mu gamma_mu) chi for one colour, where
// chi[s] holds the four spin components.  In the chiral basis
//   sum_mu n_mu gamma_mu = [[0, A], [A^dag, 0]],
//   A = [[nt - i nz, -ny - i nx], [ny - i nx, nt + i nz]].
// (NX..NT, LAM, RHO are compile-time so the products fold to adds.)
template <int NX, int NY, int NZ, int NT, typename T>
__device__ __forceinline__ void spin_accum(cx<T> out[4], const cx<T> chi[4], T lam, T rho) {
    // (a + i b) * z  with integer a, b
    auto mulc = [](int a, int b, cx<T> z) -> cx<T> {
        return {(T)a * z.re - (T)b * z.im, (T)a * z.im + (T)b * z.re};
    };
    cx<T> g0 = cadd(mulc(NT, -NZ, chi[2]), mulc(-NY, -NX, chi[3]));
    cx<T> g1 = cadd(mulc(NY, -NX, chi[2]), mulc(NT, NZ, chi[3]));
    cx<T> g2 = cadd(mulc(NT, NZ, chi[0]), mulc(NY, NX, chi[1]));
    cx<T> g3 = cadd(mulc(-NY, NX, chi[0]), mulc(NT, -NZ, chi[1]));
    out[0] = caxpy(rho, g0, caxpy(lam, chi[0], out[0]));
    out[1] = caxpy(rho, g1, caxpy(lam, chi[1], out[1]));
    out[2] = caxpy(rho, g2, caxpy(lam, chi[2], out[2]));
    out[3] = caxpy(rho, g3, caxpy(lam, chi[3], out[3]));
}

// ------------------------------------------------------------------ compile-time loop
template <int I>
struct ic {
    static constexpr int value = I;
};
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(ic<B>{});
        static_for<B + 1, E>(std::forward<F>(f));
    }
}

// XCD-aware block remap: consecutive hardware block ids go round-robin over
// the 8 XCDs; remap so that each XCD works on one contiguous range of tiles
// (neighbour reads then stay inside that XCD's L2).
__device__ __forceinline__ int xcd_block(int b, int nblk) {
    constexpr int NX = 8;
    const int xcd = b % NX, local = b / NX;
    const int q = nblk / NX, r = nblk % NX;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

}  // namespace bri
