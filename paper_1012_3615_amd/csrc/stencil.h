// Device helpers of the Brillouin stencil (Eq. def_pref, c_SW = 0):
//   (D psi)(x) = (lambda_0 + m) psi(x)
//              + sum_{n != 0} [lambda_k + rho_k sum_mu n_mu gamma_mu] W(x,x+n) psi(x+n)
// The loops over the offsets run at run time; an offset is the same for every
// lane of a wavefront, so the tests on its components are uniform (scalar)
// branches and the spin structure costs exactly the non-zero gamma terms.
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

// Coefficients of a member of the generic ultralocal class (Sec. 8): the
// offset classes k = 1..4 carry lambda_k and rho_k (index 0 unused; lambda_0
// enters through the diagonal).  Passed by value as a kernel argument, so the
// values sit in scalar registers.
template <typename T>
struct Coef {
    T lam[5], rho[5];
};
// lambda_k, rho_k (k = 1..4) from a host table (lambda_0..4, rho_1..4), or
// the Brillouin column of Tab. rholambda for nullptr
template <typename T>
inline Coef<T> make_coef(const double *table) {
    Coef<T> c{};
    for (int k = 1; k <= 4; ++k) {
        c.lam[k] = (T)(table ? table[k] : lam_k(k));
        c.rho[k] = (T)(table ? table[4 + k] : rho_k(k));
    }
    return c;
}

// select by a wavefront-uniform k in 1..4 without indexing the argument array
template <typename T>
__device__ __forceinline__ T coef_pick(const T (&a)[5], int k) {
    return k == 1 ? a[1] : k == 2 ? a[2] : k == 3 ? a[3] : a[4];
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


// FP16 colour products with FP32 accumulation (v_dot2_f32_f16), for FP16
// transporters and spinors: both operands are exact in FP32 products, so the
// result equals the converted FP32 arithmetic up to the order of the
// additions.  A transporter entry w = (re, im) (one 32-bit word, re in the
// low half) enters as the two words (re, -im) and (im, re); a spinor entry
// stays as stored.
typedef _Float16 h2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
    return __builtin_amdgcn_fdot2(__builtin_bit_cast(h2v, a), __builtin_bit_cast(h2v, b), c, false);
}
__device__ __forceinline__ void h2_pair(uint32_t w, uint32_t &wp, uint32_t &wq) {
    wp = w ^ 0x80000000u;                          // (re, -im)
    wq = __builtin_amdgcn_alignbit(w, w, 16);     // (im, re)
}
// chi[s] = w[a][.] psi[s][.] for colour row a, all spins, and accumulate
__device__ __forceinline__ void colour_spin_accum_h2(cx<float> acc[4][3], const uint32_t w[3][3],
                                                     const uint32_t psi[4][3], float lam, float rho, int nx,
                                                     int ny, int nz, int nt) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        uint32_t wp[3], wq[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) h2_pair(w[a][b], wp[b], wq[b]);
        cx<float> chi[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            chi[s].re = dot2(wp[2], psi[s][2], dot2(wp[1], psi[s][1], dot2(wp[0], psi[s][0], 0.0f)));
            chi[s].im = dot2(wq[2], psi[s][2], dot2(wq[1], psi[s][1], dot2(wq[0], psi[s][0], 0.0f)));
        }
        cx<float> o[4] = {acc[0][a], acc[1][a], acc[2][a], acc[3][a]};
        spin_accum_rt(o, chi, lam, rho, nx, ny, nz, nt);
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[s][a] = o[s];
    }
}

// ------------------------------------------------------------------ clover term
// Per site two Hermitian 6x6 blocks (spins 0,1 and spins 2,3; local index
// 3*s + colour), stored as [2][18][V] complex: planes 0..2 hold the real
// diagonal in pairs (M_00, M_11), (M_22, M_33), (M_44, M_55), planes 3..17 the
// entries M_ij, i < j, row by row.
__host__ __device__ constexpr int clover_plane(int i, int j) {
    // number of strictly-upper entries in rows 0..i-1 of a 6x6 matrix, plus column offset
    return 3 + (i * (11 - i)) / 2 + (j - i - 1);
}

template <typename A, typename CS>
__device__ __forceinline__ void clover_load_block(const CS *C, size_t V, int site, int b, cx<A> (&cl)[18]) {
#pragma unroll
    for (int p = 0; p < 18; ++p) cl[p] = ldnt<A>(C + (size_t)(b * 18 + p) * V + site);
}

// acc[s][a] += (M_b x)_(3s+a - 6b) for block b, x its six spin-colour components
template <typename A>
__device__ __forceinline__ void clover_accum_block(const cx<A> (&cl)[18], const cx<A> (&x)[6], int b,
                                                   cx<A> (&acc)[4][3]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        const int c = 6 * b + i;
        cx<A> y = acc[c / 3][c % 3];
        const A d = (i % 2 == 0) ? cl[i / 2].re : cl[i / 2].im;
        y = caxpy(d, x[i], y);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            if (j > i) y = cmac(y, cl[clover_plane(i, j)], x[j]);
            if (j < i) y = cmacc(y, cl[clover_plane(j, i)], x[j]);
        }
        acc[c / 3][c % 3] = y;
    }
}

}  // namespace bri
