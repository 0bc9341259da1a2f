// FP64 3x3 complex matrix helpers and the projection to SU(3) of Sec. 5.2
// (the SU(3) matrix closest to A in the Frobenius norm).
#pragma once
#include "common.h"

namespace bri {

using cd = cx<double>;

struct M3 {
    cd m[3][3];
};

__device__ __forceinline__ M3 mzero() {
    M3 r;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) r.m[a][b] = cmake(0.0, 0.0);
    return r;
}
__device__ __forceinline__ M3 meye() {
    M3 r = mzero();
    r.m[0][0] = r.m[1][1] = r.m[2][2] = cmake(1.0, 0.0);
    return r;
}
// a b
__device__ __forceinline__ M3 mmul(const M3 &a, const M3 &b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd t = cmul(a.m[i][0], b.m[0][j]);
            t = cmac(t, a.m[i][1], b.m[1][j]);
            r.m[i][j] = cmac(t, a.m[i][2], b.m[2][j]);
        }
    return r;
}
// a^dag b
__device__ __forceinline__ M3 mdmul(const M3 &a, const M3 &b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd t = cmake(0.0, 0.0);
            t = cmacc(t, a.m[0][i], b.m[0][j]);
            t = cmacc(t, a.m[1][i], b.m[1][j]);
            r.m[i][j] = cmacc(t, a.m[2][i], b.m[2][j]);
        }
    return r;
}
// a b^dag
__device__ __forceinline__ M3 mmuld(const M3 &a, const M3 &b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cd t = cmake(0.0, 0.0);
            t = cmacc(t, b.m[j][0], a.m[i][0]);
            t = cmacc(t, b.m[j][1], a.m[i][1]);
            r.m[i][j] = cmacc(t, b.m[j][2], a.m[i][2]);
        }
    return r;
}
__device__ __forceinline__ M3 mdag(const M3 &a) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.m[i][j] = cconj(a.m[j][i]);
    return r;
}
__device__ __forceinline__ M3 madd(const M3 &a, const M3 &b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) r.m[i][j] = cadd(a.m[i][j], b.m[i][j]);
    return r;
}
__device__ __forceinline__ cd mdet(const M3 &a) {
    const cd c0 = csub(cmul(a.m[1][1], a.m[2][2]), cmul(a.m[1][2], a.m[2][1]));
    const cd c1 = csub(cmul(a.m[1][0], a.m[2][2]), cmul(a.m[1][2], a.m[2][0]));
    const cd c2 = csub(cmul(a.m[1][0], a.m[2][1]), cmul(a.m[1][1], a.m[2][0]));
    return cadd(csub(cmul(a.m[0][0], c0), cmul(a.m[0][1], c1)), cmul(a.m[0][2], c2));
}

// SoA planes [9][stride] of double2 <-> M3
__device__ __forceinline__ M3 mload(const double2 *p, size_t stride) {
    M3 r;
#pragma unroll
    for (int e = 0; e < 9; ++e) r.m[e / 3][e % 3] = ldc<double>(p + e * stride);
    return r;
}
__device__ __forceinline__ void mstore(double2 *p, size_t stride, const M3 &a) {
#pragma unroll
    for (int e = 0; e < 9; ++e) st(p + e * stride, a.m[e / 3][e % 3]);
}

// Eigen-decomposition of a Hermitian 3x3 matrix by cyclic Jacobi rotations:
// on return h is diagonal (the eigenvalues) and the columns of v are the
// eigenvectors, h_in = v diag v^dag.  A rotation in the (p, q) plane first
// removes the phase of h[p][q] (columns q times e^{-i beta}) and then applies
// the real symmetric Jacobi rotation that zeroes the element.
__device__ inline void jacobi_herm3(M3 &h, M3 &v) {
    v = meye();
    for (int sweep = 0; sweep < 16; ++sweep) {
        const double off = h.m[0][1].re * h.m[0][1].re + h.m[0][1].im * h.m[0][1].im +
                           h.m[0][2].re * h.m[0][2].re + h.m[0][2].im * h.m[0][2].im +
                           h.m[1][2].re * h.m[1][2].re + h.m[1][2].im * h.m[1][2].im;
        const double dia = fabs(h.m[0][0].re) + fabs(h.m[1][1].re) + fabs(h.m[2][2].re);
        if (off <= 1e-36 * dia * dia) break;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int p = k == 2 ? 1 : 0, q = k == 0 ? 1 : 2;
            const cd hpq = h.m[p][q];
            const double r = sqrt(hpq.re * hpq.re + hpq.im * hpq.im);
            if (r == 0.0) continue;
            const cd ph = cmake(hpq.re / r, -hpq.im / r);  // e^{-i beta}
            const double tau = (h.m[q][q].re - h.m[p][p].re) / (2.0 * r);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            M3 g = meye();
            g.m[p][p] = cmake(c, 0.0);
            g.m[p][q] = cmake(s, 0.0);
            g.m[q][p] = cscale(-s, ph);
            g.m[q][q] = cscale(c, ph);
            h = mdmul(g, mmul(h, g));
            v = mmul(v, g);
        }
    }
}

// f(t1, t2) = s1 cos t1 + s2 cos t2 + s3 cos t3,  t3 = -phi - t1 - t2
__device__ __forceinline__ double phase_objective(const double s[3], double phi, double t1, double t2) {
    return s[0] * cos(t1) + s[1] * cos(t2) + s[2] * cos(-phi - t1 - t2);
}

// Phases theta_j, sum_j theta_j = -phi, maximising sum_j s_j cos(theta_j)
// (step 3 of Sec. 5.2): best point of a grid of spacing pi/3 in (theta_1,
// theta_2), then Newton iterations.  A Newton step longer than 0.5, or a
// gradient step (where the Hessian is not negative definite), is halved until
// the objective does not decrease; shorter Newton steps are taken whole.
__device__ inline void maximise_phases(const double s[3], double phi, double th[3]) {
    const double step0 = M_PI / 3.0;
    double t1 = 0.0, t2 = 0.0, fb = -1e300;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            const double f = phase_objective(s, phi, i * step0, j * step0);
            if (f > fb) {
                fb = f;
                t1 = i * step0;
                t2 = j * step0;
            }
        }
    const double ssum = s[0] + s[1] + s[2];
    for (int it = 0; it < 100; ++it) {
        const double t3 = -phi - t1 - t2;
        const double sn1 = sin(t1), sn2 = sin(t2), sn3 = sin(t3);
        const double c1 = cos(t1), c2 = cos(t2), c3 = cos(t3);
        const double g1 = -s[0] * sn1 + s[2] * sn3;
        const double g2 = -s[1] * sn2 + s[2] * sn3;
        if (fabs(g1) + fabs(g2) <= 1e-15 * ssum) break;
        const double h11 = -s[0] * c1 - s[2] * c3;
        const double h22 = -s[1] * c2 - s[2] * c3;
        const double h12 = -s[2] * c3;
        const double det = h11 * h22 - h12 * h12;
        const bool negdef = h11 < 0.0 && det > 0.0;
        double d1, d2;
        if (negdef) {
            d1 = -(h22 * g1 - h12 * g2) / det;
            d2 = -(-h12 * g1 + h11 * g2) / det;
        } else {
            d1 = g1 / (2.0 * ssum);
            d2 = g2 / (2.0 * ssum);
        }
        const bool whole = negdef && fmax(fabs(d1), fabs(d2)) <= 0.5;
        if (whole) {
            t1 += d1;
            t2 += d2;
            continue;
        }
        const double f0 = phase_objective(s, phi, t1, t2);
        double a = 1.0;
        int h = 0;
        while (h < 60 && phase_objective(s, phi, t1 + a * d1, t2 + a * d2) < f0) {
            a *= 0.5;
            ++h;
        }
        if (phase_objective(s, phi, t1 + a * d1, t2 + a * d2) >= f0) {
            t1 += a * d1;
            t2 += a * d2;
        }
    }
    th[0] = t1;
    th[1] = t2;
    th[2] = -phi - t1 - t2;
}

// P_SU(3){A}: with A^dag A = V S^2 V^dag (singular values sorted in
// decreasing order), A = U S V^dag and U = A V S^{-1}; det(U V^dag) = e^{i phi}
// is the phase of det A; the result is U D V^dag = A V diag(e^{i theta}/s) V^dag.
// A must be non-singular.
__device__ inline M3 project_su3(const M3 &a) {
    M3 h = mdmul(a, a), v;
    jacobi_herm3(h, v);
    double lam[3] = {h.m[0][0].re, h.m[1][1].re, h.m[2][2].re};
    int ord[3] = {0, 1, 2};
    // sort eigenvalues (squared singular values) in decreasing order
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2 - i; ++j)
            if (lam[ord[j]] < lam[ord[j + 1]]) {
                const int t = ord[j];
                ord[j] = ord[j + 1];
                ord[j + 1] = t;
            }
    double s[3];
    M3 vs;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s[k] = sqrt(fmax(lam[ord[k]], 0.0));
#pragma unroll
        for (int r = 0; r < 3; ++r) vs.m[r][k] = v.m[r][ord[k]];
    }
    const cd d = mdet(a);
    const double phi = atan2(d.im, d.re);
    double th[3];
    maximise_phases(s, phi, th);
    // B = V diag(e^{i theta}/s) V^dag
    M3 w;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double sc = 1.0 / s[k];
            w.m[r][k] = cmul(vs.m[r][k], cmake(sc * cos(th[k]), sc * sin(th[k])));
        }
    return mmul(a, mmuld(w, vs));
}

// third row of an SU(3) matrix from its first two: r2 = conj(r0 x r1)
template <typename A>
__device__ __forceinline__ void su3_third_row(cx<A> w[3][3]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        w[2][j] = cconj(csub(cmul(w[0][j1], w[1][j2]), cmul(w[0][j2], w[1][j1])));
    }
}

}  // namespace bri
