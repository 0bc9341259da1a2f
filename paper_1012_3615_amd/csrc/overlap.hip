// The overlap operator with the Brillouin kernel (Sec. 7):
//   * Lanczos on A = D^dag D, whose tridiagonal matrix gives the Ritz values
//     that estimate the extremal eigenvalues of A (Sec. 7.3);
//   * sign(H) for H = gamma5 D (the kernel at mass -rho), written as
//     H (H^2)^{-1/2} = gamma5 D p(A) with p the Chebyshev interpolant of
//     x^{-1/2} on an interval [lo, hi] that holds the spectrum of A, evaluated
//     by Clenshaw's recurrence (one application of A per degree), with optional
//     exact treatment of given low eigenmodes of H;
//   * D_ov,m = (1 - m/(2 rho)) rho (1 + gamma5 sign(H)) + m  (Eqs. def_over, def_mass).
// All fields are FP64 SoA spinors; A and H use the stored-transporter apply.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "abi_internal.h"
#include "blas.h"
#include "kernels.h"

namespace bri {
namespace {

constexpr int kB = 256;

unsigned grid_for(size_t n) {
    size_t b = (n + kB - 1) / kB;
    return (unsigned)std::min<size_t>(b, 8192);
}

// out = a0 x0 + a1 x1 + a2 x2 + a3 x3 over n reals; null inputs are skipped;
// out may be one of the inputs (each element is read before it is written)
__global__ __launch_bounds__(kB) void k_lincomb(size_t n, double a0, const double *x0, double a1,
                                                const double *x1, double a2, const double *x2, double a3,
                                                const double *x3, double *out) {
    for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < n; i += (size_t)gridDim.x * kB) {
        double v = x0 ? a0 * x0[i] : 0.0;
        if (x1) v = fma(a1, x1[i], v);
        if (x2) v = fma(a2, x2[i], v);
        if (x3) v = fma(a3, x3[i], v);
        out[i] = v;
    }
}

// out = a x + b gamma5 y for fields [nrhs][12][V] complex; gamma5 = diag(1,1,-1,-1)
// in spin (components 6..11 change sign); x may be null; out may alias x or y
__global__ __launch_bounds__(kB) void k_gamma5_comb(size_t ncx, size_t V, double a, const double *x, double b,
                                                    const double *y, double *out) {
    for (size_t q = (size_t)blockIdx.x * kB + threadIdx.x; q < ncx; q += (size_t)gridDim.x * kB) {
        const size_t plane = (q / V) % 12;
        const double s = plane >= 6 ? -b : b;
        double re = s * y[2 * q], im = s * y[2 * q + 1];
        if (x) {
            re = fma(a, x[2 * q], re);
            im = fma(a, x[2 * q + 1], im);
        }
        out[2 * q] = re;
        out[2 * q + 1] = im;
    }
}

// y += c x, c complex, over ncx complex numbers
__global__ __launch_bounds__(kB) void k_caxpy(size_t ncx, double cr, double ci, const double *x, double *y) {
    for (size_t q = (size_t)blockIdx.x * kB + threadIdx.x; q < ncx; q += (size_t)gridDim.x * kB) {
        const double xr = x[2 * q], xi = x[2 * q + 1];
        y[2 * q] = fma(cr, xr, fma(-ci, xi, y[2 * q]));
        y[2 * q + 1] = fma(cr, xi, fma(ci, xr, y[2 * q + 1]));
    }
}

// partial[i][blk] = slice sums of <V_i, w> for i < nv (V: nv consecutive fields
// of ncx complex numbers, w one field), fixed order per block
__global__ __launch_bounds__(kB) void k_multidot_partial(size_t ncx, const double *__restrict__ Vb,
                                                         const double *__restrict__ w, double *partial) {
    __shared__ double sr[kB], si[kB];
    const size_t i = blockIdx.y;
    const double *v = Vb + i * 2 * ncx;
    double re = 0.0, im = 0.0;
    for (size_t q = (size_t)blockIdx.x * kB + threadIdx.x; q < ncx; q += (size_t)gridDim.x * kB) {
        const double ar = v[2 * q], ai = v[2 * q + 1], br = w[2 * q], bi = w[2 * q + 1];
        re = fma(ar, br, fma(ai, bi, re));
        im = fma(ar, bi, fma(-ai, br, im));
    }
    sr[threadIdx.x] = re;
    si[threadIdx.x] = im;
    __syncthreads();
    for (int st = kB / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sr[threadIdx.x] += sr[threadIdx.x + st];
            si[threadIdx.x] += si[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[(i * gridDim.x + blockIdx.x) * 2 + 0] = sr[0];
        partial[(i * gridDim.x + blockIdx.x) * 2 + 1] = si[0];
    }
}

// w -= sum_{i < nv} c_i V_i with the complex c_i in device memory (pairs)
__global__ __launch_bounds__(kB) void k_multi_caxpy(size_t ncx, int nv, const double *__restrict__ Vb,
                                                    const double *__restrict__ c, double *w) {
    for (size_t q = (size_t)blockIdx.x * kB + threadIdx.x; q < ncx; q += (size_t)gridDim.x * kB) {
        double re = w[2 * q], im = w[2 * q + 1];
        for (int i = 0; i < nv; ++i) {
            const double cr = c[2 * i], ci = c[2 * i + 1];
            const double vr = Vb[(size_t)i * 2 * ncx + 2 * q], vi = Vb[(size_t)i * 2 * ncx + 2 * q + 1];
            re = fma(-cr, vr, fma(ci, vi, re));
            im = fma(-cr, vi, fma(-ci, vr, im));
        }
        w[2 * q] = re;
        w[2 * q + 1] = im;
    }
}

// Y_i = sum_{j < nv} C_ij V_j for 8 outputs i0..i0+7 per block row (blockIdx.y),
// C real [nout][nv] (cplx = 0) or complex [nout][nv][2] (cplx = 1), in device memory
__global__ __launch_bounds__(kB) void k_combine(size_t ncx, int nv, int nout, const double *__restrict__ Vb,
                                                const double *__restrict__ C, int cplx, double *Y) {
    constexpr int G = 8;
    const int i0 = blockIdx.y * G;
    for (size_t q = (size_t)blockIdx.x * kB + threadIdx.x; q < ncx; q += (size_t)gridDim.x * kB) {
        double re[G], im[G];
#pragma unroll
        for (int g = 0; g < G; ++g) re[g] = im[g] = 0.0;
        for (int j = 0; j < nv; ++j) {
            const double vr = Vb[(size_t)j * 2 * ncx + 2 * q], vi = Vb[(size_t)j * 2 * ncx + 2 * q + 1];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int i = i0 + g;
                if (i >= nout) break;
                if (cplx) {
                    const double cr = C[((size_t)i * nv + j) * 2], ci = C[((size_t)i * nv + j) * 2 + 1];
                    re[g] = fma(cr, vr, fma(-ci, vi, re[g]));
                    im[g] = fma(cr, vi, fma(ci, vr, im[g]));
                } else {
                    const double cr = C[(size_t)i * nv + j];
                    re[g] = fma(cr, vr, re[g]);
                    im[g] = fma(cr, vi, im[g]);
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int i = i0 + g;
            if (i >= nout) break;
            Y[(size_t)i * 2 * ncx + 2 * q] = re[g];
            Y[(size_t)i * 2 * ncx + 2 * q + 1] = im[g];
        }
    }
}

#define OV_TRY(expr)                      \
    do {                                  \
        bri_status _s = (expr);           \
        if (_s != BRI_OK) return _s;      \
    } while (0)
#define OV_HIP(expr, what) OV_TRY(hip_check((expr), what))

struct Ctx {
    bri_dims d;
    Geom g;
    OpDesc op;
    double mass;
    size_t n;  // reals per field (24 V)
    hipStream_t st;
    double *part;  // dot partials
    double *red;   // reduced dots (device)
};

bri_status lincomb(const Ctx &c, size_t n, double a0, const double *x0, double a1, const double *x1, double a2,
                   const double *x2, double a3, const double *x3, double *out) {
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(kB), 0, c.st, n, a0, x0, a1, x1, a2, x2, a3, x3, out);
    return hip_check(hipGetLastError(), "lincomb");
}

bri_status gamma5_comb(const Ctx &c, int nrhs, double a, const double *x, double b, const double *y, double *out) {
    const size_t ncx = c.n / 2 * nrhs;
    hipLaunchKernelGGL(k_gamma5_comb, dim3(grid_for(ncx)), dim3(kB), 0, c.st, ncx, (size_t)c.g.V, a, x, b, y, out);
    return hip_check(hipGetLastError(), "gamma5 combination");
}

bri_status caxpy(const Ctx &c, double cr, double ci, const double *x, double *y) {
    const size_t ncx = c.n / 2;
    hipLaunchKernelGGL(k_caxpy, dim3(grid_for(ncx)), dim3(kB), 0, c.st, ncx, cr, ci, x, y);
    return hip_check(hipGetLastError(), "caxpy");
}

// <a, b> for one field, to the host (synchronises the stream)
bri_status cdot(const Ctx &c, const double *a, const double *b, double *re, double *im) {
    const int nb = dot_blocks(c.n);
    OV_HIP(dot_partials_t<double>(c.n, 1, a, b, c.part, nb, c.st), "dot partials");
    OV_HIP(dot_finish(1, c.part, nb, c.red, c.st), "dot finish");
    double h[2];
    OV_HIP(hipMemcpyAsync(h, c.red, sizeof(h), hipMemcpyDeviceToHost, c.st), "copy to host");
    OV_HIP(hipStreamSynchronize(c.st), "synchronize");
    *re = h[0];
    *im = h[1];
    return BRI_OK;
}

// y = D^dag D x for nrhs fields (t: scratch)
bri_status apply_a(const Ctx &c, const double *x, double *t, double *y, int nrhs) {
    OV_TRY(apply_op(c.d, c.op, BRI_F64, c.mass, x, t, nrhs, c.st, false));
    return apply_op(c.d, c.op, BRI_F64, c.mass, t, y, nrhs, c.st, true);
}

bri_status check_op(const bri_operator *op, OpDesc *o) {
    OV_TRY(op_from_public(op, o));
    if (o->wp != BRI_F64) return fail(BRI_E_UNSUPPORTED, "the overlap routines use FP64 transporters");
    return BRI_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------------ host: tridiagonal eigenvalues
// number of eigenvalues of the symmetric tridiagonal (a, b[1..k-1]) below x (Sturm sequence)
int sturm_count(int k, const double *a, const double *b, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
        const double off = i == 0 ? 0.0 : b[i] * b[i];
        q = a[i] - x - (i == 0 ? 0.0 : off / q);
        if (q == 0.0) q = -1e-300;  // a zero pivot counts as negative
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// all eigenvalues, ascending, by bisection to full precision
std::vector<double> tridiag_eigenvalues(int k, const double *a, const double *b) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < k ? std::fabs(b[i + 1]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    const double scale = std::max(std::fabs(lo), std::fabs(hi));
    std::vector<double> ev(k);
    for (int m = 0; m < k; ++m) {
        double l = lo, h = hi;
        for (int it = 0; it < 200 && h - l > 2e-16 * scale; ++it) {
            const double mid = 0.5 * (l + h);
            if (sturm_count(k, a, b, mid) > m)
                h = mid;
            else
                l = mid;
        }
        ev[m] = 0.5 * (l + h);
    }
    return ev;
}

// eigenvector of the symmetric tridiagonal (a, b[1..k-1]) for the eigenvalue
// theta by inverse iteration: Gaussian elimination with partial pivoting of
// T - theta 1 (rows swapped where the sub-diagonal entry is larger, which
// fills a second super-diagonal), three solves from a constant start, each
// made orthogonal to the vectors in `prev` (earlier members of a cluster)
std::vector<double> tridiag_eigvec(int k, const double *a, const double *b, double theta,
                                   const std::vector<std::vector<double>> &prev) {
    double tn = 0.0;
    for (int i = 0; i < k; ++i) tn = std::max(tn, std::fabs(a[i]) + (i ? std::fabs(b[i]) : 0.0));
    const double tiny = std::max(tn, 1e-300) * 1e-15;
    std::vector<double> d(k), du(k, 0.0), du2(k, 0.0), l(k, 0.0);
    std::vector<int> swp(k, 0);
    for (int i = 0; i < k; ++i) {
        d[i] = a[i] - theta;
        if (i + 1 < k) du[i] = b[i + 1];
    }
    std::vector<double> dl(k, 0.0);
    for (int i = 0; i + 1 < k; ++i) dl[i] = b[i + 1];
    for (int i = 0; i + 1 < k; ++i) {
        if (std::fabs(d[i]) >= std::fabs(dl[i])) {
            if (d[i] == 0.0) d[i] = tiny;
            l[i] = dl[i] / d[i];
            d[i + 1] -= l[i] * du[i];
        } else {
            // swap rows i and i+1
            const double r0 = d[i], r1 = du[i];           // old row i: (d_i, du_i, 0)
            const double s0 = dl[i], s1 = d[i + 1], s2 = i + 2 < k ? du[i + 1] : 0.0;  // old row i+1
            d[i] = s0;
            du[i] = s1;
            du2[i] = s2;
            l[i] = r0 / s0;
            d[i + 1] = r1 - l[i] * s1;
            if (i + 2 < k) du[i + 1] = -l[i] * s2;
            swp[i] = 1;
        }
    }
    if (d[k - 1] == 0.0) d[k - 1] = tiny;
    std::vector<double> y(k, 1.0);
    for (int it = 0; it < 3; ++it) {
        // forward: apply the row operations to the right-hand side
        for (int i = 0; i + 1 < k; ++i) {
            if (swp[i]) std::swap(y[i], y[i + 1]);
            y[i + 1] -= l[i] * y[i];
        }
        // back substitution with U (diagonal d, super-diagonals du, du2)
        for (int i = k - 1; i >= 0; --i) {
            double v = y[i];
            if (i + 1 < k) v -= du[i] * y[i + 1];
            if (i + 2 < k) v -= du2[i] * y[i + 2];
            y[i] = v / (d[i] != 0.0 ? d[i] : tiny);
        }
        for (const auto &p : prev) {
            double dp = 0.0;
            for (int i = 0; i < k; ++i) dp += p[i] * y[i];
            for (int i = 0; i < k; ++i) y[i] -= dp * p[i];
        }
        double nrm = 0.0;
        for (double v : y) nrm += v * v;
        nrm = std::sqrt(nrm);
        for (double &v : y) v /= nrm;
    }
    return y;
}

// Hermitian n x n eigen-decomposition by cyclic complex Jacobi rotations
// (each rotation first removes the phase of the off-diagonal element, then
// applies the real symmetric rotation that zeroes it).  h row-major, z the
// eigenvectors in its columns, w the eigenvalues.
void jacobi_herm(int n, std::vector<std::complex<double>> h, std::vector<std::complex<double>> &z,
                 std::vector<double> &w) {
    using C = std::complex<double>;
    z.assign((size_t)n * n, C(0.0, 0.0));
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int p = 0; p < n; ++p) {
            dia += std::abs(h[(size_t)p * n + p]);
            for (int q = p + 1; q < n; ++q) off += std::norm(h[(size_t)p * n + q]);
        }
        if (off <= 1e-34 * dia * dia) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const C hpq = h[(size_t)p * n + q];
                const double r = std::abs(hpq);
                if (r == 0.0) continue;
                const C ph = std::conj(hpq) / r;  // e^{-i beta}
                const double tau = (h[(size_t)q * n + q].real() - h[(size_t)p * n + p].real()) / (2.0 * r);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                // G acts on columns p, q: G_pp = c, G_pq = s, G_qp = -s ph, G_qq = c ph
                const C gpp = c, gpq = s, gqp = -s * ph, gqq = c * ph;
                for (int i = 0; i < n; ++i) {  // h <- h G
                    const C hp = h[(size_t)i * n + p], hq = h[(size_t)i * n + q];
                    h[(size_t)i * n + p] = hp * gpp + hq * gqp;
                    h[(size_t)i * n + q] = hp * gpq + hq * gqq;
                }
                for (int j = 0; j < n; ++j) {  // h <- G^dag h
                    const C hp = h[(size_t)p * n + j], hq = h[(size_t)q * n + j];
                    h[(size_t)p * n + j] = std::conj(gpp) * hp + std::conj(gqp) * hq;
                    h[(size_t)q * n + j] = std::conj(gpq) * hp + std::conj(gqq) * hq;
                }
                for (int i = 0; i < n; ++i) {  // z <- z G
                    const C zp = z[(size_t)i * n + p], zq = z[(size_t)i * n + q];
                    z[(size_t)i * n + p] = zp * gpp + zq * gqp;
                    z[(size_t)i * n + q] = zp * gpq + zq * gqq;
                }
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = h[(size_t)i * n + i].real();
}

// Chebyshev interpolant of x^{-1/2} on [lo, hi] at the degree+1 Chebyshev-Gauss
// nodes: coefficients of T_k((x - mid)/hw)
std::vector<double> inv_sqrt_coeffs(double lo, double hi, int degree) {
    const int M = degree + 1;
    const double hw = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    std::vector<double> f(M), cf(M);
    for (int j = 0; j < M; ++j) f[j] = 1.0 / std::sqrt(hw * std::cos(M_PI * (j + 0.5) / M) + mid);
    for (int kk = 0; kk < M; ++kk) {
        double s = 0.0;
        for (int j = 0; j < M; ++j) s += f[j] * std::cos(M_PI * kk * (j + 0.5) / M);
        cf[kk] = 2.0 * s / M;
    }
    cf[0] *= 0.5;
    return cf;
}

// max over 20001 equidistant points of [lo, hi] of |1 - sqrt(x) p(x)|
double inv_sqrt_error(double lo, double hi, const std::vector<double> &cf) {
    const int N = (int)cf.size() - 1;
    const double hw = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    double e = 0.0;
    for (int i = 0; i <= 20000; ++i) {
        const double x = lo + (hi - lo) * i / 20000.0, tt = (x - mid) / hw;
        double u1 = 0.0, u2 = 0.0;
        for (int kk = N; kk >= 1; --kk) {
            const double u = cf[kk] + 2.0 * tt * u1 - u2;
            u2 = u1;
            u1 = u;
        }
        e = std::max(e, std::fabs(1.0 - std::sqrt(x) * (cf[0] + tt * u1 - u2)));
    }
    return e;
}

}  // namespace
}  // namespace bri

using namespace bri;

extern "C" {

size_t bri_lanczos_workspace_bytes(bri_dims d, int32_t k) {
    Geom g;
    if (!dims_ok(d, &g) || k < 1) return 0;
    const size_t fb = align256((size_t)24 * g.V * sizeof(double));
    // 4 fields, dot partials for up to k vectors, k reduced complex dots
    return 4 * fb + align256((size_t)k * 1024 * 2 * sizeof(double)) + align256((size_t)k * 2 * sizeof(double));
}

bri_status bri_lanczos(bri_dims d, const bri_operator *op, double mass, int32_t k, const double *v0, double *alpha,
                       double *beta, double *basis, int32_t *k_done, void *work, size_t work_bytes, void *stream) {
    g_last_error.clear();
    Ctx c{};
    if (!dims_ok(d, &c.g)) return fail(BRI_E_ARG, "invalid lattice extents");
    OV_TRY(check_op(op, &c.op));
    if (k < 1 || k > 100000) return fail(BRI_E_ARG, "k must be in [1, 100000]");
    if (!alpha || !beta || !k_done) return fail(BRI_E_ARG, "null host output");
    if (basis && k > 65535) return fail(BRI_E_ARG, "k must be <= 65535 when the basis is kept");
    if (!aligned(v0) || (basis && !aligned(basis))) return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t need = bri_lanczos_workspace_bytes(d, k);
    if (!aligned(work) || work_bytes < need) return fail(BRI_E_WORKSPACE, "workspace too small: need %zu bytes", need);
    c.d = d;
    c.mass = mass;
    c.n = (size_t)24 * c.g.V;
    c.st = (hipStream_t)stream;
    const size_t fb = align256(c.n * sizeof(double));
    char *w8 = (char *)work;
    double *w = (double *)w8, *t = (double *)(w8 + fb), *va = (double *)(w8 + 2 * fb), *vb = (double *)(w8 + 3 * fb);
    c.part = (double *)(w8 + 4 * fb);
    c.red = (double *)(w8 + 4 * fb + align256((size_t)k * 1024 * 2 * sizeof(double)));
    if (basis && overlap(basis, (size_t)k * c.n * sizeof(double), work, need))
        return fail(BRI_E_ARG, "the basis overlaps the workspace");

    double re, im;
    OV_TRY(cdot(c, v0, v0, &re, &im));
    const double b0 = std::sqrt(re);
    if (!(b0 > 0.0) || !std::isfinite(b0)) return fail(BRI_E_ARG, "the start vector is zero or not finite");
    beta[0] = b0;
    double *vcur = basis ? basis : va, *vprev = nullptr;
    OV_TRY(lincomb(c, c.n, 1.0 / b0, v0, 0, nullptr, 0, nullptr, 0, nullptr, vcur));
    *k_done = 0;
    for (int j = 0; j < k; ++j) {
        OV_TRY(apply_a(c, vcur, t, w, 1));
        OV_TRY(cdot(c, vcur, w, &re, &im));
        alpha[j] = re;
        // w -= alpha_j v_j + beta_j v_{j-1}
        OV_TRY(lincomb(c, c.n, 1.0, w, -re, vcur, vprev ? -beta[j] : 0.0, vprev, 0, nullptr, w));
        if (basis) {
            // two classical Gram-Schmidt passes against all kept vectors: all
            // dots in one launch, reduced on the device, one fused subtraction
            const int nv = j + 1, nb = dot_blocks(c.n);
            const size_t ncx = c.n / 2;
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_multidot_partial, dim3(nb, nv), dim3(kB), 0, c.st, ncx, basis, w, c.part);
                OV_HIP(hipGetLastError(), "multidot");
                OV_HIP(dot_finish(nv, c.part, nb, c.red, c.st), "multidot finish");
                hipLaunchKernelGGL(k_multi_caxpy, dim3(grid_for(ncx)), dim3(kB), 0, c.st, ncx, nv, basis, c.red, w);
                OV_HIP(hipGetLastError(), "multi axpy");
            }
        }
        OV_TRY(cdot(c, w, w, &re, &im));
        const double bn = std::sqrt(std::max(re, 0.0));
        *k_done = j + 1;
        if (j + 1 == k) break;
        beta[j + 1] = bn;
        if (!(bn > 1e-300)) break;  // invariant subspace: T_{j+1} is exact
        double *vnext = basis ? basis + (size_t)(j + 1) * c.n : (vcur == va ? vb : va);
        if (!basis && vprev) vnext = vprev;  // reuse the buffer of v_{j-1}
        OV_TRY(lincomb(c, c.n, 1.0 / bn, w, 0, nullptr, 0, nullptr, 0, nullptr, vnext));
        vprev = vcur;
        vcur = vnext;
    }
    return BRI_OK;
}

size_t bri_lowmodes_workspace_bytes(bri_dims d, int32_t k, int32_t n_low) {
    Geom g;
    if (!dims_ok(d, &g) || k < 1 || n_low < 1 || n_low > k) return 0;
    const size_t fb = align256((size_t)24 * g.V * n_low * sizeof(double));
    return bri_lanczos_workspace_bytes(d, k) + 3 * fb + align256((size_t)n_low * k * sizeof(double)) +
           align256((size_t)n_low * n_low * 2 * sizeof(double)) + align256((size_t)n_low * 1024 * 2 * sizeof(double)) +
           align256((size_t)n_low * n_low * 2 * sizeof(double));
}

bri_status bri_overlap_lowmodes(bri_dims d, const bri_operator *op, double mass, int32_t k, const double *v0,
                                int32_t n_low, double *basis, double *vecs, double *evals, double *resid, void *work,
                                size_t work_bytes, void *stream) {
    g_last_error.clear();
    Ctx c{};
    if (!dims_ok(d, &c.g)) return fail(BRI_E_ARG, "invalid lattice extents");
    OV_TRY(check_op(op, &c.op));
    if (k < 1 || k > 65535 || n_low < 1 || n_low > k) return fail(BRI_E_ARG, "need 1 <= n_low <= k <= 65535");
    if (!aligned(basis) || !aligned(vecs) || !evals || !resid) return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t need = bri_lowmodes_workspace_bytes(d, k, n_low);
    if (!aligned(work) || work_bytes < need) return fail(BRI_E_WORKSPACE, "workspace too small: need %zu bytes", need);
    c.d = d;
    c.mass = mass;
    c.n = (size_t)24 * c.g.V;
    c.st = (hipStream_t)stream;
    const size_t ncx = c.n / 2, nf = c.n * n_low;
    const size_t lw = bri_lanczos_workspace_bytes(d, k), fb = align256(nf * sizeof(double));
    char *w8 = (char *)work;
    double *X = (double *)(w8 + lw), *HX = (double *)(w8 + lw + fb), *T = (double *)(w8 + lw + 2 * fb);
    char *q8 = w8 + lw + 3 * fb;
    double *Cr = (double *)q8;
    q8 += align256((size_t)n_low * k * sizeof(double));
    double *Cz = (double *)q8;
    q8 += align256((size_t)n_low * n_low * 2 * sizeof(double));
    c.part = (double *)q8;
    q8 += align256((size_t)n_low * 1024 * 2 * sizeof(double));
    c.red = (double *)q8;
    if (overlap(basis, (size_t)k * c.n * sizeof(double), work, need) ||
        overlap(vecs, nf * sizeof(double), work, need) || overlap(vecs, nf * sizeof(double), basis, (size_t)k * c.n * sizeof(double)))
        return fail(BRI_E_ARG, "basis, vecs and the workspace must not overlap");

    // 1. re-orthogonalised Lanczos with the basis kept
    std::vector<double> al(k), be(k);
    int32_t kd = 0;
    OV_TRY(bri_lanczos(d, op, mass, k, v0, al.data(), be.data(), basis, &kd, work, lw, stream));
    if (kd < n_low) return fail(BRI_E_NOCONV, "Lanczos stopped after %d steps (< n_low)", kd);
    // 2. the n_low smallest eigenpairs of T by bisection and inverse iteration
    const std::vector<double> th = tridiag_eigenvalues(kd, al.data(), be.data());
    std::vector<std::vector<double>> ys;
    const double scale = std::max(std::fabs(th.front()), std::fabs(th.back()));
    for (int i = 0; i < n_low; ++i) {
        std::vector<std::vector<double>> cl;  // earlier members of this cluster
        for (int j = 0; j < i; ++j)
            if (std::fabs(th[i] - th[j]) <= 1e-8 * scale) cl.push_back(ys[j]);
        ys.push_back(tridiag_eigvec(kd, al.data(), be.data(), th[i], cl));
    }
    std::vector<double> ch((size_t)n_low * kd);
    for (int i = 0; i < n_low; ++i)
        for (int j = 0; j < kd; ++j) ch[(size_t)i * kd + j] = ys[i][j];
    OV_HIP(hipMemcpyAsync(Cr, ch.data(), ch.size() * sizeof(double), hipMemcpyHostToDevice, c.st), "copy");
    // 3. Ritz vectors X_i = sum_j y_ij V_j
    hipLaunchKernelGGL(k_combine, dim3(grid_for(ncx), (n_low + 7) / 8), dim3(kB), 0, c.st, ncx, kd, n_low, basis, Cr,
                       0, X);
    OV_HIP(hipGetLastError(), "combine");
    // 4. Rayleigh-Ritz for H = gamma5 D on span{X}: G_ij = <X_i, H X_j>
    OV_TRY(apply_op(c.d, c.op, BRI_F64, c.mass, X, T, n_low, c.st, false));
    OV_TRY(gamma5_comb(c, n_low, 0.0, nullptr, 1.0, T, HX));
    const int nb = dot_blocks(c.n);
    for (int j = 0; j < n_low; ++j) {
        hipLaunchKernelGGL(k_multidot_partial, dim3(nb, n_low), dim3(kB), 0, c.st, ncx, X, HX + (size_t)j * c.n, c.part);
        OV_HIP(hipGetLastError(), "gram");
        OV_HIP(dot_finish(n_low, c.part, nb, c.red + (size_t)j * n_low * 2, c.st), "gram finish");
    }
    std::vector<double> gh((size_t)n_low * n_low * 2);
    OV_HIP(hipMemcpyAsync(gh.data(), c.red, gh.size() * sizeof(double), hipMemcpyDeviceToHost, c.st), "copy");
    OV_HIP(hipStreamSynchronize(c.st), "synchronize");
    std::vector<std::complex<double>> G((size_t)n_low * n_low), Z;
    for (int j = 0; j < n_low; ++j)
        for (int i = 0; i < n_low; ++i)  // red[j][i] = <X_i, H X_j> = G_ij
            G[(size_t)i * n_low + j] = {gh[((size_t)j * n_low + i) * 2], gh[((size_t)j * n_low + i) * 2 + 1]};
    for (int i = 0; i < n_low; ++i)  // symmetrise (rounding)
        for (int j = i + 1; j < n_low; ++j) {
            const auto a = 0.5 * (G[(size_t)i * n_low + j] + std::conj(G[(size_t)j * n_low + i]));
            G[(size_t)i * n_low + j] = a;
            G[(size_t)j * n_low + i] = std::conj(a);
        }
    std::vector<double> mu;
    jacobi_herm(n_low, G, Z, mu);
    std::vector<int> ord(n_low);
    for (int i = 0; i < n_low; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int x, int y) { return std::fabs(mu[x]) < std::fabs(mu[y]); });
    // 5. v_i = sum_j Z_{j, ord_i} X_j
    std::vector<double> zc((size_t)n_low * n_low * 2);
    for (int i = 0; i < n_low; ++i) {
        evals[i] = mu[ord[i]];
        for (int j = 0; j < n_low; ++j) {
            zc[((size_t)i * n_low + j) * 2] = Z[(size_t)j * n_low + ord[i]].real();
            zc[((size_t)i * n_low + j) * 2 + 1] = Z[(size_t)j * n_low + ord[i]].imag();
        }
    }
    OV_HIP(hipMemcpyAsync(Cz, zc.data(), zc.size() * sizeof(double), hipMemcpyHostToDevice, c.st), "copy");
    hipLaunchKernelGGL(k_combine, dim3(grid_for(ncx), (n_low + 7) / 8), dim3(kB), 0, c.st, ncx, n_low, n_low, X, Cz,
                       1, vecs);
    OV_HIP(hipGetLastError(), "combine");
    // 6. residuals |H v_i - mu_i v_i|
    OV_TRY(apply_op(c.d, c.op, BRI_F64, c.mass, vecs, T, n_low, c.st, false));
    OV_TRY(gamma5_comb(c, n_low, 0.0, nullptr, 1.0, T, HX));
    for (int i = 0; i < n_low; ++i)
        OV_TRY(lincomb(c, c.n, 1.0, HX + (size_t)i * c.n, -evals[i], vecs + (size_t)i * c.n, 0, nullptr, 0, nullptr,
                       HX + (size_t)i * c.n));
    OV_HIP(dot_partials_t<double>(c.n, n_low, HX, HX, c.part, nb, c.st), "residual partials");
    OV_HIP(dot_finish(n_low, c.part, nb, c.red, c.st), "residual finish");
    std::vector<double> rr((size_t)n_low * 2);
    OV_HIP(hipMemcpyAsync(rr.data(), c.red, rr.size() * sizeof(double), hipMemcpyDeviceToHost, c.st), "copy");
    OV_HIP(hipStreamSynchronize(c.st), "synchronize");
    for (int i = 0; i < n_low; ++i) resid[i] = std::sqrt(std::max(rr[2 * i], 0.0));
    return BRI_OK;
}

bri_status bri_ritz_values(int32_t k, const double *alpha, const double *beta, int32_t filter, double *out,
                           int32_t *n_out) {
    g_last_error.clear();
    if (k < 1 || !alpha || !beta || !out || !n_out) return fail(BRI_E_ARG, "invalid arguments");
    std::vector<double> ev = tridiag_eigenvalues(k, alpha, beta);
    if (!filter || k == 1) {
        std::copy(ev.begin(), ev.end(), out);
        *n_out = k;
        return BRI_OK;
    }
    // Cullum-Willoughby: a simple eigenvalue of T_k that is also an eigenvalue
    // of T_k without its first row and column is spurious; numerically
    // multiple eigenvalues are converged copies and are kept once
    std::vector<double> eh = tridiag_eigenvalues(k - 1, alpha + 1, beta + 1);
    const double scale = std::max(std::fabs(ev.front()), std::fabs(ev.back()));
    const double tol = 1e-10 * scale;
    int n = 0;
    for (int i = 0; i < k;) {
        int j = i + 1;
        while (j < k && ev[j] - ev[j - 1] <= tol) ++j;
        bool keep = true;
        if (j - i == 1) {
            const auto it = std::lower_bound(eh.begin(), eh.end(), ev[i] - tol);
            keep = !(it != eh.end() && *it <= ev[i] + tol);
        }
        if (keep) out[n++] = ev[i];
        i = j;
    }
    *n_out = n;
    return BRI_OK;
}

bri_status bri_sign_approx_error(double lo, double hi, int32_t degree, double *err) {
    g_last_error.clear();
    if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi)) return fail(BRI_E_ARG, "need 0 < lo < hi");
    if (degree < 0 || degree > 100000 || !err) return fail(BRI_E_ARG, "invalid degree or output");
    *err = inv_sqrt_error(lo, hi, inv_sqrt_coeffs(lo, hi, degree));
    return BRI_OK;
}

size_t bri_sign_workspace_bytes(bri_dims d, int32_t nrhs) {
    Geom g;
    if (!dims_ok(d, &g) || nrhs < 1 || nrhs > BRI_MAX_RHS) return 0;
    const size_t fb = align256((size_t)24 * g.V * nrhs * sizeof(double));
    return 5 * fb + align256(1024 * 2 * sizeof(double)) + 256;
}

bri_status bri_sign_h(bri_dims d, const bri_operator *op, double mass, double lo, double hi, int32_t degree,
                      int32_t n_low, const double *low_vecs, const double *low_evals, const double *psi, double *out,
                      int32_t nrhs, double *approx_err, void *work, size_t work_bytes, void *stream) {
    g_last_error.clear();
    Ctx c{};
    if (!dims_ok(d, &c.g)) return fail(BRI_E_ARG, "invalid lattice extents");
    OV_TRY(check_op(op, &c.op));
    if (nrhs < 1 || nrhs > BRI_MAX_RHS) return fail(BRI_E_ARG, "nrhs must be in [1, %d]", BRI_MAX_RHS);
    if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi)) return fail(BRI_E_ARG, "need 0 < lo < hi");
    if (degree < 0 || degree > 100000) return fail(BRI_E_ARG, "degree must be in [0, 100000]");
    if (n_low < 0 || (n_low > 0 && (!aligned(low_vecs) || !low_evals)))
        return fail(BRI_E_ARG, "invalid low modes");
    if (!aligned(psi) || !aligned(out)) return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t need = bri_sign_workspace_bytes(d, nrhs);
    if (!aligned(work) || work_bytes < need) return fail(BRI_E_WORKSPACE, "workspace too small: need %zu bytes", need);
    c.d = d;
    c.mass = mass;
    c.n = (size_t)24 * c.g.V;
    c.st = (hipStream_t)stream;
    const size_t nt = c.n * nrhs;
    if (overlap(psi, nt * sizeof(double), out, nt * sizeof(double))) return fail(BRI_E_ARG, "psi and out overlap");
    const size_t fb = align256(nt * sizeof(double));
    char *w8 = (char *)work;
    double *P = (double *)w8, *b1 = (double *)(w8 + fb), *b2 = (double *)(w8 + 2 * fb);
    double *t1 = (double *)(w8 + 3 * fb), *t2 = (double *)(w8 + 4 * fb);
    c.part = (double *)(w8 + 5 * fb);
    c.red = (double *)(w8 + 5 * fb + align256(1024 * 2 * sizeof(double)));

    const int N = degree;
    const double hw = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    const std::vector<double> cf = inv_sqrt_coeffs(lo, hi, degree);
    if (approx_err) *approx_err = inv_sqrt_error(lo, hi, cf);

    // deflation: P = psi - sum_i v_i <v_i, psi> per right-hand side
    std::vector<double> cr((size_t)nrhs * n_low), ci((size_t)nrhs * n_low);
    const double *src = psi;
    if (n_low > 0) {
        OV_HIP(hipMemcpyAsync(P, psi, nt * sizeof(double), hipMemcpyDeviceToDevice, c.st), "copy");
        for (int r = 0; r < nrhs; ++r)
            for (int i = 0; i < n_low; ++i) {
                const double *vi = low_vecs + (size_t)i * c.n;
                double *pr = P + (size_t)r * c.n;
                OV_TRY(cdot(c, vi, psi + (size_t)r * c.n, &cr[(size_t)r * n_low + i], &ci[(size_t)r * n_low + i]));
                OV_TRY(caxpy(c, -cr[(size_t)r * n_low + i], -ci[(size_t)r * n_low + i], vi, pr));
            }
        src = P;
    }

    // Clenshaw: b_k = c_k P + 2 tau(A) b_{k+1} - b_{k+2}, tau(A) = (A - mid)/hw;
    // p(A) P = c_0 P + tau(A) b_1 - b_2
    double *y;
    if (N == 0) {
        OV_TRY(lincomb(c, nt, cf[0], src, 0, nullptr, 0, nullptr, 0, nullptr, b1));
        y = b1;
    } else {
        double *bk1 = b1, *bk2 = b2;  // b_{k+1}, b_{k+2}
        OV_TRY(lincomb(c, nt, cf[N], src, 0, nullptr, 0, nullptr, 0, nullptr, bk1));  // b_N
        OV_TRY(lincomb(c, nt, 0.0, src, 0, nullptr, 0, nullptr, 0, nullptr, bk2));     // b_{N+1} = 0
        for (int kk = N - 1; kk >= 1; --kk) {
            OV_TRY(apply_a(c, bk1, t1, t2, nrhs));
            OV_TRY(lincomb(c, nt, cf[kk], src, 2.0 / hw, t2, -2.0 * mid / hw, bk1, -1.0, bk2, bk2));
            std::swap(bk1, bk2);
        }
        OV_TRY(apply_a(c, bk1, t1, t2, nrhs));
        OV_TRY(lincomb(c, nt, cf[0], src, 1.0 / hw, t2, -mid / hw, bk1, -1.0, bk2, bk2));
        y = bk2;
    }
    // sign(H) P = gamma5 D p(A) P
    OV_TRY(apply_op(c.d, c.op, BRI_F64, c.mass, y, t1, nrhs, c.st, false));
    OV_TRY(gamma5_comb(c, nrhs, 0.0, nullptr, 1.0, t1, out));
    // + sum_i sign(lambda_i) v_i <v_i, psi>
    for (int r = 0; r < nrhs; ++r)
        for (int i = 0; i < n_low; ++i) {
            const double s = low_evals[i] > 0.0 ? 1.0 : (low_evals[i] < 0.0 ? -1.0 : 0.0);
            OV_TRY(caxpy(c, s * cr[(size_t)r * n_low + i], s * ci[(size_t)r * n_low + i],
                         low_vecs + (size_t)i * c.n, out + (size_t)r * c.n));
        }
    return BRI_OK;
}

bri_status bri_overlap_apply(bri_dims d, const bri_operator *op, double rho, double m, double lo, double hi,
                             int32_t degree, int32_t n_low, const double *low_vecs, const double *low_evals,
                             const double *psi, double *out, int32_t nrhs, double *approx_err, void *work,
                             size_t work_bytes, void *stream) {
    g_last_error.clear();
    if (!(rho > 0.0 && rho < 2.0)) return fail(BRI_E_ARG, "rho must be in (0, 2)");
    if (!std::isfinite(m)) return fail(BRI_E_ARG, "m must be finite");
    OV_TRY(bri_sign_h(d, op, -rho, lo, hi, degree, n_low, low_vecs, low_evals, psi, out, nrhs, approx_err, work,
                      work_bytes, stream));
    Ctx c{};
    dims_ok(d, &c.g);
    c.n = (size_t)24 * c.g.V;
    c.st = (hipStream_t)stream;
    // out = [(1 - m/(2 rho)) rho + m] psi + (1 - m/(2 rho)) rho gamma5 sign(H) psi
    const double f = (1.0 - m / (2.0 * rho)) * rho;
    return gamma5_comb(c, nrhs, f + m, psi, f, out, out);
}

}  // extern "C"
