// BLAS-1 kernels for the solver: every field is nrhs blocks of n real
// numbers (n = 24 V: 12 complex components per site), or, for the inner
// solve on the matrix cores, site-major [V][nrhs][24] FP32.  Reductions are
// deterministic: each workgroup sums a fixed slice in a fixed tree order into
// its own partial (FP64), and a second kernel adds the partials of each
// right-hand side in a fixed order.  No atomics.
#include "blas.h"

namespace bri {
namespace {

constexpr int kB = 256;
constexpr int kMaxBlocks = 1024;
// site-major kernels put every right-hand side into one workgroup, so they
// need more workgroups to keep enough loads in flight
constexpr int kMaxSiteBlocks = 4096;

template <typename T>
__device__ __forceinline__ double to_d(T v) { return (double)v; }

__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = kB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// partial[rhs][blk][0..1] = (sum a_i b_i over real and imaginary parts, sum a_re b_im - a_im b_re)
// over this block's slice, treating consecutive pairs as complex numbers.
template <typename T>
__global__ __launch_bounds__(kB) void k_dot_partial(size_t ncx, const T *__restrict__ a,
                                                    const T *__restrict__ b, double *partial) {
    __shared__ double sh[kB];
    const size_t rhs = blockIdx.y;
    const T *pa = a + rhs * 2 * ncx;
    const T *pb = b + rhs * 2 * ncx;
    double re = 0.0, im = 0.0;
    for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < ncx; i += (size_t)gridDim.x * kB) {
        const double ar = to_d(pa[2 * i]), ai = to_d(pa[2 * i + 1]);
        const double br = to_d(pb[2 * i]), bi = to_d(pb[2 * i + 1]);
        re = fma(ar, br, fma(ai, bi, re));
        im = fma(ar, bi, fma(-ai, br, im));
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0) {
        partial[(rhs * gridDim.x + blockIdx.x) * 2 + 0] = re;
        partial[(rhs * gridDim.x + blockIdx.x) * 2 + 1] = im;
    }
}

__global__ __launch_bounds__(kB) void k_dot_finish(int nblk, const double *partial, double *out) {
    __shared__ double sh[kB];
    const int rhs = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kB) {
        re += partial[((size_t)rhs * nblk + i) * 2 + 0];
        im += partial[((size_t)rhs * nblk + i) * 2 + 1];
    }
    re = block_sum(re, sh);
    im = block_sum(im, sh);
    if (threadIdx.x == 0) {
        out[2 * rhs + 0] = re;
        out[2 * rhs + 1] = im;
    }
}

// r -= alpha q  (per-rhs real alpha), and |r|^2 partials
template <typename T>
__global__ __launch_bounds__(kB) void k_update_r(size_t n, const double *__restrict__ alpha, T *__restrict__ r,
                                                 const T *__restrict__ q, double *partial) {
    __shared__ double sh[kB];
    const size_t rhs = blockIdx.y;
    const double al = alpha[rhs];
    const size_t off = rhs * n;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < n; i += (size_t)gridDim.x * kB) {
        const size_t j = off + i;
        const T rv = (T)((double)r[j] - al * (double)q[j]);
        r[j] = rv;
        acc = fma((double)rv, (double)rv, acc);
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        partial[(rhs * gridDim.x + blockIdx.x) * 2 + 0] = acc;
        partial[(rhs * gridDim.x + blockIdx.x) * 2 + 1] = 0.0;
    }
}

// x += alpha p ; p = z + beta p  (the x step of the iteration, taken with the
// p step so that p is read once)
template <typename T>
__global__ __launch_bounds__(kB) void k_update_xp(size_t n, const double *__restrict__ alpha,
                                                  const double *__restrict__ beta, T *__restrict__ x,
                                                  T *__restrict__ p, const T *__restrict__ z) {
    const size_t rhs = blockIdx.y;
    const double al = alpha[rhs], be = beta[rhs];
    const size_t off = rhs * n;
    for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < n; i += (size_t)gridDim.x * kB) {
        const size_t j = off + i;
        const double pv = (double)p[j];
        x[j] = (T)((double)x[j] + al * pv);
        p[j] = (T)((double)z[j] + be * pv);
    }
}

// dst = src * scale[rhs] (precision conversion), scale may be null (= 1)
template <typename S, typename D>
__global__ __launch_bounds__(kB) void k_convert(size_t n, const S *__restrict__ src,
                                                D *__restrict__ dst, const double *scale) {
    const size_t rhs = blockIdx.y;
    const double sc = scale ? scale[rhs] : 1.0;
    const size_t off = rhs * n;
    for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < n; i += (size_t)gridDim.x * kB)
        dst[off + i] = (D)((double)src[off + i] * sc);
}

// x += scale[rhs] * e  (FP64 x, e of type S)
template <typename S>
__global__ __launch_bounds__(kB) void k_accum(size_t n, const S *__restrict__ e,
                                              double *__restrict__ x, const double *scale) {
    const size_t rhs = blockIdx.y;
    const double sc = scale[rhs];
    const size_t off = rhs * n;
    for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < n; i += (size_t)gridDim.x * kB)
        x[off + i] = fma(sc, (double)e[off + i], x[off + i]);
}

// r = b - Dx and |r|^2 partials (FP64)
__global__ __launch_bounds__(kB) void k_residual(size_t n, const double *__restrict__ b,
                                                 const double *__restrict__ dx,
                                                 double *__restrict__ r, double *partial) {
    __shared__ double sh[kB];
    const size_t rhs = blockIdx.y;
    const size_t off = rhs * n;
    double acc = 0.0;
    for (size_t i = (size_t)blockIdx.x * kB + threadIdx.x; i < n; i += (size_t)gridDim.x * kB) {
        const double v = b[off + i] - dx[off + i];
        r[off + i] = v;
        acc = fma(v, v, acc);
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        partial[(rhs * gridDim.x + blockIdx.x) * 2 + 0] = acc;
        partial[(rhs * gridDim.x + blockIdx.x) * 2 + 1] = 0.0;
    }
}

// CG scalars, one thread per rhs.  State arrays of nrhs doubles each, at
// st + k * nrhs for k = 0 zz, 1 qq, 2 rr, 3 alpha, 4 beta, 5 active, 6 thr2.
__global__ void k_alpha(int nrhs, double *st, const double *qq2) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double *zz = st, *qq = st + nrhs, *alpha = st + 3 * nrhs, *active = st + 5 * nrhs;
    qq[r] = qq2[2 * r];
    const bool ok = active[r] != 0.0 && qq[r] > 0.0;
    alpha[r] = ok ? zz[r] / qq[r] : 0.0;
}

__global__ void k_beta(int nrhs, double *st, const double *rr2, const double *zz2) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double *zz = st, *rr = st + 2 * nrhs, *beta = st + 4 * nrhs, *active = st + 5 * nrhs,
           *thr2 = st + 6 * nrhs;
    rr[r] = rr2[2 * r];
    const double znew = zz2[2 * r];
    const bool ok = active[r] != 0.0 && zz[r] > 0.0;
    beta[r] = ok ? znew / zz[r] : 0.0;
    zz[r] = znew;
    // freeze converged (or broken-down) columns
    if (!(rr[r] > thr2[r]) || !(znew > 0.0)) active[r] = 0.0;
}

__global__ void k_init(int nrhs, double *st, const double *rr2, const double *zz2, double rel2) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    double *zz = st, *rr = st + 2 * nrhs, *alpha = st + 3 * nrhs, *beta = st + 4 * nrhs,
           *active = st + 5 * nrhs, *thr2 = st + 6 * nrhs;
    rr[r] = rr2[2 * r];
    zz[r] = zz2[2 * r];
    thr2[r] = rel2 * rr[r];
    alpha[r] = beta[r] = 0.0;
    active[r] = (rr[r] > 0.0 && zz[r] > 0.0) ? 1.0 : 0.0;
}

// ---- site-major fields [V][nrhs][24] (FP32): the inner solve on the matrix
// cores keeps its vectors in the layout of that apply.  A site's records are
// 6 nrhs chunks of 16 bytes; a workgroup of 6 nrhs m threads covers m
// consecutive sites per pass, a thread one chunk, so that the lanes of every
// load and store are consecutive 16-byte pieces and a thread keeps its
// right-hand side.  The per-rhs block sums are fixed-order: the six chunks
// of a record, then a tree over the m sites; the partials are then added by
// k_dot_finish.  Deterministic.
constexpr int kSiteMax = 6 * 64;  // largest workgroup (64 right-hand sides, one site per pass)
struct SiteBlock {
    int cps, m, sl, c;  // chunks per site, sites per pass, the thread's site in the pass and chunk
    bool on;            // thread inside the m x cps chunks
};
__device__ __forceinline__ SiteBlock site_block(int nrhs) {
    SiteBlock b;
    b.cps = 6 * nrhs;
    b.m = blockDim.x / b.cps;
    b.sl = threadIdx.x / b.cps;
    b.c = threadIdx.x % b.cps;
    b.on = b.sl < b.m;
    return b;
}
__device__ __forceinline__ void site_partial(const SiteBlock &b, int nrhs, double v, double *sh, double *partial) {
    const int t = threadIdx.x;
    sh[t] = b.on ? v : 0.0;
    __syncthreads();
    const bool lead = b.on && b.c % 6 == 0;  // first chunk of a record
    if (lead) {
        double r = sh[t];
#pragma unroll
        for (int i = 1; i < 6; ++i) r += sh[t + i];
        sh[t] = r;
    }
    __syncthreads();
    int p2 = 1;
    while (p2 < b.m) p2 <<= 1;
    for (int h = p2 >> 1; h > 0; h >>= 1) {
        if (lead && b.sl < h && b.sl + h < b.m) sh[t] += sh[t + h * b.cps];
        __syncthreads();
    }
    if (t < nrhs) {
        partial[((size_t)t * gridDim.x + blockIdx.x) * 2 + 0] = sh[6 * t];
        partial[((size_t)t * gridDim.x + blockIdx.x) * 2 + 1] = 0.0;
    }
}
__device__ __forceinline__ double sq4(float4 v, double acc) {
    acc = fma((double)v.x, (double)v.x, acc);
    acc = fma((double)v.y, (double)v.y, acc);
    acc = fma((double)v.z, (double)v.z, acc);
    return fma((double)v.w, (double)v.w, acc);
}

// |a|^2 partials per rhs
__global__ __launch_bounds__(kSiteMax) void k_norm2_sites(size_t V, int nrhs, const float4 *__restrict__ a,
                                                          double *partial) {
    __shared__ double sh[kSiteMax];
    const SiteBlock b = site_block(nrhs);
    double acc = 0.0;
    if (b.on)
        for (size_t s = (size_t)blockIdx.x * b.m + b.sl; s < V; s += (size_t)gridDim.x * b.m)
            acc = sq4(a[s * b.cps + b.c], acc);
    site_partial(b, nrhs, acc, sh, partial);
}

// x += alpha p ; r -= alpha q ; |r|^2 partials
__global__ __launch_bounds__(kSiteMax) void k_update_r_sites(size_t V, int nrhs, const double *__restrict__ alpha,
                                                             float4 *__restrict__ r, const float4 *__restrict__ q,
                                                             double *partial) {
    __shared__ double sh[kSiteMax];
    const SiteBlock b = site_block(nrhs);
    double acc = 0.0;
    if (b.on) {
        const double al = alpha[b.c / 6];
        for (size_t s = (size_t)blockIdx.x * b.m + b.sl; s < V; s += (size_t)gridDim.x * b.m) {
            const size_t o = s * b.cps + b.c;
            const float4 qv = q[o];
            float4 rv = r[o];
            rv.x = (float)((double)rv.x - al * (double)qv.x);
            rv.y = (float)((double)rv.y - al * (double)qv.y);
            rv.z = (float)((double)rv.z - al * (double)qv.z);
            rv.w = (float)((double)rv.w - al * (double)qv.w);
            r[o] = rv;
            acc = sq4(rv, acc);
        }
    }
    site_partial(b, nrhs, acc, sh, partial);
}

// x += alpha p ; p = z + beta p ; |p|^2 partials
__global__ __launch_bounds__(kSiteMax) void k_update_xp_sites(size_t V, int nrhs, const double *__restrict__ alpha,
                                                              const double *__restrict__ beta,
                                                              float4 *__restrict__ x, float4 *__restrict__ p,
                                                              const float4 *__restrict__ z, double *partial) {
    __shared__ double sh[kSiteMax];
    const SiteBlock b = site_block(nrhs);
    double acc = 0.0;
    if (b.on) {
        const double al = alpha[b.c / 6], be = beta[b.c / 6];
        for (size_t s = (size_t)blockIdx.x * b.m + b.sl; s < V; s += (size_t)gridDim.x * b.m) {
            const size_t o = s * b.cps + b.c;
            const float4 pv = p[o], zv = z[o];
            float4 xv = x[o];
            xv.x = (float)((double)xv.x + al * (double)pv.x);
            xv.y = (float)((double)xv.y + al * (double)pv.y);
            xv.z = (float)((double)xv.z + al * (double)pv.z);
            xv.w = (float)((double)xv.w + al * (double)pv.w);
            float4 pn;
            pn.x = (float)((double)zv.x + be * (double)pv.x);
            pn.y = (float)((double)zv.y + be * (double)pv.y);
            pn.z = (float)((double)zv.z + be * (double)pv.z);
            pn.w = (float)((double)zv.w + be * (double)pv.w);
            x[o] = xv;
            p[o] = pn;
            acc = sq4(pn, acc);
        }
    }
    site_partial(b, nrhs, acc, sh, partial);
}

int nblocks(size_t n) {
    size_t b = (n + kB - 1) / kB;
    return (int)(b < (size_t)kMaxBlocks ? b : (size_t)kMaxBlocks);
}

}  // namespace

int dot_blocks(size_t n) { return nblocks(n); }

// sites per pass of a site-major workgroup (6 nrhs m threads, m up to 256 / (6 nrhs))
static int site_m(int nrhs) {
    const int m = kB / (6 * nrhs);
    return m > 0 ? m : 1;
}
int site_blocks(size_t V, int nrhs) {
    const size_t m = (size_t)site_m(nrhs);
    const size_t b = (V + m - 1) / m;
    return (int)(b < (size_t)kMaxSiteBlocks ? b : (size_t)kMaxSiteBlocks);
}
hipError_t norm2_sites(size_t V, int nrhs, const float *a, double *part, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_norm2_sites, dim3(nblk), dim3(6 * nrhs * site_m(nrhs)), 0, st, V, nrhs, (const float4 *)a,
                       part);
    return hipGetLastError();
}
hipError_t update_r_sites(size_t V, int nrhs, const double *alpha, float *r, const float *q, double *part, int nblk,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_update_r_sites, dim3(nblk), dim3(6 * nrhs * site_m(nrhs)), 0, st, V, nrhs, alpha,
                       (float4 *)r, (const float4 *)q, part);
    return hipGetLastError();
}
hipError_t update_xp_sites(size_t V, int nrhs, const double *alpha, const double *beta, float *x, float *p,
                           const float *z, double *part, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_update_xp_sites, dim3(nblk), dim3(6 * nrhs * site_m(nrhs)), 0, st, V, nrhs, alpha, beta,
                       (float4 *)x, (float4 *)p, (const float4 *)z, part);
    return hipGetLastError();
}
template <typename T>
hipError_t dot_partials_t(size_t n, int nrhs, const T *a, const T *b, double *part, int nblk,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(nblk, nrhs), dim3(kB), 0, st, n / 2, a, b, part);
    return hipGetLastError();
}
template hipError_t dot_partials_t<double>(size_t, int, const double *, const double *, double *, int, hipStream_t);
template hipError_t dot_partials_t<float>(size_t, int, const float *, const float *, double *, int, hipStream_t);

hipError_t dot_finish(int nrhs, const double *part, int nblk, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_finish, dim3(nrhs), dim3(kB), 0, st, nblk, part, out);
    return hipGetLastError();
}

template <typename T>
hipError_t update_r(size_t n, int nrhs, const double *alpha, T *r, const T *q, double *part, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_update_r<T>, dim3(nblk, nrhs), dim3(kB), 0, st, n, alpha, r, q, part);
    return hipGetLastError();
}
template hipError_t update_r<double>(size_t, int, const double *, double *, const double *, double *, int, hipStream_t);
template hipError_t update_r<float>(size_t, int, const double *, float *, const float *, double *, int, hipStream_t);

template <typename T>
hipError_t update_xp(size_t n, int nrhs, const double *alpha, const double *beta, T *x, T *p, const T *z,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_update_xp<T>, dim3(nblocks(n), nrhs), dim3(kB), 0, st, n, alpha, beta, x, p, z);
    return hipGetLastError();
}
template hipError_t update_xp<double>(size_t, int, const double *, const double *, double *, double *, const double *,
                                      hipStream_t);
template hipError_t update_xp<float>(size_t, int, const double *, const double *, float *, float *, const float *,
                                     hipStream_t);

template <typename S, typename D>
hipError_t convert(size_t n, int nrhs, const S *src, D *dst, const double *scale, hipStream_t st) {
    hipLaunchKernelGGL((k_convert<S, D>), dim3(nblocks(n), nrhs), dim3(kB), 0, st, n, src, dst, scale);
    return hipGetLastError();
}
template hipError_t convert<double, float>(size_t, int, const double *, float *, const double *, hipStream_t);
template hipError_t convert<double, double>(size_t, int, const double *, double *, const double *, hipStream_t);

template <typename S>
hipError_t accum(size_t n, int nrhs, const S *e, double *x, const double *scale, hipStream_t st) {
    hipLaunchKernelGGL(k_accum<S>, dim3(nblocks(n), nrhs), dim3(kB), 0, st, n, e, x, scale);
    return hipGetLastError();
}
template hipError_t accum<float>(size_t, int, const float *, double *, const double *, hipStream_t);
template hipError_t accum<double>(size_t, int, const double *, double *, const double *, hipStream_t);

hipError_t residual(size_t n, int nrhs, const double *b, const double *dx, double *r, double *part,
                    int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_residual, dim3(nblk, nrhs), dim3(kB), 0, st, n, b, dx, r, part);
    return hipGetLastError();
}

hipError_t cg_init(int nrhs, double *stv, const double *rr2, const double *zz2, double rel2, hipStream_t st) {
    hipLaunchKernelGGL(k_init, dim3((nrhs + 63) / 64), dim3(64), 0, st, nrhs, stv, rr2, zz2, rel2);
    return hipGetLastError();
}
hipError_t cg_alpha(int nrhs, double *stv, const double *qq2, hipStream_t st) {
    hipLaunchKernelGGL(k_alpha, dim3((nrhs + 63) / 64), dim3(64), 0, st, nrhs, stv, qq2);
    return hipGetLastError();
}
hipError_t cg_beta(int nrhs, double *stv, const double *rr2, const double *zz2, hipStream_t st) {
    hipLaunchKernelGGL(k_beta, dim3((nrhs + 63) / 64), dim3(64), 0, st, nrhs, stv, rr2, zz2);
    return hipGetLastError();
}

}  // namespace bri
