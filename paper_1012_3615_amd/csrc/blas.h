// BLAS-1 kernels of the solver (blas.hip).  Fields are nrhs consecutive blocks
// of n real numbers; per-rhs scalars live in device memory.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace bri {

int dot_blocks(size_t n);
// partial sums of <a,b> (complex; n real numbers = n/2 complex) per block
template <typename T>
hipError_t dot_partials_t(size_t n, int nrhs, const T *a, const T *b, double *part, int nblk,
                          hipStream_t st);
// out[2*rhs + {0,1}] = sum of the partials (fixed order)
hipError_t dot_finish(int nrhs, const double *part, int nblk, double *out, hipStream_t st);
// r -= alpha q, |r|^2 partials
template <typename T>
hipError_t update_r(size_t n, int nrhs, const double *alpha, T *r, const T *q, double *part, int nblk, hipStream_t st);
// x += alpha p, then p = z + beta p (the x step deferred to the p step, which
// reads p anyway)
template <typename T>
hipError_t update_xp(size_t n, int nrhs, const double *alpha, const double *beta, T *x, T *p, const T *z,
                     hipStream_t st);
// dst = src * scale[rhs]
template <typename S, typename D>
hipError_t convert(size_t n, int nrhs, const S *src, D *dst, const double *scale, hipStream_t st);
// x += scale[rhs] * e
template <typename S>
hipError_t accum(size_t n, int nrhs, const S *e, double *x, const double *scale, hipStream_t st);
// site-major FP32 fields [V][nrhs][24] (nrhs <= 64): partials per rhs over
// site_blocks(V, nrhs) <= 4096 workgroups, summed by dot_finish
int site_blocks(size_t V, int nrhs);
hipError_t norm2_sites(size_t V, int nrhs, const float *a, double *part, int nblk, hipStream_t st);
// r -= alpha q, |r|^2 partials
hipError_t update_r_sites(size_t V, int nrhs, const double *alpha, float *r, const float *q, double *part, int nblk,
                          hipStream_t st);
// x += alpha p, p = z + beta p, |p|^2 partials
hipError_t update_xp_sites(size_t V, int nrhs, const double *alpha, const double *beta, float *x, float *p,
                           const float *z, double *part, int nblk, hipStream_t st);
// r = b - dx, |r|^2 partials
hipError_t residual(size_t n, int nrhs, const double *b, const double *dx, double *r, double *part,
                    int nblk, hipStream_t st);
// CG scalar state: 7 arrays of nrhs doubles at st + k*nrhs:
// k = 0 zz, 1 qq, 2 rr, 3 alpha, 4 beta, 5 active, 6 thr2
hipError_t cg_init(int nrhs, double *stv, const double *rr2, const double *zz2, double rel2,
                   hipStream_t st);
hipError_t cg_alpha(int nrhs, double *stv, const double *qq2, hipStream_t st);
hipError_t cg_beta(int nrhs, double *stv, const double *rr2, const double *zz2, hipStream_t st);

}  // namespace bri
