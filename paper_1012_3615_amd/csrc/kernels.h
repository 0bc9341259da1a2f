// Host-side launchers of the HIP kernels (internal to the library; the public
// C ABI is include/bri.h).  Precision codes: 0 = FP64, 1 = FP32, 2 = FP16.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace bri {

// apply.hip
hipError_t apply_stored(const Geom &g, int noff, int wp, int sp, int kernel, int rblk, const void *W,
                        const void *in, void *out, double diag, int nrhs, bool dag, hipStream_t st,
                        const double *table = nullptr);
#define BRI_DECL_APPLY(tag)                                                                        \
    hipError_t apply_stored_##tag(const Geom &g, int noff, int kernel, int rblk, const void *W,    \
                                  const void *in, void *out, double diag, int nrhs, bool dag,     \
                                  hipStream_t st, const double *table);
BRI_DECL_APPLY(f64)
BRI_DECL_APPLY(f32)
BRI_DECL_APPLY(f16)
BRI_DECL_APPLY(f16h)
#undef BRI_DECL_APPLY
// apply_prod_*.hip: production-operator and generic-class forms of the
// stored apply (80 offsets; rows 3 or 2; clover in the spinor precision or
// nullptr; table lambda_0..4, rho_1..4 or nullptr for the Brillouin column)
#define BRI_DECL_PROD(tag)                                                                         \
    hipError_t apply_prod_##tag(const Geom &g, int rows, int rblk, const void *W, const void *in,  \
                                void *out, double diag, int nrhs, bool dag, hipStream_t st,        \
                                const void *clover, const double *table);
BRI_DECL_PROD(f64)
BRI_DECL_PROD(f32)
BRI_DECL_PROD(f16)
BRI_DECL_PROD(f16h)
#undef BRI_DECL_PROD
hipError_t apply_recompute(const Geom &g, int up, int sp, const void *U, const void *in, void *out,
                           double diag, int nrhs, bool dag, hipStream_t st);

// wilson.hip: the Wilson comparison operator from SoA links (prec 0 = FP64, 1 = FP32)
hipError_t apply_wilson(const Geom &g, int prec, const void *U, const void *in, void *out, double diag,
                        int nrhs, bool dag, hipStream_t st);

// build.hip: the FP64 40-offset store (the fused build), and its conversion
// to another store
hipError_t build_w40_f64(const Geom &g, const double2 *U, double2 *W40, hipStream_t st);
hipError_t convert_w40(const Geom &g, const double2 *W40, void *W, int wp, int noff, hipStream_t st);
// all transporters of a site in one kernel (no FP64 stage in HBM), into the
// store of precision wp with 40 or 80 offsets
hipError_t build_fused(const Geom &g, const double2 *U, void *W, int wp, int noff, hipStream_t st);

// mfma.hip: the site-major FP16 store of the matrix-core apply (V x 2880 B
// from a 40- or 80-offset store of precision wp), per-right-hand-side bounds
// of an FP32 SoA field, and the apply itself (FP32 site-major fields
// [V][nrhs][12], 12 right-hand sides per workgroup; bound2 per right-hand
// side with stride bstride; tlen <= 0 picks the t-chunk)
hipError_t pack_w_mfma(const Geom &g, const void *W, int wp, int noff, void *Wm, hipStream_t st);
hipError_t spinor_bound2(const Geom &g, int nrhs, const float2 *in, double *bound2, hipStream_t st);
// SoA [nrhs][12][V] <-> site-major [V][nrhs][12] FP32 spinors; to_sites with
// bound2 != nullptr also writes the per-right-hand-side bounds
hipError_t spinor_sites(const Geom &g, int nrhs, const float2 *src, float2 *dst, bool to_sites, double *bound2,
                        hipStream_t st);
hipError_t apply_mfma(const Geom &g, const void *Wm, const float2 *in, float2 *out, int nrhs, double diag,
                      const double *table, bool dag, const double *bound2, int bstride, int tlen, hipStream_t st,
                      double *nrm = nullptr);
// workgroups per block of 12 right-hand sides of apply_mfma (tlen as there):
// with nrm != nullptr the apply also writes, per right-hand side r and such
// workgroup i, the partial |out|^2 of its sites at nrm[2 (r n + i)] (and 0 at
// the odd index), n being this count, for dot_finish
long long mfma_workgroups(const Geom &g, int tlen);

// production.hip
hipError_t project_su3_soa(const double2 *A, double2 *Y, int64_t n, hipStream_t st);
hipError_t project_w40(const Geom &g, double2 *W40, hipStream_t st);
hipError_t ape_smear(const Geom &g, const double2 *U, double2 *Vout, double alpha, hipStream_t st);
hipError_t build_clover(const Geom &g, const double2 *U, void *C, int cp, double csw, hipStream_t st);
hipError_t convert_w40_rows2(const Geom &g, const double2 *W40, void *W, int wp, int noff, hipStream_t st);

// pack.hip
hipError_t pack_links(const Geom &g, const double2 *canon, void *soa, int p, hipStream_t st);
hipError_t pack_spinor(const Geom &g, int nrhs, const double2 *canon, void *soa, int p,
                       hipStream_t st);
hipError_t unpack_spinor(const Geom &g, int nrhs, const void *soa, int p, double2 *canon,
                         hipStream_t st);
hipError_t unpack_links(const Geom &g, const void *soa, int p, double2 *canon, hipStream_t st);

}  // namespace bri
