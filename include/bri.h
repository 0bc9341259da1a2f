/*
 * bri.h - C ABI of the MI355X (gfx950) Brillouin Dirac operator library.
 *
 * The operator is the "Brillouin operator" of Durr & Koutsou,
 * arXiv:1012.3615, Eq. def_pref with lattice spacing a = 1; the core entry
 * points apply it with c_SW = 0 and path-averaged transporters, the
 * production-operator section at the end adds the SU(3) back-projection, the
 * APE smearing and the clover term of the paper's Sec. 5:
 *
 *   D = sum_mu gamma_mu nabla^iso_mu - (1/2) Lap^bri + m,
 *
 * both stencils living on the 81 points x + n, n in {-1,0,1}^4 (App. C),
 * made gauge covariant by the transporter W(x, x+n) = average of the link
 * products over all k! shortest lattice paths from x to x+n (Sec. 5.1,
 * averaged, not back-projected).  Per site
 *
 *   (D psi)(x) = (lambda_0 + m) psi(x)
 *              + sum_{n != 0} [lambda_k + rho_k sum_mu n_mu gamma_mu] W(x,x+n) psi(x+n)
 *
 * with k = |n|_1, lambda_k = -2^(4-k)/128 (k >= 1), lambda_0 = 240/128 and
 * rho_k = 4^(4-k)/432 (Tab. rholambda).  Boundary conditions are periodic.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Extents: dims.L[0..3] = (Lx, Ly, Lz, Lt), each >= 2.  The linear site
 *   index is  site = x + Lx*(y + Ly*(z + Lz*t)).
 * - Directions mu = 0..3 are x, y, z, t.  U_mu(x) transports from x+mu to x,
 *   i.e. it multiplies psi(x+mu) (the Wilson-operator orientation, Sec. 1).
 * - Gamma matrices: Hermitian chiral basis
 *     gamma_{x,y,z} = [[0, -i sigma_k], [i sigma_k, 0]], gamma_t = [[0,1],[1,0]],
 *     gamma_5 = gamma_x gamma_y gamma_z gamma_t = diag(1,1,-1,-1).
 * - Canonical (user) layouts, complex128 = two doubles (re, im):
 *     links   U[mu][site][a][b]            (4 * V * 9 complex)
 *     spinors psi[rhs][site][spin][colour] (nrhs * V * 12 complex)
 * - Internal structure-of-arrays (SoA) layouts, one complex scalar per
 *   element, site index fastest ("planes" of V complex numbers):
 *     links        [mu][9][V]          element e = 3*a + b
 *     spinors      [rhs][12][V]        component = 3*spin + colour
 *     transporters [n_offsets][9][V]
 *   The complex scalar is double2 (BRI_F64), float2 (BRI_F32) or two IEEE
 *   binary16 halves (BRI_F16).  Casts to narrower types round to nearest even.
 * - Offsets n are numbered i = (nx+1) + 3(ny+1) + 9(nz+1) + 27(nt+1) in 0..80;
 *   i = 40 is n = 0.  With n_offsets = 80, plane j holds offset i = j (j < 40)
 *   or i = j+1 (j >= 40).  With n_offsets = 40, plane c holds the offset
 *   i = 41 + c (the offsets whose last non-zero component is +1) and the other
 *   40 are recovered from W(x, x-n) = W(x-n, x)^dag.
 * - All pointers are DEVICE pointers owned by the caller, unless a comment
 *   says "host".  The library never allocates or frees device memory; scratch
 *   is passed in as a workspace whose size the *_workspace_bytes query gives.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   calls are asynchronous on it, except bri_solve_cgne, which synchronises
 *   the stream to read convergence data and returns after completion.
 * - Errors: every call returns a bri_status; nothing throws or aborts across
 *   the ABI.  BRI_E_ARG for null / misaligned (16-byte) pointers, bad sizes,
 *   unsupported enum values and in == out aliasing; BRI_E_HIP for HIP runtime
 *   failures; bri_last_error() then returns a message (thread-local, valid
 *   until the next bri_* call on the same thread).
 */
#ifndef BRI_H
#define BRI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { int32_t L[4]; } bri_dims;

typedef enum { BRI_F64 = 0, BRI_F32 = 1, BRI_F16 = 2 } bri_prec;
typedef enum { BRI_STORED = 0, BRI_RECOMPUTE = 1 } bri_variant;
typedef enum {
    BRI_OK = 0,
    BRI_E_ARG = -1,
    BRI_E_UNSUPPORTED = -2,
    BRI_E_HIP = -3,
    BRI_E_NOCONV = -4,
    BRI_E_WORKSPACE = -5
} bri_status;

/* Message for the last failing call on this thread ("" if none). */
const char *bri_last_error(void);
/* ABI revision of this header (incremented on incompatible change; 3 added
 * the coefficient table to bri_operator and to the gradient calls, 5
 * replaced the per-precision kernel choice by per-shape configurations, 6
 * added the matrix-core apply, its site-major spinor conversions and
 * bri_solve_params.inner_mfma).  bri_abi_version() returns the
 * revision the library was built with; a caller compares it to
 * BRI_ABI_VERSION. */
#define BRI_ABI_VERSION 6
int32_t bri_abi_version(void);

/* ---- sizes (bytes) of the SoA buffers ----------------------------------- */
size_t bri_spinor_bytes(bri_dims d, bri_prec p, int32_t nrhs);
size_t bri_links_bytes(bri_dims d, bri_prec p);
size_t bri_transporter_bytes(bri_dims d, bri_prec p, int32_t n_offsets);

/* ---- layout conversion (canonical complex128 <-> SoA) --------------------
 * Links are the input of the transporter construction (Sec. 5.1; the gauge
 * field U_mu(x) of Eq. def_pref).  p selects the SoA precision; U_soa must
 * hold bri_links_bytes(d, p).  psi_canon/psi_soa hold nrhs fields. */
bri_status bri_pack_links(bri_dims d, const double *U_canon, void *U_soa, bri_prec p, void *stream);
bri_status bri_pack_spinor(bri_dims d, int32_t nrhs, const double *psi_canon, void *psi_soa,
                           bri_prec p, void *stream);
bri_status bri_unpack_spinor(bri_dims d, int32_t nrhs, const void *psi_soa, bri_prec p,
                             double *psi_canon, void *stream);
/* SoA links (or a link-shaped gradient) back to the canonical layout. */
bri_status bri_unpack_links(bri_dims d, const void *U_soa, bri_prec p, double *U_canon,
                            void *stream);

/* ---- transporter construction (Sec. 5.1) ---------------------------------
 * W(x, x+n) for n_offsets = 80 (all) or 40 (hermitian half) offsets, built in
 * FP64 from FP64 SoA links and stored in w_prec.  The k-hop transporters are
 * obtained in hop order from the (k-1)-hop ones at the same site,
 *   W(x, x+n) = (1/k) sum_{mu in supp n} W(x, x+n-s_mu mu) V_mu(x+n-s_mu mu),
 * V_mu(y) = U_mu(y) for s_mu = +1 and U_mu(y-mu)^dag for s_mu = -1, which is
 * the average over all k! paths.  All 80 transporters of a site are built in
 * one kernel, each once, in FP64, and cast to w_prec on store; no scratch is
 * needed: bri_build_workspace_bytes returns 0 and work may be NULL (the
 * argument is kept for the SU(3) forms of bri_build_transporters_ex). */
size_t bri_build_workspace_bytes(bri_dims d, bri_prec w_prec, int32_t n_offsets);
bri_status bri_build_transporters(bri_dims d, const double *U_soa, void *W, bri_prec w_prec,
                                  int32_t n_offsets, void *work, size_t work_bytes, void *stream);

/* ---- operator application (Eq. def_pref, c_SW = 0) -----------------------
 * out = D in (bri_apply) or out = D^dag in (bri_apply_dag) for nrhs fields.
 * variant BRI_STORED:    W_or_U = transporters (w_prec, n_offsets = 40|80).
 * variant BRI_RECOMPUTE: W_or_U = SoA links in w_prec (F64 or F32), the
 *                        transporters are rebuilt on the fly; n_offsets ignored.
 * Spinor precision s_prec: F64 (needs w_prec F64), F32 (w_prec F32 or F16),
 * or F16 (w_prec F16).  Accumulation is FP64 for F64 and FP32 otherwise.
 * D^dag = gamma5 D gamma5 (Sec. 1), i.e. D with rho_k -> -rho_k.
 * nrhs >= 1 fields are processed in one fused launch that reads each
 * transporter once per group of right-hand sides.  in and out must not
 * overlap. */
bri_status bri_apply(bri_dims d, bri_variant v, const void *W_or_U, bri_prec w_prec,
                     int32_t n_offsets, bri_prec s_prec, double mass, const void *in, void *out,
                     int32_t nrhs, void *stream);
bri_status bri_apply_dag(bri_dims d, bri_variant v, const void *W_or_U, bri_prec w_prec,
                         int32_t n_offsets, bri_prec s_prec, double mass, const void *in,
                         void *out, int32_t nrhs, void *stream);

/* ---- the Wilson comparison operator (Sec. 1; Wilson column of Tab. rholambda)
 * out = D_W in (dagger = 0) or D_W^dag in (dagger = 1), with
 *   (D_W psi)(x) = (4 + m) psi(x) - 1/2 sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                            + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)]
 * and D_W^dag the same with gamma_mu -> -gamma_mu (the gamma matrices of the
 * Brillouin apply).  U = SoA links [mu][9][V] and in/out = SoA spinors
 * [rhs][12][V], all device memory in prec (F64 or F32; F16 gives
 * BRI_E_UNSUPPORTED); accumulation in prec.  It is the 9-point operator the
 * paper compares the Brillouin operator with; the same operator is the Wilson
 * row of the generic class (bri_operator.coef), which reads all 80
 * transporters.  nrhs in [1, 65535]; in and out must not overlap; pointers
 * 16-byte aligned (BRI_E_ARG otherwise).  Enqueued on stream, asynchronous. */
bri_status bri_apply_wilson(bri_dims d, const void *U_soa, bri_prec prec, double mass, const void *in,
                            void *out, int32_t nrhs, int32_t dagger, void *stream);

/* ---- matrix-core apply for blocks of right-hand sides (Eq. def_pref)
 * The operator of bri_apply (80 offsets, c_SW = 0, any member of the generic
 * class of Sec. 8) evaluated with the matrix cores: the spin matrix
 * lambda_k + rho_k sum_mu n_mu gamma_mu is split into five colour sums,
 *   X_0 = sum_n lambda_k W(x,x+n) psi(x+n),  X_mu = sum_n rho_k n_mu W(x,x+n) psi(x+n),
 * and D psi = (lambda_0 + m) psi + X_0 + sum_mu gamma_mu X_mu.  The five sums
 * of a site are one matrix product with FP16 operands (transporters times
 * lambda_k or rho_k normalised to at most 1; psi scaled by a power of two per
 * right-hand side) and FP32 accumulation; the gamma matrices, the diagonal term
 * (from psi in FP32) and the output are FP32.  Relative error per output
 * component is about 1e-3 of the field's scale: an operator for inner solves
 * and other FP16-transporter work, not a replacement of the FP32 apply.
 *
 * bri_pack_w_mfma: the transporter store of this apply, written from a store
 *   of bri_build_transporters (W: [n_offsets][9][V] complex in w_prec,
 *   n_offsets 40 or 80).  W_mfma: device, BRI_MFMA_W_BYTES_PER_SITE bytes per
 *   site, caller-allocated: per site the 80 offsets in the order of the
 *   80-offset store, each a row-major 3x3 matrix of FP16 complex numbers
 *   (real part first).  W and W_mfma must not overlap.
 * Spinors of this apply are site-major: [V][nrhs][12] FP32 complex (one
 *   contiguous record of all right-hand sides per site); bri_spinor_to_sites
 *   and bri_spinor_from_sites convert from and to the SoA layout
 *   [nrhs][12][V] of the other entry points.
 * bri_spinor_to_sites: psi (SoA) -> psi_sites (site-major); with bound2 !=
 *   NULL also bound2[r] = (largest |real or imaginary part| of psi_r)^2
 *   (device doubles).  bri_spinor_from_sites: the inverse.  FP32; the two
 *   fields must not overlap.
 * bri_spinor_bound2: the same bounds from an SoA field (FP32 [nrhs][12][V]).
 * bri_apply_mfma: out = D in (dagger = 0) or D^dag in (dagger = 1); in, out
 *   FP32 site-major [V][nrhs][12] complex, nrhs in [1, 65535] (blocks of 12
 *   per workgroup; a partial block pads with zeros); bound2: device, nrhs doubles,
 *   bound2[r] >= the largest squared real or imaginary part of in_r
 *   (bri_spinor_to_sites gives it, or a squared 2-norm: any upper bound
 *   works; the looser it is, the closer small components come to the FP16
 *   subnormal range); coef: NULL for the Brillouin column of Tab. rholambda
 *   or 9 host doubles lambda_0..4, rho_1..4.  in and out must not overlap;
 *   pointers 16-byte aligned (BRI_E_ARG otherwise); a t plane of the fields
 *   (V / Lt sites x nrhs x 96 B) must stay below 4 GiB (BRI_E_UNSUPPORTED
 *   otherwise).  Enqueued on stream, asynchronous; no allocation. */
#define BRI_MFMA_W_BYTES_PER_SITE 2880
bri_status bri_pack_w_mfma(bri_dims d, const void *W, bri_prec w_prec, int32_t n_offsets, void *W_mfma,
                           void *stream);
bri_status bri_spinor_bound2(bri_dims d, int32_t nrhs, const float *psi, double *bound2, void *stream);
bri_status bri_spinor_to_sites(bri_dims d, int32_t nrhs, const float *psi, float *psi_sites, double *bound2,
                               void *stream);
bri_status bri_spinor_from_sites(bri_dims d, int32_t nrhs, const float *psi_sites, float *psi, void *stream);
bri_status bri_apply_mfma(bri_dims d, const void *W_mfma, double mass, const float *in, float *out,
                          int32_t nrhs, int32_t dagger, const double *coef, const double *bound2,
                          void *stream);

/* Launch configuration of the stored apply, per shape.  A shape is
 * (extents, w_prec, s_prec, n_offsets, nrhs).  Kernel codes:
 *   1  built-in selection (the default for every shape): LDS tiles whose
 *      shape follows Lx; each workgroup stages the spinor of its x-y tile
 *      plus a one-site halo layer by layer in LDS.  For Lx > 16 a 32x8 tile
 *      (24x8 or 48x4 when Lx is a multiple of 24 or 48 but not of 32; 32x16
 *      for FP32 or FP64 transporters (80 offsets) with spinors of the same
 *      precision and one right-hand side, when Lx is a multiple of 32 and Ly
 *      of 16) with the next transporter prefetched and each layer's offsets
 *      unrolled; for Lx <= 16 a 16x16 tile (one right-hand side per thread;
 *      16x4 with unrolled offsets for FP32 when Lx = 16) or 16x8 (several);
 *   2..5   LDS tiles of 32x8, 16x16, 64x4 or 16x8 sites;
 *   6, 7   tiles 32x8, 16x16 with transporter prefetch;
 *   8      tile 32x8 with prefetch and each layer's offsets unrolled;
 *   9, 10  tiles 32x8, 16x8 with the offsets unrolled, no prefetch;
 *   11, 12 tiles 24x8, 48x4 with prefetch and unrolled offsets;
 *   13, 14 tiles 32x16, 16x4 with prefetch and unrolled offsets, one
 *          right-hand side per thread;
 *   0      direct neighbour gathers through the caches.
 * rhs_per_thread (1, 2, 3, 4, 6 or 12; the built-in value is 2) is clamped to
 * what the kernel holds: tiles 1-4 right-hand sides per thread (16x16, 64x4,
 * 32x16, 16x4: 1; 32x8, 24x8 and 48x4 with prefetch: 1, 2), the gather form
 * any of the six values.  All kernels add the 81 terms of a site in the same
 * order (offset index 0..80), so their results agree bit for bit.
 *
 * bri_set_apply_config installs (kernel, rhs_per_thread) for exactly the
 * given shape: every later apply of that shape (bri_apply, bri_apply_dag,
 * bri_apply_op without the two-row form or clover term, and the applies
 * inside the solver, Lanczos and the sign function) launches it, and every
 * other shape keeps its own entry or the built-in selection.  kernel = -1
 * removes the entry.  At most 256 shapes carry an entry (BRI_E_ARG beyond).
 * The table is host-side library state shared by all threads, guarded by a
 * lock.  This is what the autotuner (paper_1012_3615_amd/autotune.py) uses. */
bri_status bri_set_apply_config(bri_dims d, bri_prec w_prec, bri_prec s_prec, int32_t n_offsets, int32_t nrhs,
                                int32_t kernel, int32_t rhs_per_thread);
/* The configuration an apply of this shape launches: the kernel code (code 1
 * resolved to the tile it picks, so never 1) and the right-hand sides per
 * thread after clamping.  Outputs are host pointers. */
bri_status bri_get_apply_config(bri_dims d, bri_prec w_prec, bri_prec s_prec, int32_t n_offsets, int32_t nrhs,
                                int32_t *kernel, int32_t *rhs_per_thread);
/* Remove every installed configuration (all shapes back to the built-in
 * selection). */
void bri_clear_apply_configs(void);

/* ---- solver: CG on the normal equations D^dag D x = D^dag b ----------------
 * The paper inverts D for propagators (Sec. 6.4, BiCGstab to 1e-7); here the
 * solver is CGNE, stopped on the true relative residual ||b - D x||/||b||
 * computed in FP64 for every right-hand side.
 * With dagger = 1 the same machinery solves D^dag x = b (D and D^dag swap).
 * inner_prec == BRI_F64: plain FP64 CGNE with W_hi (FP64 transporters).
 * inner_prec == BRI_F32 / BRI_F16: defect correction; the outer loop forms
 * r = b - D x in FP64 with W_hi, the inner CGNE solves D e = r in FP32
 * arithmetic with W_lo (F32 or F16 transporters, same n_offsets) to relative
 * inner_tol (or to max(inner_tol, tol / (2 r)) with r the worst relative
 * true residual left, so the last cycle does not overshoot), and x += e.  b and x are FP64 SoA spinors ([rhs][12][V]); x holds
 * the initial guess on entry and the solution on exit.  All right-hand sides
 * iterate together (one fused apply per iteration) with their own scalars;
 * converged columns are frozen.  Reductions are deterministic FP64. */
typedef struct {
    double tol;              /* target true relative residual, per RHS          */
    double inner_tol;        /* inner relative residual for defect correction    */
    int32_t max_iter;        /* cap on inner CG iterations (summed over outers)  */
    int32_t max_outer;       /* cap on defect-correction cycles                  */
    int32_t n_offsets;       /* 40 or 80, for both W_hi and W_lo                 */
    bri_prec inner_prec;     /* F64 (plain), F32 or F16 (transporters of W_lo)   */
    int32_t check_every;     /* iterations between host convergence checks (>=1) */
    int32_t use_initial_guess; /* 0: x is zeroed first                           */
    int32_t dagger;          /* 1: solve D^dag x = b (CG on D D^dag) instead     */
    int32_t inner_mfma;      /* 1: inner applies on the matrix cores              */
                             /*    (bri_apply_mfma, through site-major copies in  */
                             /*    the workspace): inner_prec BRI_F16 and W_lo    */
                             /*    from bri_pack_w_mfma                            */
} bri_solve_params;

#define BRI_MAX_RHS 64
typedef struct {
    int32_t iterations;      /* inner CG iterations (all cycles)                 */
    int32_t outer;           /* defect-correction cycles (1 for plain FP64)      */
    int32_t applies;         /* operator applications (D or D^dag), per RHS block*/
    int32_t converged;       /* 1 if every RHS met tol                           */
    double true_residual[BRI_MAX_RHS]; /* final ||b - D x||/||b|| per RHS        */
} bri_solve_stats;

size_t bri_solve_workspace_bytes(bri_dims d, const bri_solve_params *p, int32_t nrhs);
bri_status bri_solve_cgne(bri_dims d, const bri_solve_params *p, const void *W_hi,
                          const void *W_lo, double mass, const double *b, double *x,
                          int32_t nrhs, void *work, size_t work_bytes,
                          bri_solve_stats *stats /* host */, void *stream);

/* Allocation-free form of bri_solve_cgne, for callers that cannot allocate
 * device memory (serving loops and harnesses that forbid hipMalloc between
 * set-up and tear-down).  Same arguments and results as bri_solve_cgne
 * without the workspace: the library keeps a static device array of
 * BRI_SOLVE_NOALLOC_MAX_BYTES (128 MiB) per device, present from the time the
 * library's code is loaded on that device until the process ends, and calls
 * no allocating routine.  A solve whose bri_solve_workspace_bytes exceeds
 * that size is rejected with BRI_E_WORKSPACE before any device work (at
 * 128 MiB: plain FP64 with one right-hand side up to ~99k sites, FP32 inner
 * solves up to ~155k sites, 16^3 x 32 included).  The array is shared by
 * every call on the device: calls on one device are serialised by a lock held
 * until the call's work on `stream` has finished, so they never overlap; the
 * array keeps the last call's contents, and nothing in it needs to start at
 * zero (the solver writes each buffer before reading it).  `stream` must
 * belong to the current device. */
#define BRI_SOLVE_NOALLOC_MAX_BYTES (128u << 20)
bri_status bri_solve_cgne_noalloc(bri_dims d, const bri_solve_params *p, const void *W_hi,
                                  const void *W_lo, double mass, const double *b, double *x,
                                  int32_t nrhs, bri_solve_stats *stats /* host */, void *stream);

/* ---- gradient with respect to the links -----------------------------------
 * For S = Re sum_rhs <chi, D psi> (FP64 SoA spinors, nrhs fields each) writes
 * gradU = scale * (dS/dRe U + i dS/dIm U) in the FP64 SoA link layout, treating link
 * entries as unconstrained complex numbers, through the path averaging of
 * the transporters.  The transporters are rebuilt from U inside the call
 * (not stored across calls).  The psi gradient is D^dag chi (bri_apply_dag).
 * coef: NULL for the Brillouin operator, or the nine host doubles of another
 * member of the generic class of Sec. 8 (as in bri_operator; BRI_E_ARG if
 * not finite).  work: bri_grad_workspace_bytes(d). */
size_t bri_grad_workspace_bytes(bri_dims d);
bri_status bri_grad_links(bri_dims d, const double *U_soa, const double *chi, const double *psi,
                          int32_t nrhs, double scale, const double *coef, double *gradU, void *work,
                          size_t work_bytes, void *stream);
/* The same with the FP64 40-offset transporters of U given (built by
 * bri_build_transporters(d, U_soa, W40, BRI_F64, 40, ...) in the same
 * backward pass, e.g. for the psi gradient), so that they are built once.
 * work: bri_grad_workspace_bytes_w(d). */
size_t bri_grad_workspace_bytes_w(bri_dims d);
bri_status bri_grad_links_w(bri_dims d, const double *U_soa, const double *W40, const double *chi,
                            const double *psi, int32_t nrhs, double scale, const double *coef, double *gradU,
                            void *work, size_t work_bytes, void *stream);

/* ---- production operator (Sec. 5) -----------------------------------------
 * The operator of the paper's quenched tests uses (i) links after one APE
 * smearing step (Eq. def_ape), (ii) transporters back-projected to SU(3)
 * after the path averaging (Sec. 5.1) with the projection of Sec. 5.2, and
 * (iii) the clover term of Eq. def_pref,
 *     -(c_SW/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu},  c_SW = 1 at tree level (Sec. 5.3),
 * with sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu] and F_{mu nu} the Hermitian
 * clover-leaf field strength (Q - Q^dag)/(8i), Q the sum of the four
 * plaquettes at x in the (mu, nu) plane, made traceless.  D^dag is again D
 * with rho_k -> -rho_k (the clover term is Hermitian and commutes with
 * gamma5).  All construction steps compute in FP64. */

/* Nearest SU(3) matrix in the Frobenius norm (Sec. 5.2, Eq. proj_SU) for n
 * FP64 matrices in the SoA layout [9][n] (element e = 3a + b, one complex
 * double each): A = U S V^dag from the eigen-decomposition of A^dag A, then
 * the phases D that maximise Re tr(A^dag U D V^dag) under det = 1, found by a
 * scan of spacing pi/3 over two free phases and Newton refinement; the result
 * is U D V^dag.  Y may equal A (in place); other overlap is BRI_E_ARG.  The
 * matrices must be non-singular.  n = 0 is a no-op. */
bri_status bri_project_su3(int64_t n, const double *A, double *Y, void *stream);

/* One APE step (Eq. def_ape) on FP64 SoA links [mu][9][V]:
 *   V_mu(x) = P_SU(3){ (1-alpha) 1 + (alpha/6) sum_{+-nu != mu}
 *             U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag U_mu(x)^dag } U_mu(x),
 * where the link of a -nu step from y is U_nu(y-nu)^dag.  The paper uses
 * alpha = 0.72.  U_soa and V_soa must not overlap. */
bri_status bri_ape_smear(bri_dims d, const double *U_soa, double *V_soa, double alpha, void *stream);

/* Storage form of the transporters. */
typedef enum {
    BRI_W_AVERAGE = 0,  /* path average (as bri_build_transporters), 9 complex each          */
    BRI_W_SU3 = 1,      /* back-projected to SU(3), 9 complex each                             */
    BRI_W_SU3_2ROW = 2  /* back-projected, rows 0 and 1 only (6 complex each, layout
                           [n_offsets][6][V]); the apply rebuilds row 2 = conj(row0 x row1) */
} bri_wform;

/* Transporters in the given form.  For the SU(3) forms the 2-, 3- and 4-hop
 * path averages are built in FP64 exactly as by bri_build_transporters, then
 * each is projected (the 1-hop transporters are the links, already in SU(3)),
 * then converted to w_prec.  work: bri_build_workspace_bytes_ex bytes. */
size_t bri_transporter_bytes_ex(bri_dims d, bri_prec p, int32_t n_offsets, bri_wform form);
size_t bri_build_workspace_bytes_ex(bri_dims d, bri_prec p, int32_t n_offsets, bri_wform form);
bri_status bri_build_transporters_ex(bri_dims d, const double *U_soa, void *W, bri_prec w_prec,
                                     int32_t n_offsets, bri_wform form, void *work, size_t work_bytes,
                                     void *stream);

/* Clover term per site from FP64 SoA links, stored in c_prec.  In the chiral
 * basis it is block diagonal: one Hermitian 6x6 block on spins (0,1) and one
 * on spins (2,3), local index 3*spin' + colour.  Layout [2][18][V] complex:
 * planes 0..2 hold the real diagonal in pairs (M00, M11), (M22, M33),
 * (M44, M55) as (re, im); planes 3..17 hold M_ij for i < j, row by row. */
size_t bri_clover_bytes(bri_dims d, bri_prec p);
bri_status bri_build_clover(bri_dims d, const double *U_soa, double csw, void *C, bri_prec c_prec,
                            void *stream);

/* An operator: transporters, their form and, optionally, the clover term and
 * the coefficients of another member of the generic ultralocal class of
 * Sec. 8,
 *   D(x,y) = sum_mu gamma_mu rho_mu(x-y) + lambda(x-y),
 * where an offset n with k non-zero components carries lambda(n) = lambda_k
 * and rho_mu(n) = rho_k n_mu (each of the 80 offsets counted once), made
 * covariant with the same transporters:
 *   (D psi)(x) = (lambda_0 + m) psi(x)
 *     + sum_{n != 0} [lambda_k + rho_k sum_mu n_mu gamma_mu] W(x,x+n) psi(x+n).
 * coef = {lambda_0, lambda_1, lambda_2, lambda_3, lambda_4, rho_1, rho_2,
 * rho_3, rho_4} (Tab. rholambda lists the Wilson, hypercube and Brillouin
 * columns); NULL is the Brillouin column.  The nine doubles are host memory,
 * owned by the caller and read on every call that uses the operator; they
 * must be finite (BRI_E_ARG otherwise).  The dagger of every member is the
 * same stencil with rho -> -rho (lambda even, rho odd in n). */
typedef struct {
    const void *W;       /* transporters (bri_build_transporters or _ex)                     */
    bri_prec w_prec;
    int32_t n_offsets;   /* 40 or 80; 80 for BRI_W_SU3_2ROW or with a clover term           */
    bri_wform w_form;
    const void *clover;  /* bri_build_clover output in the spinor precision; NULL: c_SW = 0  */
    const double *coef;  /* 9 host doubles of the generic class; NULL: Brillouin            */
} bri_operator;

/* out = D in (dagger = 0) or D^dag in (dagger = 1) for the stored variant,
 * with the spinor and precision rules of bri_apply.  The two-row form and the
 * clover term use the default LDS-tile kernel (one or two right-hand sides
 * per thread); otherwise this is bri_apply / bri_apply_dag (same kernel
 * selection), with the operator's coefficient table if it has one. */
bri_status bri_apply_op(bri_dims d, const bri_operator *op, bri_prec s_prec, double mass,
                        const void *in, void *out, int32_t nrhs, int32_t dagger, void *stream);

/* bri_solve_cgne for a general operator: op_hi in FP64 (w_prec F64, clover
 * F64) for the outer residual and the plain solver; op_lo for the inner
 * solve of defect correction (w_prec = p->inner_prec, clover F32), the same
 * operator at lower precision (a different coefficient table, or a clover
 * term on one side only, is BRI_E_ARG).  p->n_offsets is ignored (each operator
 * carries its own).  Workspace: bri_solve_workspace_bytes. */
bri_status bri_solve_cgne_op(bri_dims d, const bri_solve_params *p, const bri_operator *op_hi,
                             const bri_operator *op_lo, double mass, const double *b, double *x,
                             int32_t nrhs, void *work, size_t work_bytes, bri_solve_stats *stats,
                             void *stream);

/* ---- overlap operator with the Brillouin kernel (Sec. 7) ------------------
 *   D_ov,m = (1 - m/(2 rho)) rho [1 + gamma5 sign(H)] + m,   H = gamma5 D(-rho),
 * (Eqs. def_over and def_mass, a = 1, 0 < rho < 2), D(-rho) the kernel operator
 * `op` at mass -rho.  H is Hermitian and H^2 = D^dag D.  All fields are FP64
 * SoA spinors and `op` must have FP64 transporters (and an FP64 clover term if
 * any).  The spectrum of A = D^dag D is estimated by Lanczos (the Ritz values
 * of Sec. 7.3); sign(H) = H (H^2)^{-1/2} is evaluated as gamma5 D p(A) with p
 * the Chebyshev interpolant of x^{-1/2} on [lo, hi], which must contain the
 * spectrum of A (outside the optional low modes). */

/* k Lanczos steps on A = D^dag D (op at `mass`) from the FP64 field v0 (one
 * field, need not be normalised).  Host outputs: alpha[0..k-1] (diagonal of
 * the tridiagonal T), beta[0..k-1] with beta[0] = |v0| and beta[j] the
 * off-diagonal (j, j-1) element; *k_done = steps performed (fewer than k only
 * if an invariant subspace was found).  basis: NULL, or caller memory for k
 * fields ([k][12][V]) in which the Lanczos vectors are kept; each new vector
 * is then re-orthogonalised against all kept ones (two classical Gram-Schmidt
 * passes, each one batched dot launch and one fused update), otherwise only
 * the three-term recurrence is used.  Synchronises the stream twice per step
 * (alpha and beta go to the host).  Workspace: bri_lanczos_workspace_bytes(d, k). */
size_t bri_lanczos_workspace_bytes(bri_dims d, int32_t k);
bri_status bri_lanczos(bri_dims d, const bri_operator *op, double mass, int32_t k, const double *v0,
                       double *alpha, double *beta, double *basis, int32_t *k_done, void *work,
                       size_t work_bytes, void *stream);

/* Ritz values: the eigenvalues of the k x k symmetric tridiagonal matrix
 * (alpha, beta[1..k-1]) in ascending order, by bisection on Sturm counts
 * (host only, no device work).  With filter = 1, numerically equal values
 * (relative 1e-10) are kept once and a simple value that is also an eigenvalue
 * of the matrix without its first row and column is dropped as spurious
 * (the Cullum-Willoughby test for Lanczos without re-orthogonalisation).
 * out: host array of k doubles; *n_out: number written. */
bri_status bri_ritz_values(int32_t k, const double *alpha, const double *beta, int32_t filter, double *out,
                           int32_t *n_out);

/* The n_low eigenmodes of H = gamma5 D (op at `mass`) of smallest |eigenvalue|:
 * k re-orthogonalised Lanczos steps on A = H^2 from v0 (basis: caller memory
 * for k fields), the eigenvectors of the tridiagonal for its n_low smallest
 * eigenvalues (bisection, inverse iteration), the Ritz vectors X_i, then
 * Rayleigh-Ritz for H on span{X}.  Outputs: vecs [n_low][12][V] orthonormal
 * (FP64), evals (host, signed eigenvalues of H by increasing |.|), resid
 * (host, |H v_i - evals_i v_i|).  The modes are exact only as far as the
 * residuals say; the cost is O(k^2) field reads for the re-orthogonalisation
 * and k fields of basis memory (24^3 x 48, k = 160: 20 GB, about 2 s on one
 * MI355X).  Workspace:
 * bri_lowmodes_workspace_bytes(d, k, n_low). */
size_t bri_lowmodes_workspace_bytes(bri_dims d, int32_t k, int32_t n_low);
bri_status bri_overlap_lowmodes(bri_dims d, const bri_operator *op, double mass, int32_t k, const double *v0,
                                int32_t n_low, double *basis, double *vecs, double *evals, double *resid,
                                void *work, size_t work_bytes, void *stream);

/* out = sign(H) psi for nrhs FP64 fields, H = gamma5 D (op at `mass`):
 *   sign(H) psi = sum_i s_i v_i <v_i, psi> + gamma5 D p(A) (psi - sum_i v_i <v_i, psi>),
 * with n_low >= 0 orthonormal eigenvectors v_i of H (low_vecs, FP64
 * [n_low][12][V]) and their eigenvalues (low_evals, host; s_i = their sign),
 * and p of the given degree on [lo, hi].  Cost: 2*degree + 3 applications of D.
 * *approx_err (host, may be NULL): max over [lo, hi] of |1 - sqrt(x) p(x)|.
 * psi and out must not overlap.  Workspace: bri_sign_workspace_bytes(d, nrhs). */
size_t bri_sign_workspace_bytes(bri_dims d, int32_t nrhs);
/* The error bound *err of the interpolant of the given degree on [lo, hi]
 * (host only), to choose the degree before applying. */
bri_status bri_sign_approx_error(double lo, double hi, int32_t degree, double *err);
bri_status bri_sign_h(bri_dims d, const bri_operator *op, double mass, double lo, double hi, int32_t degree,
                      int32_t n_low, const double *low_vecs, const double *low_evals, const double *psi,
                      double *out, int32_t nrhs, double *approx_err, void *work, size_t work_bytes,
                      void *stream);

/* out = D_ov,m psi with sign(H) from bri_sign_h at mass -rho (same arguments). */
bri_status bri_overlap_apply(bri_dims d, const bri_operator *op, double rho, double m, double lo, double hi,
                             int32_t degree, int32_t n_low, const double *low_vecs, const double *low_evals,
                             const double *psi, double *out, int32_t nrhs, double *approx_err, void *work,
                             size_t work_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* BRI_H */
