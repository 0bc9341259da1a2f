// CG on the normal equations D^dag D x = D^dag b, with FP64 defect
// correction around a lower-precision inner solve.
//
// Outer loop (FP64, W_hi):  r = b - D x;  stop when |r_i|/|b_i| <= tol for
//   every right-hand side i;  otherwise solve D e = r/|r| approximately and
//   set x += |r| e.  The inner solve reduces its residual by inner_tol, or
//   only by what the final tolerance still needs (times 1/2) when that is less.
// Inner loop (CGNE, FP32 storage with W_lo in FP32 or FP16, or FP64 with
//   W_hi for the plain solver), per right-hand side i:
//     z = D^dag r, p = z, zz = |z|^2
//     repeat: q = D p; alpha = zz/|q|^2; r -= alpha q;
//             z = D^dag r; beta = |z|^2/zz; e += alpha p; p = z + beta p
//   (e is updated in the pass that forms the next p, so p is read once)
//   until |r| <= inner_tol |r_0|.  All right-hand sides share each fused
//   apply; a converged column is frozen on the device (alpha = 0).  The host
//   reads the per-column state every check_every iterations.
// The paper solves with BiCGstab (Sec. 6.4); CGNE is the solver of this
// library, stopped on the FP64 true residual.
#include <cmath>
#include <mutex>
#include <vector>

#include "abi_internal.h"
#include "blas.h"
#include "kernels.h"

namespace bri {
namespace {

__global__ void k_zero(size_t n, float *p) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}
__global__ void k_zero(size_t n, double *p) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
template <typename T>
hipError_t zero(size_t n, T *p, hipStream_t st) {
    size_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)b), dim3(256), 0, st, n, p);
    return hipGetLastError();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t r_hi, dx_hi, e, r, p, q, z, part, red, stv, scale, unscale, total;
};

Layout layout(size_t n, int nrhs, size_t tbytes) {
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align256(bytes);
        return at;
    };
    const size_t hv = n * nrhs * sizeof(double), lv = n * nrhs * tbytes;
    L.r_hi = take(hv);
    L.dx_hi = take(hv);
    L.e = take(lv);
    L.r = take(lv);
    L.p = take(lv);
    L.q = take(lv);
    L.z = take(lv);
    L.part = take((size_t)nrhs * 4096 * 2 * sizeof(double));  // per-workgroup partials (site-major: up to 4096)
    L.red = take((size_t)4 * nrhs * 2 * sizeof(double));
    L.stv = take((size_t)7 * nrhs * sizeof(double));
    L.scale = take((size_t)nrhs * sizeof(double));
    L.unscale = take((size_t)nrhs * sizeof(double));
    L.total = o;
    return L;
}

struct Ctx {
    bri_dims d;
    Geom g;
    size_t n;  // reals per rhs
    int nrhs;
    double mass;
    bool dag;  // solve D^dag x = b
    hipStream_t st;
    char *w;
    Layout L;
};

#define BRI_TRY(expr)                       \
    do {                                    \
        bri_status _s = (expr);             \
        if (_s != BRI_OK) return _s;        \
    } while (0)
#define BRI_HIP(expr, what) BRI_TRY(hip_check((expr), what))

template <typename T>
bri_status norm2(const Ctx &c, const T *a, double *out2, bool sites = false) {
    double *part = (double *)(c.w + c.L.part);
    if (sites) {
        const int nb = site_blocks(c.g.V, c.nrhs);
        BRI_HIP(norm2_sites(c.g.V, c.nrhs, (const float *)a, part, nb, c.st), "norm partials");
        BRI_HIP(dot_finish(c.nrhs, part, nb, out2, c.st), "norm finish");
        return BRI_OK;
    }
    const int nb = dot_blocks(c.n);
    BRI_HIP(dot_partials_t<T>(c.n, c.nrhs, a, a, part, nb, c.st), "norm partials");
    BRI_HIP(dot_finish(c.nrhs, part, nb, out2, c.st), "norm finish");
    return BRI_OK;
}

bri_status fetch(const Ctx &c, const double *dev, double *host, size_t count) {
    BRI_HIP(hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, c.st), "copy to host");
    BRI_HIP(hipStreamSynchronize(c.st), "synchronize");
    return BRI_OK;
}

// inner CGNE on D e = r with e = 0 initially; r holds the right-hand side.
// With the matrix-core operator (op.mfma, T = float) every inner vector is
// site-major [V][nrhs][24], the layout of that apply, and each apply takes
// the squared 2-norm of its input, which the iteration computes anyway, as
// the bound of its components.
template <typename T>
bri_status inner_cgne(const Ctx &c, const OpDesc &op, bri_prec sp, double rel, int max_it, int check_every,
                      int *iters, int *applies) {
    T *e = (T *)(c.w + c.L.e), *r = (T *)(c.w + c.L.r), *p = (T *)(c.w + c.L.p);
    T *q = (T *)(c.w + c.L.q), *z = (T *)(c.w + c.L.z);
    double *part = (double *)(c.w + c.L.part);
    double *qq2 = (double *)(c.w + c.L.red), *rr2 = qq2 + 2 * c.nrhs, *zz2 = rr2 + 2 * c.nrhs;
    double *pp2 = zz2 + 2 * c.nrhs;
    const bool sites = op.mfma;
    const double diag = (op.coef ? op.coef[0] : lam_k(0)) + c.mass;
    // out = D in (or D^dag in) and out2 = |out|^2 per right-hand side; the
    // matrix-core apply forms the norm partials itself when they fit the
    // partial buffer (up to 4096 per right-hand side)
    const long long mwg = sites ? mfma_workgroups(c.g, 0) : 0;
    const bool fused_norm = sites && mwg <= 4096;
    auto apply_norm = [&](const T *in, T *out, bool dag, const double *in2, double *out2) -> bri_status {
        if (sites) {
            BRI_HIP(apply_mfma(c.g, op.W, (const float2 *)in, (float2 *)out, c.nrhs, diag, op.coef, dag, in2, 2, 0,
                               c.st, fused_norm ? part : nullptr),
                    "apply (matrix cores)");
            if (fused_norm) {
                BRI_HIP(dot_finish(c.nrhs, part, (int)mwg, out2, c.st), "norm finish");
                return BRI_OK;
            }
        } else {
            BRI_TRY(apply_op(c.d, op, sp, c.mass, in, out, c.nrhs, c.st, dag));
        }
        return norm2<T>(c, out, out2, sites);
    };
    double *stv = (double *)(c.w + c.L.stv);
    const int nb = sites ? site_blocks(c.g.V, c.nrhs) : dot_blocks(c.n);
    const size_t bytes = c.n * c.nrhs * sizeof(T);

    BRI_HIP(zero(c.n * c.nrhs, e, c.st), "zero");
    BRI_TRY(norm2<T>(c, r, rr2, sites));
    BRI_TRY(apply_norm(r, z, !c.dag, rr2, zz2));
    ++*applies;
    BRI_HIP(cg_init(c.nrhs, stv, rr2, zz2, rel * rel, c.st), "cg init");
    BRI_HIP(hipMemcpyAsync(p, z, bytes, hipMemcpyDeviceToDevice, c.st), "copy");
    if (sites) BRI_HIP(hipMemcpyAsync(pp2, zz2, 2 * c.nrhs * sizeof(double), hipMemcpyDeviceToDevice, c.st), "copy");
    std::vector<double> hs(7 * c.nrhs);
    for (int it = 1; it <= max_it; ++it) {
        BRI_TRY(apply_norm(p, q, c.dag, pp2, qq2));
        BRI_HIP(cg_alpha(c.nrhs, stv, qq2, c.st), "alpha");
        if (sites)
            BRI_HIP(update_r_sites(c.g.V, c.nrhs, stv + 3 * c.nrhs, (float *)r, (const float *)q, part, nb, c.st),
                    "update r");
        else
            BRI_HIP(update_r<T>(c.n, c.nrhs, stv + 3 * c.nrhs, r, q, part, nb, c.st), "update r");
        BRI_HIP(dot_finish(c.nrhs, part, nb, rr2, c.st), "rr finish");
        BRI_TRY(apply_norm(r, z, !c.dag, rr2, zz2));
        BRI_HIP(cg_beta(c.nrhs, stv, rr2, zz2, c.st), "beta");
        // x += alpha p with this iteration's alpha, taken in the pass that
        // also forms the next p
        if (sites) {
            BRI_HIP(update_xp_sites(c.g.V, c.nrhs, stv + 3 * c.nrhs, stv + 4 * c.nrhs, (float *)e, (float *)p,
                                    (const float *)z, part, nb, c.st),
                    "update x,p");
            BRI_HIP(dot_finish(c.nrhs, part, nb, pp2, c.st), "pp finish");
        } else {
            BRI_HIP(update_xp<T>(c.n, c.nrhs, stv + 3 * c.nrhs, stv + 4 * c.nrhs, e, p, z, c.st), "update x,p");
        }
        *applies += 2;
        *iters = it;
        if (it % check_every == 0 || it == max_it) {
            BRI_TRY(fetch(c, stv, hs.data(), hs.size()));
            bool any = false;
            const int R = c.nrhs;
            for (int i = 0; i < R; ++i) {
                if (!std::isfinite(hs[2 * R + i]) || !std::isfinite(hs[i]))
                    return fail(BRI_E_NOCONV, "non-finite residual in the inner solve (rhs %d)", i);
                any = any || hs[5 * R + i] != 0.0;
            }
            if (!any) return BRI_OK;
        }
    }
    return BRI_OK;  // the outer loop decides convergence
}

}  // namespace

// the solver for operators hi (FP64) and lo (inner precision, used when mixed)
static bri_status solve_core(bri_dims d, const bri_solve_params *p, const OpDesc &hi, const OpDesc &lo, double mass,
                      const double *b, double *x, int32_t nrhs, void *work, size_t work_bytes,
                      bri_solve_stats *stats, void *stream) {
    Geom g;
    if (!p || !stats) return fail(BRI_E_ARG, "null params or stats");
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (nrhs < 1 || nrhs > BRI_MAX_RHS) return fail(BRI_E_ARG, "nrhs must be in [1, %d]", BRI_MAX_RHS);
    if (!(p->tol > 0.0) || p->max_iter < 1 || p->max_outer < 1 || p->check_every < 1)
        return fail(BRI_E_ARG, "invalid solver parameters");
    const bool mixed = p->inner_prec != BRI_F64;
    if (mixed && p->inner_prec != BRI_F32 && p->inner_prec != BRI_F16)
        return fail(BRI_E_ARG, "invalid inner precision");
    if (mixed && !(p->inner_tol > 0.0 && p->inner_tol < 1.0))
        return fail(BRI_E_ARG, "inner_tol must be in (0, 1)");
    if (hi.wp != BRI_F64) return fail(BRI_E_ARG, "the outer operator must have FP64 transporters");
    if (mixed && lo.wp != p->inner_prec) return fail(BRI_E_ARG, "inner operator precision differs from inner_prec");
    if (p->inner_mfma != 0 && p->inner_mfma != 1) return fail(BRI_E_ARG, "inner_mfma must be 0 or 1");
    if (p->inner_mfma && p->inner_prec != BRI_F16)
        return fail(BRI_E_ARG, "the matrix-core inner apply needs inner_prec = BRI_F16");
    if (p->inner_mfma && (lo.rows != 3 || lo.clover))
        return fail(BRI_E_UNSUPPORTED, "the matrix-core inner apply has no two-row store or clover term");
    if (p->inner_mfma && (size_t)g.V / g.L[3] * (size_t)nrhs * 96 > 0xffffffffull)
        return fail(BRI_E_UNSUPPORTED, "a t plane of the matrix-core inner vectors exceeds 4 GiB");
    if (!aligned(hi.W) || !aligned(b) || !aligned(x) || (mixed && !aligned(lo.W)))
        return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t n = (size_t)24 * g.V;
    const Layout L = layout(n, nrhs, mixed ? sizeof(float) : sizeof(double));
    if (!aligned(work) || work_bytes < L.total)
        return fail(BRI_E_WORKSPACE, "workspace too small: need %zu bytes", L.total);
    const size_t vb = n * nrhs * sizeof(double);
    if (overlap(b, vb, x, vb) || overlap(work, L.total, x, vb) || overlap(work, L.total, b, vb))
        return fail(BRI_E_ARG, "b, x and the workspace must not overlap");

    Ctx c{d, g, n, nrhs, mass, p->dagger != 0, (hipStream_t)stream, (char *)work, L};
    *stats = bri_solve_stats{};
    double *r_hi = (double *)(c.w + L.r_hi), *dx = (double *)(c.w + L.dx_hi);
    double *part = (double *)(c.w + L.part), *red = (double *)(c.w + L.red);
    double *scale = (double *)(c.w + L.scale), *unscale = (double *)(c.w + L.unscale);
    const int nb = dot_blocks(n);

    std::vector<double> bb(2 * nrhs), rr(2 * nrhs), sc(nrhs), usc(nrhs);
    BRI_TRY(norm2<double>(c, b, red));
    BRI_TRY(fetch(c, red, bb.data(), bb.size()));
    if (!p->use_initial_guess) BRI_HIP(zero(n * nrhs, x, c.st), "zero x");

    int iters = 0, applies = 0;
    bool converged = false;
    for (int outer = 0;; ++outer) {
        BRI_TRY(apply_op(d, hi, BRI_F64, mass, x, dx, nrhs, c.st, c.dag));
        ++applies;
        BRI_HIP(residual(n, nrhs, b, dx, r_hi, part, nb, c.st), "residual");
        BRI_HIP(dot_finish(nrhs, part, nb, red, c.st), "residual finish");
        BRI_TRY(fetch(c, red, rr.data(), rr.size()));
        converged = true;
        for (int i = 0; i < nrhs; ++i) {
            const double rel = bb[2 * i] > 0.0 ? std::sqrt(rr[2 * i] / bb[2 * i]) : std::sqrt(rr[2 * i]);
            stats->true_residual[i] = rel;
            if (!std::isfinite(rel)) {
                stats->outer = outer;
                stats->iterations = iters;
                stats->applies = applies;
                return fail(BRI_E_NOCONV, "non-finite true residual (rhs %d)", i);
            }
            const bool done = rel <= p->tol;
            converged = converged && done;
            sc[i] = (done || rr[2 * i] == 0.0) ? 0.0 : 1.0 / std::sqrt(rr[2 * i]);
            usc[i] = done ? 0.0 : std::sqrt(rr[2 * i]);
        }
        stats->outer = outer;
        if (converged || outer >= p->max_outer || iters >= p->max_iter) break;
        BRI_HIP(hipMemcpyAsync(scale, sc.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c.st), "copy");
        BRI_HIP(hipMemcpyAsync(unscale, usc.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c.st), "copy");
        int it = 0;
        // worst relative residual among the unconverged columns
        double worst = 0.0;
        for (int i = 0; i < nrhs; ++i)
            if (sc[i] > 0.0) worst = std::fmax(worst, std::sqrt(rr[2 * i] / std::fmax(bb[2 * i], 1e-300)));
        if (mixed) {
            // reduce by inner_tol per cycle, but no further than the final
            // tolerance needs (half of it, for the inner solve's rounding):
            // the last cycle then stops early instead of overshooting
            const double need = worst > 0.0 ? 0.5 * p->tol / worst : 0.5;
            const double rel = std::fmin(0.5, std::fmax(p->inner_tol, need));
            float *r_lo = (float *)(c.w + L.r), *e_lo = (float *)(c.w + L.e);
            // the matrix-core inner solve works on site-major vectors: the
            // scaled residual goes there through q, the correction comes back
            // through q (free outside the inner solve)
            float *t_lo = (float *)(c.w + L.q);
            BRI_HIP((convert<double, float>(n, nrhs, r_hi, lo.mfma ? t_lo : r_lo, scale, c.st)), "convert");
            if (lo.mfma)
                BRI_HIP(spinor_sites(g, nrhs, (const float2 *)t_lo, (float2 *)r_lo, true, nullptr, c.st), "to site-major");
            BRI_TRY(inner_cgne<float>(c, lo, BRI_F32, rel, p->max_iter - iters, p->check_every, &it, &applies));
            if (lo.mfma)
                BRI_HIP(spinor_sites(g, nrhs, (const float2 *)e_lo, (float2 *)t_lo, false, nullptr, c.st),
                        "from site-major");
            BRI_HIP(accum<float>(n, nrhs, lo.mfma ? t_lo : e_lo, x, unscale, c.st), "accumulate");
        } else {
            // plain FP64: aim the inner solve at the final tolerance of the worst column
            const double rel = worst > 0.0 ? std::fmin(0.5, 0.5 * p->tol / worst) : 0.5;
            BRI_HIP((convert<double, double>(n, nrhs, r_hi, (double *)(c.w + L.r), scale, c.st)), "convert");
            BRI_TRY(inner_cgne<double>(c, hi, BRI_F64, rel, p->max_iter - iters, p->check_every, &it,
                                       &applies));
            BRI_HIP(accum<double>(n, nrhs, (const double *)(c.w + L.e), x, unscale, c.st), "accumulate");
        }
        iters += it;
        stats->iterations = iters;
    }
    stats->iterations = iters;
    stats->applies = applies;
    stats->converged = converged ? 1 : 0;
    if (!converged) return fail(BRI_E_NOCONV, "not converged after %d iterations, %d outer cycles", iters, stats->outer);
    return BRI_OK;
}

// ------------------------------------------------------------ allocation-free form
// The workspace of bri_solve_cgne_noalloc: a static device array, one copy per
// device (each device that loads the library's code holds it until the process
// ends).  In host code `scratch` is only the host-side stand-in of the device
// symbol: the device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is ever handed to
// kernels or copies.
static __device__ __align__(256) unsigned char scratch[BRI_SOLVE_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                  // guards g_scratch_ptr
void *g_scratch_ptr[kMaxDevices] = {};    // device address of scratch, per device
std::mutex g_noalloc_mu[kMaxDevices];     // serialises the calls on one device

// the device address of `scratch` on the current device (set up on the first
// call on that device)
bri_status scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail(BRI_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        if (!ptr) return fail(BRI_E_HIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return BRI_OK;
}
}  // namespace

}  // namespace bri

using namespace bri;

extern "C" {

size_t bri_solve_workspace_bytes(bri_dims d, const bri_solve_params *p, int32_t nrhs) {
    Geom g;
    if (!p || !dims_ok(d, &g) || nrhs < 1 || nrhs > BRI_MAX_RHS) return 0;
    const size_t tb = p->inner_prec == BRI_F64 ? sizeof(double) : sizeof(float);
    return layout((size_t)24 * g.V, nrhs, tb).total;
}

bri_status bri_solve_cgne(bri_dims d, const bri_solve_params *p, const void *W_hi, const void *W_lo,
                          double mass, const double *b, double *x, int32_t nrhs, void *work,
                          size_t work_bytes, bri_solve_stats *stats, void *stream) {
    g_last_error.clear();
    if (!p) return fail(BRI_E_ARG, "null params or stats");
    if (p->n_offsets != 40 && p->n_offsets != 80) return fail(BRI_E_ARG, "n_offsets must be 40 or 80");
    const OpDesc hi{W_hi, BRI_F64, p->n_offsets, 3, nullptr, nullptr};
    const OpDesc lo{W_lo, p->inner_prec, p->n_offsets, 3, nullptr, nullptr, p->inner_mfma == 1};
    return solve_core(d, p, hi, lo, mass, b, x, nrhs, work, work_bytes, stats, stream);
}

bri_status bri_solve_cgne_noalloc(bri_dims d, const bri_solve_params *p, const void *W_hi, const void *W_lo,
                                  double mass, const double *b, double *x, int32_t nrhs, bri_solve_stats *stats,
                                  void *stream) {
    g_last_error.clear();
    if (!p) return fail(BRI_E_ARG, "null params or stats");
    if (p->n_offsets != 40 && p->n_offsets != 80) return fail(BRI_E_ARG, "n_offsets must be 40 or 80");
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (nrhs < 1 || nrhs > BRI_MAX_RHS) return fail(BRI_E_ARG, "nrhs must be in [1, %d]", BRI_MAX_RHS);
    const size_t need = bri_solve_workspace_bytes(d, p, nrhs);
    if (need > (size_t)BRI_SOLVE_NOALLOC_MAX_BYTES)
        return fail(BRI_E_WORKSPACE,
                    "the allocation-free solver holds %zu bytes of workspace; this solve needs %zu "
                    "(use bri_solve_cgne with a caller workspace)",
                    (size_t)BRI_SOLVE_NOALLOC_MAX_BYTES, need);
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(BRI_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(BRI_E_UNSUPPORTED, "device index %d out of range", dev);
    void *work = nullptr;
    bri_status s = scratch_address(dev, &work);
    if (s != BRI_OK) return s;
    const OpDesc hi{W_hi, BRI_F64, p->n_offsets, 3, nullptr, nullptr};
    const OpDesc lo{W_lo, p->inner_prec, p->n_offsets, 3, nullptr, nullptr, p->inner_mfma == 1};
    // one call at a time per device: the array is shared, and a call holds it
    // until its work on the stream has finished (also on an error return)
    std::lock_guard<std::mutex> lock(g_noalloc_mu[dev]);
    s = solve_core(d, p, hi, lo, mass, b, x, nrhs, work, (size_t)BRI_SOLVE_NOALLOC_MAX_BYTES, stats, stream);
    const hipError_t es = hipStreamSynchronize((hipStream_t)stream);
    if (s == BRI_OK && es != hipSuccess) return fail(BRI_E_HIP, "synchronize: %s", hipGetErrorString(es));
    return s;
}

bri_status bri_solve_cgne_op(bri_dims d, const bri_solve_params *p, const bri_operator *op_hi,
                             const bri_operator *op_lo, double mass, const double *b, double *x, int32_t nrhs,
                             void *work, size_t work_bytes, bri_solve_stats *stats, void *stream) {
    g_last_error.clear();
    if (!p) return fail(BRI_E_ARG, "null params or stats");
    OpDesc hi{}, lo{};
    bri_status s = op_from_public(op_hi, &hi);
    if (s != BRI_OK) return s;
    if (p->inner_prec != BRI_F64) {
        s = op_from_public(op_lo, &lo);
        if (s != BRI_OK) return s;
        lo.mfma = p->inner_mfma == 1;
        // the inner operator is the same operator at lower precision
        const double *ch = hi.coef, *cl = lo.coef;
        bool same = (ch == nullptr) == (cl == nullptr);
        for (int i = 0; same && ch && i < 9; ++i) same = ch[i] == cl[i];
        if (!same || (hi.clover == nullptr) != (lo.clover == nullptr))
            return fail(BRI_E_ARG, "op_lo must be op_hi at lower precision (same coefficient table and clover term)");
    }
    return solve_core(d, p, hi, lo, mass, b, x, nrhs, work, work_bytes, stats, stream);
}

}  // extern "C"
