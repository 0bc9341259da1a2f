// extern "C" entry points of the library (declared in include/bri.h):
// argument validation, precision dispatch and error reporting.
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/bri.h"
#include "common.h"
#include "kernels.h"
#include "abi_internal.h"

namespace bri {

thread_local std::string g_last_error;

bri_status fail(bri_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

bri_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return BRI_OK;
    return fail(BRI_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool dims_ok(bri_dims d, Geom *g) {
    long long v = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (d.L[mu] < 2 || d.L[mu] > 4096) return false;
        v *= d.L[mu];
    }
    if (v > (1LL << 30)) return false;
    *g = make_geom(d.L);
    return true;
}

size_t cbytes(bri_prec p) { return p == BRI_F64 ? 16 : p == BRI_F32 ? 8 : 4; }

bool prec_ok(bri_prec p) { return p == BRI_F64 || p == BRI_F32 || p == BRI_F16; }

bool aligned(const void *p) { return p != nullptr && ((uintptr_t)p & 15) == 0; }

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

namespace {
// rhs-per-thread setting of the fused multi-RHS apply, per (w_prec, s_prec)
int g_rhs_block[3][3] = {{2, 2, 2}, {2, 2, 2}, {2, 2, 2}};
// apply kernel per (w_prec, s_prec): 0 = register-blocked gather, 1 = LDS tiles
// with the tile shape chosen from Lx, 2..5 = LDS tiles 32x8, 16x16, 64x4, 16x8,
// 6, 7 = tiles 32x8, 16x16 with transporter prefetch
int g_apply_kernel[3][3] = {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}};

int snap_rblk(int want, int nrhs) {
    static const int allowed[] = {12, 6, 4, 3, 2, 1};  // snapped down to one of these
    if (want > nrhs) want = nrhs;
    for (int a : allowed)
        if (a <= want) return a;
    return 1;
}
}  // namespace

bri_status apply_impl(bri_dims d, bri_variant v, const void *W, bri_prec wp, int32_t noff,
                      bri_prec sp, double mass, const void *in, void *out, int32_t nrhs,
                      void *stream, bool dag, const double *table) {
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(wp) || !prec_ok(sp)) return fail(BRI_E_ARG, "invalid precision");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!aligned(W) || !aligned(in) || !aligned(out))
        return fail(BRI_E_ARG, "null or misaligned (16 B) pointer");
    const size_t sb = (size_t)g.V * 12 * nrhs * cbytes(sp);
    if (overlap(in, sb, out, sb)) return fail(BRI_E_ARG, "in and out overlap");
    const double diag = (table ? table[0] : lam_k(0)) + mass;
    hipStream_t st = (hipStream_t)stream;
    if (table && v != BRI_STORED) return fail(BRI_E_UNSUPPORTED, "a coefficient table needs stored transporters");
    if (v == BRI_STORED) {
        if (noff != 40 && noff != 80) return fail(BRI_E_ARG, "n_offsets must be 40 or 80");
        const bool combo = (wp == BRI_F64 && sp == BRI_F64) || (wp == BRI_F32 && sp == BRI_F32) ||
                           (wp == BRI_F16 && (sp == BRI_F32 || sp == BRI_F16));
        if (!combo) return fail(BRI_E_UNSUPPORTED, "unsupported (w_prec, s_prec) combination");
        const int kernel = g_apply_kernel[wp][sp];
        int rblk = nrhs == 1 ? 1 : snap_rblk(g_rhs_block[wp][sp], nrhs);
        if (kernel >= 1) {
            // LDS tiles hold 1..4 right-hand sides per thread (shapes 16x16, 64x4: 1)
            if (kernel == 3 || kernel == 4 || kernel == 7 || kernel == 13 || kernel == 14) rblk = 1;
            if ((kernel == 6 || kernel == 8 || kernel == 11 || kernel == 12) && rblk > 2) rblk = 2;
            if (kernel == 9 && rblk > 3) rblk = 3;
            if (kernel == 10 && rblk < 2) rblk = 2;
            if (rblk > 4) rblk = 4;
            if (wp == BRI_F64 && rblk > 2 && kernel != 5 && kernel != 10 && !(kernel == 1 && g.L[0] <= 16))
                rblk = 2;  // LDS of a 32x8 tile
        }
        return hip_check(apply_stored(g, noff, (int)wp, (int)sp, kernel, rblk, W, in, out, diag, nrhs,
                                      dag, st, table),
                         "apply (stored)");
    }
    if (v == BRI_RECOMPUTE) {
        if (!((wp == BRI_F64 && sp == BRI_F64) || (wp == BRI_F32 && sp == BRI_F32)))
            return fail(BRI_E_UNSUPPORTED, "recompute variant supports F64/F64 and F32/F32");
        return hip_check(apply_recompute(g, (int)wp, (int)sp, W, in, out, diag, nrhs, dag, st),
                         "apply (recompute)");
    }
    return fail(BRI_E_ARG, "invalid variant");
}

}  // namespace bri

using namespace bri;

extern "C" {

const char *bri_last_error(void) { return g_last_error.c_str(); }

int32_t bri_abi_version(void) { return BRI_ABI_VERSION; }

size_t bri_spinor_bytes(bri_dims d, bri_prec p, int32_t nrhs) {
    Geom g;
    if (!dims_ok(d, &g) || !prec_ok(p) || nrhs < 1) return 0;
    return (size_t)g.V * 12 * nrhs * cbytes(p);
}

size_t bri_links_bytes(bri_dims d, bri_prec p) {
    Geom g;
    if (!dims_ok(d, &g) || !prec_ok(p)) return 0;
    return (size_t)g.V * 36 * cbytes(p);
}

size_t bri_transporter_bytes(bri_dims d, bri_prec p, int32_t noff) {
    Geom g;
    if (!dims_ok(d, &g) || !prec_ok(p) || (noff != 40 && noff != 80)) return 0;
    return (size_t)g.V * 9 * noff * cbytes(p);
}

size_t bri_build_workspace_bytes(bri_dims d, bri_prec p, int32_t noff) {
    Geom g;
    if (!dims_ok(d, &g) || !prec_ok(p) || (noff != 40 && noff != 80)) return 0;
    if (p == BRI_F64 && noff == 40) return 0;
    return (size_t)g.V * 9 * 40 * 16;
}

bri_status bri_pack_links(bri_dims d, const double *U, void *soa, bri_prec p, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(p)) return fail(BRI_E_ARG, "invalid precision");
    if (!aligned(U) || !aligned(soa)) return fail(BRI_E_ARG, "null or misaligned pointer");
    return hip_check(pack_links(g, (const double2 *)U, soa, (int)p, (hipStream_t)stream), "pack_links");
}

bri_status bri_pack_spinor(bri_dims d, int32_t nrhs, const double *psi, void *soa, bri_prec p,
                           void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(p)) return fail(BRI_E_ARG, "invalid precision");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!aligned(psi) || !aligned(soa)) return fail(BRI_E_ARG, "null or misaligned pointer");
    return hip_check(pack_spinor(g, nrhs, (const double2 *)psi, soa, (int)p, (hipStream_t)stream),
                     "pack_spinor");
}

bri_status bri_unpack_spinor(bri_dims d, int32_t nrhs, const void *soa, bri_prec p, double *psi,
                             void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(p)) return fail(BRI_E_ARG, "invalid precision");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!aligned(psi) || !aligned(soa)) return fail(BRI_E_ARG, "null or misaligned pointer");
    return hip_check(unpack_spinor(g, nrhs, soa, (int)p, (double2 *)psi, (hipStream_t)stream),
                     "unpack_spinor");
}

bri_status bri_unpack_links(bri_dims d, const void *soa, bri_prec p, double *U, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(p)) return fail(BRI_E_ARG, "invalid precision");
    if (!aligned(U) || !aligned(soa)) return fail(BRI_E_ARG, "null or misaligned pointer");
    return hip_check(unpack_links(g, soa, (int)p, (double2 *)U, (hipStream_t)stream), "unpack_links");
}

bri_status bri_build_transporters(bri_dims d, const double *U, void *W, bri_prec wp, int32_t noff,
                                  void *work, size_t work_bytes, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(wp)) return fail(BRI_E_ARG, "invalid precision");
    if (noff != 40 && noff != 80) return fail(BRI_E_ARG, "n_offsets must be 40 or 80");
    if (!aligned(U) || !aligned(W)) return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t need = bri_build_workspace_bytes(d, wp, noff);
    hipStream_t st = (hipStream_t)stream;
    if (need == 0) {
        return hip_check(build_w40_f64(g, (const double2 *)U, (double2 *)W, st), "build transporters");
    }
    if (!aligned(work) || work_bytes < need)
        return fail(BRI_E_WORKSPACE, "workspace too small: need %zu bytes", need);
    if (overlap(work, need, W, bri_transporter_bytes(d, wp, noff)))
        return fail(BRI_E_ARG, "workspace overlaps the transporter store");
    return hip_check(build_cast(g, (const double2 *)U, (double2 *)work, W, (int)wp, noff, st), "build transporters");
}

bri_status bri_apply(bri_dims d, bri_variant v, const void *W, bri_prec wp, int32_t noff,
                     bri_prec sp, double mass, const void *in, void *out, int32_t nrhs,
                     void *stream) {
    g_last_error.clear();
    return apply_impl(d, v, W, wp, noff, sp, mass, in, out, nrhs, stream, false);
}

bri_status bri_apply_dag(bri_dims d, bri_variant v, const void *W, bri_prec wp, int32_t noff,
                         bri_prec sp, double mass, const void *in, void *out, int32_t nrhs,
                         void *stream) {
    g_last_error.clear();
    return apply_impl(d, v, W, wp, noff, sp, mass, in, out, nrhs, stream, true);
}

bri_status bri_apply_wilson(bri_dims d, const void *U, bri_prec prec, double mass, const void *in, void *out,
                            int32_t nrhs, int32_t dagger, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (prec != BRI_F64 && prec != BRI_F32) return fail(BRI_E_UNSUPPORTED, "the Wilson apply runs in F64 or F32");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (dagger != 0 && dagger != 1) return fail(BRI_E_ARG, "dagger must be 0 or 1");
    if (!aligned(U) || !aligned(in) || !aligned(out))
        return fail(BRI_E_ARG, "null or misaligned (16 B) pointer");
    const size_t sb = (size_t)g.V * 12 * nrhs * cbytes(prec);
    if (overlap(in, sb, out, sb)) return fail(BRI_E_ARG, "in and out overlap");
    return hip_check(apply_wilson(g, (int)prec, U, in, out, 4.0 + mass, nrhs, dagger != 0, (hipStream_t)stream),
                     "apply (Wilson)");
}

bri_status bri_set_rhs_block(bri_prec wp, bri_prec sp, int32_t r) {
    g_last_error.clear();
    if (!prec_ok(wp) || !prec_ok(sp)) return fail(BRI_E_ARG, "invalid precision");
    if (r == 0) r = 2;
    if (r != 1 && r != 2 && r != 3 && r != 4 && r != 6 && r != 12)
        return fail(BRI_E_ARG, "rhs_per_thread must be 1, 2, 3, 4, 6 or 12");
    g_rhs_block[wp][sp] = r;
    return BRI_OK;
}

bri_status bri_set_apply_kernel(bri_prec wp, bri_prec sp, int32_t kernel) {
    g_last_error.clear();
    if (!prec_ok(wp) || !prec_ok(sp)) return fail(BRI_E_ARG, "invalid precision");
    if (kernel < 0 || kernel > 14) return fail(BRI_E_ARG, "kernel must be in 0..14");
    g_apply_kernel[wp][sp] = kernel;
    return BRI_OK;
}

int32_t bri_get_apply_kernel(bri_prec wp, bri_prec sp) {
    if (!prec_ok(wp) || !prec_ok(sp)) return -1;
    return g_apply_kernel[wp][sp];
}

int32_t bri_get_rhs_block(bri_prec wp, bri_prec sp) {
    if (!prec_ok(wp) || !prec_ok(sp)) return 0;
    return g_rhs_block[wp][sp];
}

}  // extern "C"
