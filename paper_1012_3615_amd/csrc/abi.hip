// extern "C" entry points of the library (declared in include/bri.h):
// argument validation, precision dispatch and error reporting.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

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
// Launch configurations installed for particular shapes (the autotuner's
// choices).  A shape is (extents, w_prec, s_prec, n_offsets, nrhs); an apply
// of any other shape takes the built-in selection.  Guarded by a mutex: an
// apply looks its shape up once per call.
struct ApplyConfig {
    int32_t L[4];
    int wp, sp, noff, nrhs, kernel, rblk;
};
constexpr size_t kMaxConfigs = 256;
std::mutex g_cfg_mu;
std::vector<ApplyConfig> g_cfg;

bool same_shape(const ApplyConfig &c, const Geom &g, int wp, int sp, int noff, int nrhs) {
    return c.L[0] == g.L[0] && c.L[1] == g.L[1] && c.L[2] == g.L[2] && c.L[3] == g.L[3] && c.wp == wp &&
           c.sp == sp && c.noff == noff && c.nrhs == nrhs;
}

int snap_rblk(int want, int nrhs) {
    static const int allowed[] = {12, 6, 4, 3, 2, 1};  // snapped down to one of these
    if (want > nrhs) want = nrhs;
    for (int a : allowed)
        if (a <= want) return a;
    return 1;
}
}  // namespace

// The kernel code (never 1) and right-hand sides per thread that an apply of
// this shape launches, from the requested code and blocking (code 1 and
// blocking 2 are the built-in selection).
void resolve_apply_config(const Geom &g, int wp, int sp, int noff, int nrhs, int kernel, int want_rblk,
                          int *kernel_out, int *rblk_out) {
    int rblk = nrhs == 1 ? 1 : snap_rblk(want_rblk, nrhs);
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
    if (kernel == 1) {
        // built-in shapes: transporter prefetch where it is instantiated; the
        // tile width follows Lx so that no lanes idle (24 and 48 wide tiles
        // for extents that are multiples of those but not of 32)
        const int lx = g.L[0];
        if (lx == 16 && rblk == 1 && wp == BRI_F32 && sp == BRI_F32)
            kernel = 14;  // 16x4 with unrolled offsets: four times the workgroups of 16x16 on small lattices
        else if (lx <= 16)
            kernel = rblk == 1 ? 7 : 10;
        else if (rblk <= 2 && lx % 32 != 0 && lx % 48 == 0)
            kernel = 12;
        else if (rblk <= 2 && lx % 32 != 0 && lx % 24 == 0)
            kernel = 11;
        else if (noff == 80 && wp == sp && wp != BRI_F16 && rblk == 1 && lx % 32 == 0 && g.L[1] % 16 == 0)
            kernel = 13;  // 32x16 (halo 1.2x a tile's sites instead of 1.33x): faster for FP32 and FP64 W80
        else
            kernel = rblk <= 2 ? 8 : rblk == 3 ? 9 : 2;
    }
    *kernel_out = kernel;
    *rblk_out = rblk;
}

// the configuration installed for this shape, else the built-in one
void lookup_apply_config(const Geom &g, int wp, int sp, int noff, int nrhs, int *kernel, int *rblk) {
    int k = 1, r = 2;
    {
        std::lock_guard<std::mutex> lock(g_cfg_mu);
        for (const ApplyConfig &c : g_cfg)
            if (same_shape(c, g, wp, sp, noff, nrhs)) {
                k = c.kernel;
                r = c.rblk;
                break;
            }
    }
    resolve_apply_config(g, wp, sp, noff, nrhs, k, r, kernel, rblk);
}

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
        int kernel, rblk;
        lookup_apply_config(g, (int)wp, (int)sp, noff, nrhs, &kernel, &rblk);
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
    (void)d;
    (void)p;
    (void)noff;
    return 0;  // the fused build keeps its lower levels on chip
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
    (void)work;
    (void)work_bytes;
    return hip_check(build_fused(g, (const double2 *)U, W, (int)wp, noff, (hipStream_t)stream), "build transporters");
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

bri_status bri_set_apply_config(bri_dims d, bri_prec wp, bri_prec sp, int32_t noff, int32_t nrhs, int32_t kernel,
                                int32_t rblk) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(wp) || !prec_ok(sp)) return fail(BRI_E_ARG, "invalid precision");
    if (noff != 40 && noff != 80) return fail(BRI_E_ARG, "n_offsets must be 40 or 80");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (kernel < -1 || kernel > 14) return fail(BRI_E_ARG, "kernel must be in 0..14 (or -1 to remove)");
    if (kernel >= 0 && rblk != 1 && rblk != 2 && rblk != 3 && rblk != 4 && rblk != 6 && rblk != 12)
        return fail(BRI_E_ARG, "rhs_per_thread must be 1, 2, 3, 4, 6 or 12");
    std::lock_guard<std::mutex> lock(g_cfg_mu);
    for (size_t i = 0; i < g_cfg.size(); ++i)
        if (same_shape(g_cfg[i], g, wp, sp, noff, nrhs)) {
            if (kernel < 0) {
                g_cfg.erase(g_cfg.begin() + (long)i);
            } else {
                g_cfg[i].kernel = kernel;
                g_cfg[i].rblk = rblk;
            }
            return BRI_OK;
        }
    if (kernel < 0) return BRI_OK;
    if (g_cfg.size() >= kMaxConfigs)
        return fail(BRI_E_ARG, "at most %zu shapes can carry an installed configuration", kMaxConfigs);
    g_cfg.push_back(ApplyConfig{{g.L[0], g.L[1], g.L[2], g.L[3]}, (int)wp, (int)sp, noff, nrhs, kernel, rblk});
    return BRI_OK;
}

bri_status bri_get_apply_config(bri_dims d, bri_prec wp, bri_prec sp, int32_t noff, int32_t nrhs, int32_t *kernel,
                                int32_t *rblk) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(wp) || !prec_ok(sp)) return fail(BRI_E_ARG, "invalid precision");
    if (noff != 40 && noff != 80) return fail(BRI_E_ARG, "n_offsets must be 40 or 80");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!kernel || !rblk) return fail(BRI_E_ARG, "null output pointer");
    int k, r;
    lookup_apply_config(g, (int)wp, (int)sp, noff, nrhs, &k, &r);
    *kernel = k;
    *rblk = r;
    return BRI_OK;
}

void bri_clear_apply_configs(void) {
    std::lock_guard<std::mutex> lock(g_cfg_mu);
    g_cfg.clear();
}

}  // extern "C"
