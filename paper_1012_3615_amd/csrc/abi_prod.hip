// C ABI of the production-operator ingredients (Sec. 5): SU(3) projection,
// APE smearing, back-projected transporters, the clover term, and the apply
// of a general stored-transporter operator (any member of the generic class
// of Sec. 8).
#include <cmath>

#include "abi_internal.h"
#include "kernels.h"

namespace bri {

bri_status op_from_public(const bri_operator *op, OpDesc *out) {
    if (!op) return fail(BRI_E_ARG, "null operator");
    if (op->w_form != BRI_W_AVERAGE && op->w_form != BRI_W_SU3 && op->w_form != BRI_W_SU3_2ROW)
        return fail(BRI_E_ARG, "invalid transporter form");
    if (op->coef)
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(op->coef[i])) return fail(BRI_E_ARG, "coefficient %d of the table is not finite", i);
    *out = OpDesc{op->W, op->w_prec, op->n_offsets, op->w_form == BRI_W_SU3_2ROW ? 2 : 3, op->clover, op->coef};
    return BRI_OK;
}

bri_status apply_op(bri_dims d, const OpDesc &op, bri_prec sp, double mass, const void *in, void *out,
                    int32_t nrhs, void *stream, bool dag) {
    if (op.rows == 3 && !op.clover)
        return apply_impl(d, BRI_STORED, op.W, op.wp, op.noff, sp, mass, in, out, nrhs, stream, dag, op.coef);
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(op.wp) || !prec_ok(sp)) return fail(BRI_E_ARG, "invalid precision");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!aligned(op.W) || !aligned(in) || !aligned(out) || (op.clover && !aligned(op.clover)))
        return fail(BRI_E_ARG, "null or misaligned (16 B) pointer");
    const size_t sb = (size_t)g.V * 12 * nrhs * cbytes(sp);
    if (overlap(in, sb, out, sb)) return fail(BRI_E_ARG, "in and out overlap");
    if (op.noff != 80)
        return fail(BRI_E_UNSUPPORTED, "the two-row store and the clover term need n_offsets = 80");
    const double diag = (op.coef ? op.coef[0] : lam_k(0)) + mass;
    const int rblk = nrhs >= 2 ? 2 : 1;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (op.wp == BRI_F64 && sp == BRI_F64)
        e = apply_prod_f64(g, op.rows, rblk, op.W, in, out, diag, nrhs, dag, st, op.clover, op.coef);
    else if (op.wp == BRI_F32 && sp == BRI_F32)
        e = apply_prod_f32(g, op.rows, rblk, op.W, in, out, diag, nrhs, dag, st, op.clover, op.coef);
    else if (op.wp == BRI_F16 && sp == BRI_F32)
        e = apply_prod_f16(g, op.rows, rblk, op.W, in, out, diag, nrhs, dag, st, op.clover, op.coef);
    else if (op.wp == BRI_F16 && sp == BRI_F16)
        e = apply_prod_f16h(g, op.rows, rblk, op.W, in, out, diag, nrhs, dag, st, op.clover, op.coef);
    else
        return fail(BRI_E_UNSUPPORTED, "unsupported (w_prec, s_prec) combination");
    return hip_check(e, "apply (production operator)");
}

}  // namespace bri

using namespace bri;

extern "C" {

bri_status bri_project_su3(int64_t n, const double *A, double *Y, void *stream) {
    g_last_error.clear();
    if (n < 0) return fail(BRI_E_ARG, "n must be >= 0");
    if (n == 0) return BRI_OK;
    if (!aligned(A) || !aligned(Y)) return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t bytes = (size_t)n * 9 * 16;
    if (A != Y && overlap(A, bytes, Y, bytes)) return fail(BRI_E_ARG, "A and Y overlap partially");
    return hip_check(project_su3_soa((const double2 *)A, (double2 *)Y, n, (hipStream_t)stream), "project_su3");
}

bri_status bri_ape_smear(bri_dims d, const double *U, double *V, double alpha, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!std::isfinite(alpha)) return fail(BRI_E_ARG, "alpha must be finite");
    if (!aligned(U) || !aligned(V)) return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t bytes = (size_t)g.V * 36 * 16;
    if (overlap(U, bytes, V, bytes)) return fail(BRI_E_ARG, "input and output links overlap");
    return hip_check(ape_smear(g, (const double2 *)U, (double2 *)V, alpha, (hipStream_t)stream), "ape_smear");
}

size_t bri_transporter_bytes_ex(bri_dims d, bri_prec p, int32_t noff, bri_wform form) {
    Geom g;
    if (!dims_ok(d, &g) || !prec_ok(p) || (noff != 40 && noff != 80)) return 0;
    if (form == BRI_W_AVERAGE || form == BRI_W_SU3) return (size_t)g.V * 9 * noff * cbytes(p);
    if (form == BRI_W_SU3_2ROW) return (size_t)g.V * 6 * noff * cbytes(p);
    return 0;
}

size_t bri_build_workspace_bytes_ex(bri_dims d, bri_prec p, int32_t noff, bri_wform form) {
    Geom g;
    if (!dims_ok(d, &g) || !prec_ok(p) || (noff != 40 && noff != 80)) return 0;
    if (form == BRI_W_AVERAGE) return bri_build_workspace_bytes(d, p, noff);
    // the SU(3) form projects the FP64 40-offset store, which is the output
    // itself only for FP64 with 40 offsets
    if (form == BRI_W_SU3) return (p == BRI_F64 && noff == 40) ? 0 : (size_t)g.V * 9 * 40 * 16;
    if (form == BRI_W_SU3_2ROW) return (size_t)g.V * 9 * 40 * 16;
    return 0;
}

bri_status bri_build_transporters_ex(bri_dims d, const double *U, void *W, bri_prec wp, int32_t noff,
                                     bri_wform form, void *work, size_t work_bytes, void *stream) {
    g_last_error.clear();
    if (form == BRI_W_AVERAGE) return bri_build_transporters(d, U, W, wp, noff, work, work_bytes, stream);
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(wp)) return fail(BRI_E_ARG, "invalid precision");
    if (noff != 40 && noff != 80) return fail(BRI_E_ARG, "n_offsets must be 40 or 80");
    if (form != BRI_W_SU3 && form != BRI_W_SU3_2ROW) return fail(BRI_E_ARG, "invalid transporter form");
    if (!aligned(U) || !aligned(W)) return fail(BRI_E_ARG, "null or misaligned pointer");
    const size_t need = bri_build_workspace_bytes_ex(d, wp, noff, form);
    hipStream_t st = (hipStream_t)stream;
    double2 *stage = (double2 *)W;
    if (need > 0) {
        if (!aligned(work) || work_bytes < need)
            return fail(BRI_E_WORKSPACE, "workspace too small: need %zu bytes", need);
        if (overlap(work, need, W, bri_transporter_bytes_ex(d, wp, noff, form)))
            return fail(BRI_E_ARG, "workspace overlaps the transporter store");
        stage = (double2 *)work;
    }
    bri_status s = hip_check(build_w40_f64(g, (const double2 *)U, stage, st), "build transporters");
    if (s != BRI_OK) return s;
    s = hip_check(project_w40(g, stage, st), "project transporters");
    if (s != BRI_OK) return s;
    if (form == BRI_W_SU3_2ROW)
        return hip_check(convert_w40_rows2(g, stage, W, (int)wp, noff, st), "convert transporters");
    if (need == 0) return BRI_OK;  // FP64, 40 offsets: built in place
    return hip_check(convert_w40(g, stage, W, (int)wp, noff, st), "convert transporters");
}

size_t bri_clover_bytes(bri_dims d, bri_prec p) {
    Geom g;
    if (!dims_ok(d, &g) || !prec_ok(p)) return 0;
    return (size_t)g.V * 36 * cbytes(p);
}

bri_status bri_build_clover(bri_dims d, const double *U, double csw, void *C, bri_prec cp, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(cp)) return fail(BRI_E_ARG, "invalid precision");
    if (!std::isfinite(csw)) return fail(BRI_E_ARG, "c_SW must be finite");
    if (!aligned(U) || !aligned(C)) return fail(BRI_E_ARG, "null or misaligned pointer");
    return hip_check(build_clover(g, (const double2 *)U, C, (int)cp, csw, (hipStream_t)stream), "build_clover");
}

bri_status bri_apply_op(bri_dims d, const bri_operator *op, bri_prec sp, double mass, const void *in, void *out,
                        int32_t nrhs, int32_t dagger, void *stream) {
    g_last_error.clear();
    OpDesc o;
    bri_status s = op_from_public(op, &o);
    if (s != BRI_OK) return s;
    return apply_op(d, o, sp, mass, in, out, nrhs, stream, dagger != 0);
}

}  // extern "C"
