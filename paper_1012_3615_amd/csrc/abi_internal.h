// Helpers shared by the translation units that implement include/bri.h.
#pragma once

#include <cstdarg>
#include <string>

#include "../../include/bri.h"
#include "common.h"

namespace bri {

extern thread_local std::string g_last_error;

bri_status fail(bri_status s, const char *fmt, ...);
bri_status hip_check(hipError_t e, const char *what);
bool dims_ok(bri_dims d, Geom *g);
size_t cbytes(bri_prec p);
bool prec_ok(bri_prec p);
bool aligned(const void *p);
bool overlap(const void *a, size_t na, const void *b, size_t nb);
// table: lambda_0..4, rho_1..4 of the generic class (host), nullptr for the
// Brillouin operator; the stored variant only
bri_status apply_impl(bri_dims d, bri_variant v, const void *W, bri_prec wp, int32_t noff,
                      bri_prec sp, double mass, const void *in, void *out, int32_t nrhs,
                      void *stream, bool dag, const double *table = nullptr);

// A stored-transporter operator: W, its precision and offset count, the number
// of stored rows per transporter (3, or 2 for the two-row SU(3) store), the
// clover term (nullptr for c_SW = 0) and the coefficient table of the generic
// class (lambda_0..4, rho_1..4 on the host; nullptr for the Brillouin column).
struct OpDesc {
    const void *W;
    bri_prec wp;
    int32_t noff;
    int rows;
    const void *clover;
    const double *coef;
    bool mfma = false;  // W is the matrix-core store (bri_pack_w_mfma); FP32 fields
};
bri_status op_from_public(const bri_operator *op, OpDesc *out);
bri_status apply_op(bri_dims d, const OpDesc &op, bri_prec sp, double mass, const void *in, void *out,
                    int32_t nrhs, void *stream, bool dag);

}  // namespace bri
