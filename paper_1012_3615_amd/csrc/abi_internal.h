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
bri_status apply_impl(bri_dims d, bri_variant v, const void *W, bri_prec wp, int32_t noff,
                      bri_prec sp, double mass, const void *in, void *out, int32_t nrhs,
                      void *stream, bool dag);

}  // namespace bri
