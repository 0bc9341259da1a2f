// Layout conversion between the canonical complex128 arrays
// (links [mu][site][3][3], spinors [rhs][site][4][3]) and the structure-of-
// arrays planes used by the kernels ([mu][9][V], [rhs][12][V]).
#include "common.h"
#include "kernels.h"

namespace bri {
namespace {

template <typename T, int NE>
__global__ __launch_bounds__(256) void k_pack(int V, int nblk, const double2 *__restrict__ canon,
                                              T *__restrict__ soa) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= V) return;
    const size_t b = blockIdx.y;  // mu or rhs
    const double2 *src = canon + (b * (size_t)V + site) * NE;
    T *dst = soa + b * NE * (size_t)V + site;
#pragma unroll
    for (int e = 0; e < NE; ++e) st(dst + e * (size_t)V, ldc<double>(src + e));
}

template <typename T, int NE>
__global__ __launch_bounds__(256) void k_unpack(int V, const T *__restrict__ soa,
                                                double2 *__restrict__ canon) {
    const int site = blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= V) return;
    const size_t b = blockIdx.y;
    const T *src = soa + b * NE * (size_t)V + site;
    double2 *dst = canon + (b * (size_t)V + site) * NE;
#pragma unroll
    for (int e = 0; e < NE; ++e) st(dst + e, ldc<double>(src + e * (size_t)V));
}

constexpr int kBlock = 256;

template <int NE>
hipError_t pack_any(const Geom &g, int nb, const double2 *canon, void *soa, int p, hipStream_t st) {
    dim3 grid((g.V + kBlock - 1) / kBlock, nb);
    if (p == 0)
        hipLaunchKernelGGL((k_pack<double2, NE>), grid, dim3(kBlock), 0, st, g.V, nb, canon, (double2 *)soa);
    else if (p == 1)
        hipLaunchKernelGGL((k_pack<float2, NE>), grid, dim3(kBlock), 0, st, g.V, nb, canon, (float2 *)soa);
    else if (p == 2)
        hipLaunchKernelGGL((k_pack<__half2, NE>), grid, dim3(kBlock), 0, st, g.V, nb, canon, (__half2 *)soa);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
}  // namespace

hipError_t pack_links(const Geom &g, const double2 *canon, void *soa, int p, hipStream_t st) {
    return pack_any<9>(g, 4, canon, soa, p, st);
}

hipError_t pack_spinor(const Geom &g, int nrhs, const double2 *canon, void *soa, int p,
                       hipStream_t st) {
    return pack_any<12>(g, nrhs, canon, soa, p, st);
}

hipError_t unpack_links(const Geom &g, const void *soa, int p, double2 *canon, hipStream_t st) {
    dim3 grid((g.V + kBlock - 1) / kBlock, 4);
    if (p == 0)
        hipLaunchKernelGGL((k_unpack<double2, 9>), grid, dim3(kBlock), 0, st, g.V, (const double2 *)soa, canon);
    else if (p == 1)
        hipLaunchKernelGGL((k_unpack<float2, 9>), grid, dim3(kBlock), 0, st, g.V, (const float2 *)soa, canon);
    else if (p == 2)
        hipLaunchKernelGGL((k_unpack<__half2, 9>), grid, dim3(kBlock), 0, st, g.V, (const __half2 *)soa, canon);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t unpack_spinor(const Geom &g, int nrhs, const void *soa, int p, double2 *canon,
                         hipStream_t st) {
    dim3 grid((g.V + kBlock - 1) / kBlock, nrhs);
    if (p == 0)
        hipLaunchKernelGGL((k_unpack<double2, 12>), grid, dim3(kBlock), 0, st, g.V, (const double2 *)soa, canon);
    else if (p == 1)
        hipLaunchKernelGGL((k_unpack<float2, 12>), grid, dim3(kBlock), 0, st, g.V, (const float2 *)soa, canon);
    else if (p == 2)
        hipLaunchKernelGGL((k_unpack<__half2, 12>), grid, dim3(kBlock), 0, st, g.V, (const __half2 *)soa, canon);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace bri
