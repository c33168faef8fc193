// Device helpers shared by the kernels: storage <-> compute conversions,
// bfloat16 rounding, 64-lane cross-lane moves (DPP), wave reductions and the
// deterministic last-block norm reduction with the device-side stop test.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "mg_internal.h"

namespace mgx {

// ---- bfloat16: round to nearest, ties to even on the 16 dropped bits; NaN
// stays NaN (quiet bit set).  Written from the format definition.
__device__ __forceinline__ float bf16_to_f32(bf16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ bf16_t f32_to_bf16(float x)
{
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu)) return (bf16_t)((b | 0x00400000u) >> 16);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (bf16_t)(b >> 16);
}
__device__ __forceinline__ float bf16_round(float x) { return bf16_to_f32(f32_to_bf16(x)); }

// ---- storage traits: S = stored type, C = arithmetic type ----------------
template <class S> struct Traits;
template <> struct Traits<double> {
    using C = double;
    static __device__ __forceinline__ double ld(const double *p) { return *p; }
    static __device__ __forceinline__ void st(double *p, double v) { *p = v; }
    static __device__ __forceinline__ double rnd(double v) { return v; }
};
template <> struct Traits<float> {
    using C = float;
    static __device__ __forceinline__ float ld(const float *p) { return *p; }
    static __device__ __forceinline__ void st(float *p, float v) { *p = v; }
    static __device__ __forceinline__ float rnd(float v) { return v; }
};
template <> struct Traits<bf16_t> {
    using C = float;
    static __device__ __forceinline__ float ld(const bf16_t *p) { return bf16_to_f32(*p); }
    // values are rounded by rnd() when computed, so the store is exact
    static __device__ __forceinline__ void st(bf16_t *p, float v) { *p = (bf16_t)(__float_as_uint(v) >> 16); }
    static __device__ __forceinline__ float rnd(float v) { return bf16_round(v); }
};

// ---- cross-lane moves within one 64-lane wavefront -------------------------
// DPP wave_shr:1 (lane l <- lane l-1) and wave_shl:1 (lane l <- lane l+1);
// the edge lane receives `edge`.
__device__ __forceinline__ int dpp_from_prev(int x, int edge)
{
    return __builtin_amdgcn_update_dpp(edge, x, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_from_next(int x, int edge)
{
    return __builtin_amdgcn_update_dpp(edge, x, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float from_prev(float x, float edge)
{
    return __int_as_float(dpp_from_prev(__float_as_int(x), __float_as_int(edge)));
}
__device__ __forceinline__ float from_next(float x, float edge)
{
    return __int_as_float(dpp_from_next(__float_as_int(x), __float_as_int(edge)));
}
__device__ __forceinline__ double from_prev(double x, double edge)
{
    int2 v = *reinterpret_cast<int2 *>(&x), e = *reinterpret_cast<int2 *>(&edge);
    int2 r;
    r.x = dpp_from_prev(v.x, e.x);
    r.y = dpp_from_prev(v.y, e.y);
    return *reinterpret_cast<double *>(&r);
}
__device__ __forceinline__ double from_next(double x, double edge)
{
    int2 v = *reinterpret_cast<int2 *>(&x), e = *reinterpret_cast<int2 *>(&edge);
    int2 r;
    r.x = dpp_from_next(v.x, e.x);
    r.y = dpp_from_next(v.y, e.y);
    return *reinterpret_cast<double *>(&r);
}
__device__ __forceinline__ float lane_value(float x, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ double lane_value(double x, int lane)
{
    int2 v = *reinterpret_cast<int2 *>(&x);
    int2 r;
    r.x = __builtin_amdgcn_readlane(v.x, lane);
    r.y = __builtin_amdgcn_readlane(v.y, lane);
    return *reinterpret_cast<double *>(&r);
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---- deterministic norm reduction + stop test ------------------------------
// Every work item of system `sys` writes its partial sum(s) to
// partials[slot*2 + {0,1}], then the item that finishes last adds all of the
// system's partials in slot order (so the result does not depend on which
// item ran when) and applies the stop test:
//   rel = sqrt(rr / ff); hist[nres] = rel; done = 1 if rel <= tol,
//   2 if not finite, 3 if nres reached the cycle limit.
// `first` marks the norm before the first cycle: it also fixes ff = ||f||^2.
// Called by one thread (thread 0 of the block).
__device__ inline void finish_norm(SolveState *st, double *partials, int slot0, int nslots, int myslot,
                                   double rr, double ff, int first)
{
    partials[2 * myslot] = rr;
    partials[2 * myslot + 1] = ff;
    __threadfence();
    unsigned prev = atomicAdd(&st->counter, 1u);
    if (prev + 1 != (unsigned)nslots) return;
    __threadfence();
    double srr = 0.0, sff = 0.0;
    const volatile double *vp = partials;
    for (int k = 0; k < nslots; ++k) {
        srr += vp[2 * (slot0 + k)];
        sff += vp[2 * (slot0 + k) + 1];
    }
    st->counter = 0u;
    if (first) {
        st->ff = sff;
        st->nres = 0;
    }
    double rel = sqrt(srr) / sqrt(st->ff);
    int k = st->nres;
    if (k <= 200) st->hist[k] = rel;
    st->rel = rel;
    st->nres = k + 1;
    int done = 0;
    if (!isfinite(rel)) done = 2;
    else if (rel <= st->tol) done = 1;
    else if (k >= st->maxc) done = 3;
    __threadfence();
    st->done = done;
}

}  // namespace mgx
