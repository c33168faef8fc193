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
// stays NaN.  gfx950 converts in hardware (v_cvt_pk_bf16_f32, two values per
// instruction), which the compiler emits for a conversion to __bf16.
__device__ __forceinline__ float bf16_to_f32(bf16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ __forceinline__ bf16_t f32_to_bf16(float x) { return __builtin_bit_cast(bf16_t, (__bf16)x); }
// two values packed into one dword, lo in the low half
__device__ __forceinline__ uint32_t f32x2_to_bf16x2(float lo, float hi)
{
    typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
    typedef float f32x2_t __attribute__((ext_vector_type(2)));
    const f32x2_t v = {lo, hi};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}
__device__ __forceinline__ float bf16_round(float x) { return bf16_to_f32(f32_to_bf16(x)); }

// ---- explicit global-address-space access (global_load / global_store
// instead of flat ones when the pointer came through a descriptor) --------
template <class T>
__device__ __forceinline__ T gld(const T *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ void gst(T *p, T v)
{
    *(__attribute__((address_space(1))) T *)p = v;
}

// ---- buffer (resource-descriptor) memory access ---------------------------
// A raw buffer load whose byte offset lies beyond the descriptor's record
// count returns 0 and such a store is dropped, so masked lanes and rows need
// no branch: they use the offset kOOB.  Records are 32-bit byte counts (arrays
// below 4 GiB).  Dword 3 = 0x00020000 is the gfx9-family data format word.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr uint32_t kOOB = 0xFFFFFFF0u;
__device__ __forceinline__ rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <class T> __device__ __forceinline__ T bld(rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ double bld<double>(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <> __device__ __forceinline__ float bld<float>(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <> __device__ __forceinline__ bf16_t bld<bf16_t>(rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(bf16_t, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t off, double v)
{
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t off, bf16_t v)
{
    __builtin_amdgcn_raw_buffer_store_b16(v, r, off, 0, 0);
}

// ---- storage traits: S = stored type, C = arithmetic type ----------------
template <class S> struct Traits;
template <> struct Traits<double> {
    using C = double;
    static __device__ __forceinline__ double bload(rsrc_t r, uint32_t off) { return bld<double>(r, off); }
    static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, double v) { bst(r, off, v); }
    static __device__ __forceinline__ double ld(const double *p) { return gld(p); }
    static __device__ __forceinline__ void st(double *p, double v) { gst(p, v); }
    static __device__ __forceinline__ double rnd(double v) { return v; }
};
template <> struct Traits<float> {
    using C = float;
    static __device__ __forceinline__ float bload(rsrc_t r, uint32_t off) { return bld<float>(r, off); }
    static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, float v) { bst(r, off, v); }
    static __device__ __forceinline__ float ld(const float *p) { return gld(p); }
    static __device__ __forceinline__ void st(float *p, float v) { gst(p, v); }
    static __device__ __forceinline__ float rnd(float v) { return v; }
};
template <> struct Traits<bf16_t> {
    using C = float;
    static __device__ __forceinline__ float bload(rsrc_t r, uint32_t off) { return bf16_to_f32(bld<bf16_t>(r, off)); }
    static __device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, float v)
    {
        bst(r, off, (bf16_t)(__float_as_uint(v) >> 16));
    }
    static __device__ __forceinline__ float ld(const bf16_t *p) { return bf16_to_f32(gld(p)); }
    // values are rounded by rnd() when computed, so the store is exact
    static __device__ __forceinline__ void st(bf16_t *p, float v) { gst(p, (bf16_t)(__float_as_uint(v) >> 16)); }
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
// Work items write their partial sums (rr = sum r^2, ff = sum f^2) to
// partials[2 slot + {0, 1}] with plain stores; the next kernel on the stream
// (k_norm_finish, one wavefront per system) reduces a system's slots in a
// fixed order -- lane l adds slots l, l+64, ..., then a fixed butterfly
// across the lanes -- so the total does not depend on scheduling, and applies
// the stop test:
//   rel = sqrt(rr / ff); hist[nres] = rel; done = 1 if rel <= tol,
//   2 if not finite, 3 if nres reached the cycle limit.
// `first` marks the norm before the first cycle: it also fixes ff = ||f||^2.
__device__ inline void put_partial(double *partials, int slot, double rr, double ff)
{
    if ((threadIdx.x & 63) == 0) {
        partials[2 * slot] = rr;
        partials[2 * slot + 1] = ff;
    }
}

}  // namespace mgx
