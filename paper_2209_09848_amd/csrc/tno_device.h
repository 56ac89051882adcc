// tno_device.h -- device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tno_internal.h"

namespace tno {

typedef __attribute__((address_space(4))) int32_t cint32_t;   // constant address space
typedef __attribute__((address_space(3))) float lfloat_t;      // LDS
// Word 3 of a raw (unformatted, stride 0) buffer resource on gfx9-family GPUs.
constexpr int BUF_DWORD3 = 0x00020000;

__device__ __forceinline__ uint32_t ordered_key(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key_to_float(uint32_t k)
{
    uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(u);
}

// Work-item index of block b when items are dealt to the 8 XCDs in contiguous
// ranges: consecutive blocks go round-robin to XCDs, so block b runs on XCD
// b % 8; giving each XCD a contiguous item range keeps the trajectories of one
// tile (which read the same frame region) on one XCD and its L2.
__device__ __forceinline__ int xcd_item(int b, int nblocks)
{
    int per = nblocks >> 3;
    return (b & 7) * per + (b >> 3);
}

// The request entry and work item of this block of a serving-loop step;
// false for the padding blocks of an entry (its count is below nblk).
// The step's tables are read-only for the whole launch: they are read through
// the constant address space, so that the entry and the request's arguments
// are scalar loads into scalar registers, as a single-request launch's are.
// (The host compilation pass, which only parses device functions, takes the
// plain reads: the address-space-qualified copies exist in device code only.)
__device__ __forceinline__ StepEntry step_entry(const StepArgs &s, int r)
{
#if defined(__HIP_DEVICE_COMPILE__)
    typedef __attribute__((address_space(4))) const StepEntry centry_t;
    return ((centry_t *)s.ent)[r];
#else
    return s.ent[r];
#endif
}

__device__ __forceinline__ SearchArgs step_args(const StepArgs &s, int r)
{
#if defined(__HIP_DEVICE_COMPILE__)
    typedef __attribute__((address_space(4))) const SearchArgs cargs_t;
    return ((cargs_t *)s.reqs)[r];
#else
    return s.reqs[r];
#endif
}

__device__ __forceinline__ bool step_item(const StepArgs &s, int &r, int &item)
{
    const int b = blockIdx.x;
    r = 0;
    while (r + 1 < s.n && b >= step_entry(s, r + 1).begin)
        ++r;
    const StepEntry e = step_entry(s, r);
    const int li = xcd_item(b - e.begin, e.nblk);
    item = e.item0 + li;
    return li < e.count;
}

__host__ inline int xcd_grid(int n_items)
{
    int per = (n_items + 7) / 8;
    return per * 8;
}

__device__ __forceinline__ float decode_e4m3(uint32_t c)
{
    // E4M3fn code -> binary16 with the same sign/exponent/mantissa bits shifted
    // into place: value(binary16) = value(E4M3) * 2^-8 for normals and
    // subnormals alike; the caller's scale absorbs the 2^8.
    uint16_t hb = (uint16_t)(((c & 0x80u) << 8) | ((c & 0x7Fu) << 7));
    _Float16 hv;
    __builtin_memcpy(&hv, &hb, 2);
    return (float)hv;
}

// One staged group (4 image columns) as loaded, before decoding.
constexpr int SRC_Z = -1;   // source of a search's window: the staged FP32 stack; else the dtype read in place

template <int SRC>
struct Raw {
    float4 z;                  // SRC_Z: the staged values
};
template <>
struct Raw<TNO_F32> {
    float4 r, iv;
};
template <>
struct Raw<TNO_BF16> {
    uint2 c;
    float4 iv;
    float s;
};
template <>
struct Raw<TNO_F16> {
    uint2 c;
    float4 iv;
    float s;
};
template <>
struct Raw<TNO_FP8_E4M3> {
    uint32_t c;
    float4 iv;
    float s;
};

template <int SRC>
constexpr int src_bytes() { return SRC == SRC_Z || SRC == TNO_F32 ? 4 : SRC == TNO_FP8_E4M3 ? 1 : 2; }

template <class V>
__device__ __forceinline__ float4 as_f4(const V &v)
{
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]), __uint_as_float(v[3]));
}

// Decode a staged group into image column order: Z reordered; otherwise
// (code * scale) * ivar per column, rounded as the staging of Z rounds them.
template <int SRC>
__device__ __forceinline__ float4 decode_group(const Raw<SRC> &g)
{
    if constexpr (SRC == SRC_Z) {
        return make_float4(g.z.x, g.z.z, g.z.y, g.z.w);   // Z holds 4g, 4g+2, 4g+1, 4g+3
    } else if constexpr (SRC == TNO_F32) {
        return make_float4(g.r.x * g.iv.x, g.r.y * g.iv.y, g.r.z * g.iv.z, g.r.w * g.iv.w);
    } else {
        float r[4];
        if constexpr (SRC == TNO_BF16) {
            r[0] = __uint_as_float(g.c.x << 16) * g.s;
            r[1] = __uint_as_float(g.c.x & 0xFFFF0000u) * g.s;
            r[2] = __uint_as_float(g.c.y << 16) * g.s;
            r[3] = __uint_as_float(g.c.y & 0xFFFF0000u) * g.s;
        } else if constexpr (SRC == TNO_F16) {
            const uint32_t c[4] = {g.c.x & 0xFFFFu, g.c.x >> 16, g.c.y & 0xFFFFu, g.c.y >> 16};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint16_t hb = (uint16_t)c[e];
                _Float16 hv;
                __builtin_memcpy(&hv, &hb, 2);
                r[e] = (float)hv * g.s;
            }
        } else {
            const float s8 = g.s * 256.0f;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                r[e] = decode_e4m3((g.c >> (8 * e)) & 0xFFu) * s8;
        }
        return make_float4(r[0] * g.iv.x, r[1] * g.iv.y, r[2] * g.iv.z, r[3] * g.iv.w);
    }
}

}  // namespace tno
