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

}  // namespace tno
