// Device helpers shared by the gfx950 kernel sources: wave geometry,
// wave-uniform loads through the scalar unit, FP16 unpacking and global
// loads and stores through pointers read from a view descriptor.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "ivde_internal.h"

namespace ivde {
namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Wave-wide minimum and sum through DPP lane moves (no LDS traffic): row
// shifts by 1, 2, 4 and 8 leave each 16-lane row's result in its lane 15,
// the row broadcasts 15 and 31 carry it to lane 63, which is returned to
// every lane.  Every lane of the wave must be active.  `old` is what a lane
// reads when its source lane lies outside the row or its row is masked off.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp(int old, int v)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}

__device__ __forceinline__ int wave_min_i32(int v)
{
    v = min(v, dpp<0x111, 0xf>(v, v));   // row_shr:1
    v = min(v, dpp<0x112, 0xf>(v, v));   // row_shr:2
    v = min(v, dpp<0x114, 0xf>(v, v));   // row_shr:4
    v = min(v, dpp<0x118, 0xf>(v, v));   // row_shr:8
    v = min(v, dpp<0x142, 0xa>(v, v));   // row_bcast:15 into rows 1 and 3
    v = min(v, dpp<0x143, 0xc>(v, v));   // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t u)
{
    int v = (int)u;
    v = (int)((uint32_t)v + (uint32_t)dpp<0x111, 0xf>(0, v));
    v = (int)((uint32_t)v + (uint32_t)dpp<0x112, 0xf>(0, v));
    v = (int)((uint32_t)v + (uint32_t)dpp<0x114, 0xf>(0, v));
    v = (int)((uint32_t)v + (uint32_t)dpp<0x118, 0xf>(0, v));
    v = (int)((uint32_t)v + (uint32_t)dpp<0x142, 0xa>(0, v));
    v = (int)((uint32_t)v + (uint32_t)dpp<0x143, 0xc>(0, v));
    return (uint32_t)__builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ float h_lo(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w & 0xffffu))); }
__device__ __forceinline__ float h_hi(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w >> 16))); }

// One 16-bit channel of a packed texel or colour word as FP32.  Channels
// hold halves (code values up to 11 bits, exact) or, with U16, the unsigned
// 16-bit code values themselves (any bit depth up to 16, exact).
template <bool U16>
__device__ __forceinline__ float ch_lo(uint32_t w)
{
    if constexpr (U16)
        return (float)(w & 0xffffu);
    else
        return h_lo(w);
}
template <bool U16>
__device__ __forceinline__ float ch_hi(uint32_t w)
{
    if constexpr (U16)
        return (float)(w >> 16);
    else
        return h_hi(w);
}

// Wave-uniform loads through the scalar unit: the address must be uniform
// and the data must not be written by the running kernel.
#define IVDE_AS4 __attribute__((address_space(4)))
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ T ldu(const T *p) { return *(const IVDE_AS4 T *)(p); }
__device__ __forceinline__ f32x4 ldu4(const float *p) { return *(const IVDE_AS4 f32x4 *)(p); }
__device__ __forceinline__ Task ldu_task(const Task *p)
{
    const i32x4 v = *(const IVDE_AS4 i32x4 *)(p);
    Task t;
    t.problem = v.x;
    t.view = v.y;
    t.seg = v.z;
    t.lblock = v.w;
    return t;
}

// Global-memory access through pointers read from a descriptor (the
// compiler cannot tell their address space by itself).
#define IVDE_AS1 __attribute__((address_space(1)))
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ T ldg(const T *p) { return *(const IVDE_AS1 T *)(p); }
template <typename T>
__device__ __forceinline__ void stg(T *p, T v) { *(IVDE_AS1 T *)(p) = v; }
__device__ __forceinline__ float2 ldg(const float2 *p)
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    const f32x2 v = *(const IVDE_AS1 f32x2 *)(p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ uint2 ldg2u(const uint2 *p)
{
    const u32x2 v = *(const IVDE_AS1 u32x2 *)(p);
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ float4 ldg(const float4 *p)
{
    const f32x4 v = *(const IVDE_AS1 f32x4 *)(p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void stg(float4 *p, const float4 &v)
{
    f32x4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *(IVDE_AS1 f32x4 *)(p) = w;
}
__device__ __forceinline__ void stg(uint2 *p, const uint2 &v)
{
    u32x2 w;
    w.x = v.x;
    w.y = v.y;
    *(IVDE_AS1 u32x2 *)(p) = w;
}

// A view's planes, read once per wave into scalar registers, so stores of
// the kernel do not force the descriptor to be read again.
struct Planes {
    const void *p[3];
    int64_t pitch[3];
    int k;       // chroma shift
    bool wide;   // 16-bit samples
};

__device__ __forceinline__ Planes planes_of(const Problem *P, const ViewDesc *vd)
{
    Planes pl;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        pl.p[i] = ldu(&vd->plane[i]);
        pl.pitch[i] = ldu(&vd->pitch[i]);
    }
    pl.k = ldu(&P->chroma_shift);
    pl.wide = ldu(&P->bit_depth) > 8;
    return pl;
}

__device__ __forceinline__ uint32_t plane_u(const Planes &pl, int i, int64_t off)
{
    return pl.wide ? (uint32_t)ldg(static_cast<const uint16_t *>(pl.p[i]) + off)
                   : (uint32_t)ldg(static_cast<const uint8_t *>(pl.p[i]) + off);
}

__device__ __forceinline__ float plane_at(const Planes &pl, int i, int64_t off) { return (float)plane_u(pl, i, off); }

// Y, Cb, Cr of pixel (x, y), chroma at (x >> k, y >> k).
__device__ __forceinline__ void yuv_at(const Planes &pl, int x, int y, float &c0, float &c1, float &c2)
{
    c0 = plane_at(pl, 0, (int64_t)y * pl.pitch[0] + x);
    c1 = plane_at(pl, 1, (int64_t)(y >> pl.k) * pl.pitch[1] + (x >> pl.k));
    c2 = plane_at(pl, 2, (int64_t)(y >> pl.k) * pl.pitch[2] + (x >> pl.k));
}

}  // namespace
}  // namespace ivde
