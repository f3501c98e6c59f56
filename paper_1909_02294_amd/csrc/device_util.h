// Device helpers shared by the gfx950 kernel sources: wave geometry,
// wave-uniform loads through the scalar unit and FP16 unpacking.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "ivde_internal.h"

namespace ivde {
namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ float h_lo(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w & 0xffffu))); }
__device__ __forceinline__ float h_hi(uint32_t w) { return __half2float(__ushort_as_half((unsigned short)(w >> 16))); }

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

}  // namespace
}  // namespace ivde
