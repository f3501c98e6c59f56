// Calibration kernels for the sweep's roofline (libivde_calib.so, used by the
// benchmark only): the issue cost of each VALU instruction class the sweep
// uses, and the rate at which the texture path returns buffer gathers that
// hit the L1 cache.  Every kernel runs at full occupancy (8 waves per SIMD)
// with eight independent dependency chains per wave, so issue and not
// latency sets its time; the shader clock during the run is measured from the
// ratio of the shader-cycle counter (s_memtime) to the 100 MHz real-time
// counter (s_memrealtime).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kBlocks = 256 * 8 * 2;      // 8 waves per SIMD on 256 CUs, twice over
constexpr int kChains = 8;
constexpr int kPerIter = 4 * kChains;     // instructions of the class per loop iteration

// One instruction of class OP on chain value a (float) or u (integer).
template <int OP>
__device__ __forceinline__ void op(float &a, uint32_t &u, uint64_t m, float b, float c, uint32_t k)
{
    if constexpr (OP == 0) asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    else if constexpr (OP == 1) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    else if constexpr (OP == 2) asm volatile("v_mul_f32 %0, %0, %1" : "+v"(a) : "v"(b));
    else if constexpr (OP == 3) asm volatile("v_add_f32 %0, %0, %1" : "+v"(a) : "v"(b));
    else if constexpr (OP == 4) asm volatile("v_sub_f32 %0, %0, %1" : "+v"(a) : "v"(b));
    else if constexpr (OP == 5) asm volatile("v_mov_b32 %0, %1" : "=v"(a) : "v"(u));
    else if constexpr (OP == 6) asm volatile("v_add_f32_e64 %0, |%0|, |%1|" : "+v"(a) : "v"(b));
    else if constexpr (OP == 7) asm volatile("v_fma_mix_f32 %0, %1, %2, %0 op_sel_hi:[1,0,0]" : "+v"(a) : "v"(k), "v"(b));
    else if constexpr (OP == 8) asm volatile("v_med3_f32 %0, %0, %1, %2" : "+v"(a) : "v"(b), "v"(c));
    else if constexpr (OP == 9) asm volatile("v_fract_f32 %0, %0" : "+v"(a));
    else if constexpr (OP == 10) asm volatile("v_cvt_i32_f32 %0, %1" : "=v"(u) : "v"(a));
    else if constexpr (OP == 11) {
        uint64_t r;
        asm volatile("v_cmp_eq_f32_e64 %0, %1, %2" : "=s"(r) : "v"(a), "v"(b));
        asm volatile("" ::"s"(r));
    } else if constexpr (OP == 12) asm volatile("v_cndmask_b32_e64 %0, 0, %0, %1" : "+v"(a) : "s"(m));
    else if constexpr (OP == 13) asm volatile("v_rcp_f32 %0, %0" : "+v"(a));
    else if constexpr (OP == 14) asm volatile("v_mad_u32_u24 %0, %0, %1, %1" : "+v"(u) : "v"(k));
    else if constexpr (OP == 15) asm volatile("v_lshlrev_b32 %0, 3, %0" : "+v"(u));
    else if constexpr (OP == 16) {
        uint64_t cy;
        asm volatile("v_addc_co_u32_e64 %0, %1, %0, %2, %3" : "+v"(u), "=s"(cy) : "v"(k), "s"(m));
        asm volatile("" ::"s"(cy));
    } else if constexpr (OP == 17) asm volatile("v_add_u32 %0, %0, %1" : "+v"(u) : "v"(k));
    else if constexpr (OP == 18)   // the high 16-bit word of u to FP32 (texels of 16-bit code values)
        asm volatile("v_cvt_f32_u32_sdwa %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1"
                     : "=v"(a) : "v"(u));
}

template <int OP>
__global__ __launch_bounds__(256) void k_issue(float *out, int iters, unsigned long long *clk)
{
    float a[kChains];
    uint32_t u[kChains];
    for (int i = 0; i < kChains; ++i) {
        a[i] = (float)(threadIdx.x + i) * 1e-3f;
        u[i] = threadIdx.x + i;
    }
    const float b = 1.0001f, c = 0.5f;
    const uint32_t k = threadIdx.x;
    const uint64_t m = 0x5555555555555555ull;
    unsigned long long t0 = 0, r0 = 0;
    if (threadIdx.x == 0) {
        t0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int rep = 0; rep < 4; ++rep)
#pragma unroll
            for (int i = 0; i < kChains; ++i) op<OP>(a[i], u[i], m, b, c, k);
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk[0] = __builtin_amdgcn_s_memtime() - t0;
        clk[1] = __builtin_amdgcn_s_memrealtime() - r0;
    }
    float sum = 0.f;
    for (int i = 0; i < kChains; ++i) sum += a[i] + (float)u[i];
    out[blockIdx.x * 256 + threadIdx.x] = sum;
}

// Gathers of 16 bytes per lane from 8-byte cells, lanes three cells apart
// (as the sweep's lanes walk an epipolar line), from a 32 KB window.
constexpr int kSpanCells = 4096;

__global__ __launch_bounds__(256) void k_gather(const unsigned char *buf, int iters, unsigned *out,
                                                unsigned long long *clk)
{
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char *>(buf), (short)0,
                                                                       kSpanCells * 8 + 64, (int)0x00020000u);
    unsigned acc = 0;
    int base = (wave * 977) & (kSpanCells - 1);
    unsigned long long t0 = 0, r0 = 0;
    if (threadIdx.x == 0) {
        t0 = __builtin_amdgcn_s_memtime();
        r0 = __builtin_amdgcn_s_memrealtime();
    }
    for (int it = 0; it < iters; ++it) {
        const int c0 = (base + lane * 3) & (kSpanCells - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cell = (c0 + q * 53) & (kSpanCells - 1);
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, cell * 8, 0, 0);
            acc ^= v[0] ^ v[1] ^ v[2] ^ v[3];
        }
        base = (base + 97) & (kSpanCells - 1);
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk[0] = __builtin_amdgcn_s_memtime() - t0;
        clk[1] = __builtin_amdgcn_s_memrealtime() - r0;
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc;
}

struct Buffers {
    float *out = nullptr;
    unsigned *uout = nullptr;
    unsigned char *src = nullptr;
    unsigned long long *clk = nullptr;
};

template <int OP>
hipError_t launch_issue(const Buffers &b, int iters, hipStream_t s)
{
    hipLaunchKernelGGL(k_issue<OP>, dim3(kBlocks), dim3(256), 0, s, b.out, iters, b.clk);
    return hipGetLastError();
}

hipError_t launch_class(int cls, const Buffers &b, int iters, hipStream_t s)
{
    switch (cls) {
    case 0: return launch_issue<0>(b, iters, s);
    case 1: return launch_issue<1>(b, iters, s);
    case 2: return launch_issue<2>(b, iters, s);
    case 3: return launch_issue<3>(b, iters, s);
    case 4: return launch_issue<4>(b, iters, s);
    case 5: return launch_issue<5>(b, iters, s);
    case 6: return launch_issue<6>(b, iters, s);
    case 7: return launch_issue<7>(b, iters, s);
    case 8: return launch_issue<8>(b, iters, s);
    case 9: return launch_issue<9>(b, iters, s);
    case 10: return launch_issue<10>(b, iters, s);
    case 11: return launch_issue<11>(b, iters, s);
    case 12: return launch_issue<12>(b, iters, s);
    case 13: return launch_issue<13>(b, iters, s);
    case 14: return launch_issue<14>(b, iters, s);
    case 15: return launch_issue<15>(b, iters, s);
    case 16: return launch_issue<16>(b, iters, s);
    case 17: return launch_issue<17>(b, iters, s);
    case 18: return launch_issue<18>(b, iters, s);
    default: return hipErrorInvalidValue;
    }
}

const char *const kNames[] = {"v_fma_f32", "v_fmac_f32", "v_mul_f32", "v_add_f32", "v_sub_f32", "v_mov_b32",
                              "v_add_f32_abs", "v_fma_mix_f32", "v_med3_f32", "v_fract_f32", "v_cvt_i32_f32",
                              "v_cmp_f32", "v_cndmask_b32", "v_rcp_f32", "v_mad_u32_u24", "v_lshlrev_b32",
                              "v_addc_co_u32", "v_add_u32", "v_cvt_f32_u32_sdwa"};
constexpr int kClasses = 19;

}  // namespace

extern "C" {

int ivde_calib_classes(void) { return kClasses; }

const char *ivde_calib_class_name(int cls) { return cls >= 0 && cls < kClasses ? kNames[cls] : ""; }

// Runs class `cls` (or, with cls = -1, the gather kernel) twice and times the
// second run.  Outputs: cycles per wave-level instruction (or gather) per
// SIMD for the VALU classes and per CU for the gathers, at the shader clock
// measured during the run (GHz).  Returns 0 on success, -1 on a HIP error.
int ivde_calibrate(int cls, double *cycles, double *clock_ghz, double *ms)
{
    Buffers b;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = -1;
    const int iters = cls < 0 ? 512 : 2048;
    if (hipMalloc(&b.out, sizeof(float) * kBlocks * 256) != hipSuccess) goto done;
    if (hipMalloc(&b.uout, sizeof(unsigned) * kBlocks * 256) != hipSuccess) goto done;
    if (hipMalloc(&b.src, kSpanCells * 8 + 64) != hipSuccess) goto done;
    if (hipMalloc(&b.clk, 16) != hipSuccess) goto done;
    if (hipMemset(b.src, 1, kSpanCells * 8 + 64) != hipSuccess) goto done;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
    for (int rep = 0; rep < 2; ++rep) {
        if (hipEventRecord(e0, nullptr) != hipSuccess) goto done;
        if (cls < 0) {
            hipLaunchKernelGGL(k_gather, dim3(kBlocks), dim3(256), 0, nullptr, b.src, iters, b.uout, b.clk);
            if (hipGetLastError() != hipSuccess) goto done;
        } else if (launch_class(cls, b, iters, nullptr) != hipSuccess) {
            goto done;
        }
        if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) goto done;
    }
    {
        float t = 0.f;
        unsigned long long h[2] = {0, 0};
        if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) goto done;
        if (hipMemcpy(h, b.clk, 16, hipMemcpyDeviceToHost) != hipSuccess) goto done;
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            goto done;
        const double ghz = h[1] ? (double)h[0] / ((double)h[1] / 100e6) / 1e9 : 0.0;
        const double waves = kBlocks * 4.0;
        const double seconds = t * 1e-3;
        if (cls < 0) {
            const double loads = waves * iters * 4.0;
            *cycles = seconds * ghz * 1e9 * cus / loads;                 // per CU
        } else {
            const double instr = waves * iters * (double)kPerIter;
            *cycles = seconds * ghz * 1e9 * cus * 4.0 / instr;           // per SIMD
        }
        *clock_ghz = ghz;
        *ms = t;
        rc = 0;
    }
done:
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(b.out);
    (void)hipFree(b.uout);
    (void)hipFree(b.src);
    (void)hipFree(b.clk);
    return rc;
}

}  // extern "C"
