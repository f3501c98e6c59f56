// gfx950 kernels of libivde: image packing, segment index, spatial work
// list, the plane-sweep cost kernel (plain and persistent), argmin and the
// temporal task compaction.
//
// The sweep kernel maps one wavefront to one (view, segment, label block)
// task.  Lanes are labels: lane i of block b owns labels 64 J b + 64 j + i,
// j < J.  The wave walks the segment's pixels in a fixed order (raster order
// inside the segment), so per-pixel data are wave-uniform and come through
// scalar loads, and every lane accumulates its own labels' sums without
// cross-lane traffic.  The projection of a pixel into a target is affine in
// the label's inverse depth sigma (h = H p~ + sigma (g . p~) e), so each
// (pixel, label) costs three FMAs and a reciprocal before sampling.  The
// texel gathers of the 64 lanes fall along the pixel's epipolar line in the
// target and go through buffer loads (out-of-range reads return zero, never
// fault).  Per-row results are produced entirely inside one wave in a fixed
// order, so plain, batched and served launches give bitwise equal costs.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "ivde_internal.h"

namespace ivde {

namespace {

constexpr int kWave = 64;
constexpr uint32_t kRsrcWord3 = 0x00020000u;   // raw buffer, gfx9 family

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             (int)kRsrcWord3);
}

__device__ __forceinline__ float sample_plane(const void *p, int64_t off, int bit_depth)
{
    if (bit_depth <= 8) return (float)static_cast<const uint8_t *>(p)[off];
    return (float)static_cast<const uint16_t *>(p)[off];
}

// ------------------------------------------------------------------ upload
struct UploadChunk {
    unsigned char bytes[2048];
};

__global__ void k_upload(unsigned char *__restrict__ dst, UploadChunk c, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.bytes[i];
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int32_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------ prepare
// Reset the per-view index: counts 0, bbox empty, band counts 0.
__global__ void k_index_init(const Problem *__restrict__ P)
{
    const ViewDesc &v = P->views[blockIdx.y];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < v.S) {
        v.counts[i] = 0;
        v.bbox[4 * i + 0] = 0x7fffffff;
        v.bbox[4 * i + 1] = 0x7fffffff;
        v.bbox[4 * i + 2] = -1;
        v.bbox[4 * i + 3] = -1;
    }
    if (i < 2 * v.n_bands) v.band_count[i] = 0;
}

// Packed texels: (W + 1) x (H + 1) of {Y, Cb, Cr, 0}, chroma replicated to
// full resolution (pixel (x, y) owns chroma (x >> k, y >> k)), zero border
// column and row so a bilinear pair read at x0 = W - 1 stays in bounds.
template <typename TexT>
__global__ void k_pack(const Problem *__restrict__ P)
{
    const ViewDesc &v = P->views[blockIdx.z];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    if (x > v.W || y > v.H) return;
    const int k = P->chroma_shift, b = P->bit_depth;
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
    if (x < v.W && y < v.H) {
        c0 = sample_plane(v.plane[0], (int64_t)y * v.pitch[0] + x, b);
        c1 = sample_plane(v.plane[1], (int64_t)(y >> k) * v.pitch[1] + (x >> k), b);
        c2 = sample_plane(v.plane[2], (int64_t)(y >> k) * v.pitch[2] + (x >> k), b);
    }
    TexT *t = static_cast<TexT *>(v.tex) + (int64_t)y * v.tex_pitch + x;
    if constexpr (sizeof(TexT) == 8) {
        __half2 a = __floats2half2_rn(c0, c1);
        __half2 bb = __floats2half2_rn(c2, 0.f);
        uint2 w;
        w.x = __builtin_bit_cast(uint32_t, a);
        w.y = __builtin_bit_cast(uint32_t, bb);
        *reinterpret_cast<uint2 *>(t) = w;
    } else {
        *reinterpret_cast<float4 *>(t) = make_float4(c0, c1, c2, 0.f);
    }
}

// Pixel counts and boxes.  A wave covers 64 consecutive pixels of one row;
// runs of equal ids are merged so one lane per run issues the atomics.
__global__ void k_seg_count(const Problem *__restrict__ P)
{
    const ViewDesc &v = P->views[blockIdx.z];
    const int lane = threadIdx.x;
    const int x = blockIdx.x * kWave + lane;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const bool in = x < v.W && y < v.H;
    int id = in ? v.seg[(int64_t)y * v.seg_pitch + x] : -1;
    if (in && (id < 0 || id >= v.S)) {
        atomicOr(P->flag, 1);
        id = -1;
    }
    const int prev = __shfl_up(id, 1);
    const int next = __shfl_down(id, 1);
    const bool head = id >= 0 && (lane == 0 || prev != id);
    const bool tail = id >= 0 && (lane == kWave - 1 || next != id);
    const uint64_t tails = __ballot(tail);
    if (head) {
        const uint64_t after = tails & (~0ull << lane);
        const int end = __builtin_ctzll(after);
        const int len = end - lane + 1;
        atomicAdd(&v.counts[id], len);
        atomicMin(&v.bbox[4 * id + 0], x);
        atomicMin(&v.bbox[4 * id + 1], y);
        atomicMax(&v.bbox[4 * id + 2], x + len - 1);
        atomicMax(&v.bbox[4 * id + 3], y);
    }
}

// Exclusive scan of the counts, one 1024-thread block per view.
__global__ __launch_bounds__(1024) void k_scan(const Problem *__restrict__ P)
{
    const ViewDesc &v = P->views[blockIdx.x];
    __shared__ int wsum[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int carry = 0;
    for (int base = 0; base < v.S; base += 1024) {
        const int i = base + threadIdx.x;
        const int c = i < v.S ? v.counts[i] : 0;
        int x = c;
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        if (wave == 0) {
            int s = lane < 16 ? wsum[lane] : 0;
            for (int d = 1; d < 16; d <<= 1) {
                const int y = __shfl_up(s, d);
                if (lane >= d) s += y;
            }
            if (lane < 16) wsum[lane] = s;
        }
        __syncthreads();
        const int excl = carry + (wave > 0 ? wsum[wave - 1] : 0) + x - c;
        if (i < v.S) v.offsets[i] = excl;
        const int total = wsum[15];
        __syncthreads();
        carry += total;
    }
    if (threadIdx.x == 0) v.offsets[v.S] = carry;
}

// Pixel records in raster order inside each segment: one wave scans its
// segment's box row by row and compacts the member pixels with a ballot.
__global__ void k_seg_fill(const Problem *__restrict__ P)
{
    const ViewDesc &v = P->views[blockIdx.y];
    const int lane = lane_id();
    const int s = uniform(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    if (s >= v.S) return;
    const int x0 = v.bbox[4 * s + 0], y0 = v.bbox[4 * s + 1];
    const int x1 = v.bbox[4 * s + 2], y1 = v.bbox[4 * s + 3];
    if (x1 < x0) return;   // empty segment
    const int k = P->chroma_shift, b = P->bit_depth;
    const int base = v.offsets[s];
    const int cap = v.offsets[s + 1];
    const float g0 = v.g[0], g1 = v.g[1], g2 = v.g[2];
    int run = 0;
    for (int y = y0; y <= y1; ++y) {
        for (int xb = x0; xb <= x1; xb += kWave) {
            const int x = xb + lane;
            const bool m = x <= x1 && v.seg[(int64_t)y * v.seg_pitch + x] == s;
            const uint64_t bal = __ballot(m);
            const int pos = base + run + __builtin_popcountll(bal & ((1ull << lane) - 1));
            if (m && pos < cap) {
                const float fx = (float)x, fy = (float)y;
                float4 r0, r1;
                r0.x = fx;
                r0.y = fy;
                r0.z = fmaf(g0, fx, fmaf(g1, fy, g2));
                r0.w = sample_plane(v.plane[0], (int64_t)y * v.pitch[0] + x, b);
                r1.x = sample_plane(v.plane[1], (int64_t)(y >> k) * v.pitch[1] + (x >> k), b);
                r1.y = sample_plane(v.plane[2], (int64_t)(y >> k) * v.pitch[2] + (x >> k), b);
                r1.z = 0.f;
                r1.w = 0.f;
                float4 *dst = reinterpret_cast<float4 *>(v.pixrec) + 2 * (int64_t)pos;
                dst[0] = r0;
                dst[1] = r1;
            }
            run += __builtin_popcountll(bal);
        }
    }
}

// ------------------------------------------------------------------ work list
__device__ __forceinline__ int segment_band(const ViewDesc &v, int s)
{
    const int y0 = v.bbox[4 * s + 1], y1 = v.bbox[4 * s + 3];
    if (y1 < y0) return 0;
    const int b = ((y0 + y1) >> 1) / kBand;
    return b < v.n_bands ? b : v.n_bands - 1;
}

__global__ void k_band_count(const Problem *__restrict__ P)
{
    const ViewDesc &v = P->views[blockIdx.y];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= v.S) return;
    atomicAdd(&v.band_count[segment_band(v, s)], 1);
}

// Band cursors: exclusive scan of the band counts (one thread per view; a
// few dozen bands).
__global__ void k_band_scan(const Problem *__restrict__ P)
{
    const int vi = blockIdx.x * blockDim.x + threadIdx.x;
    if (vi >= P->n_views) return;
    const ViewDesc &v = P->views[vi];
    int acc = 0;
    for (int b = 0; b < v.n_bands; ++b) {
        v.band_count[v.n_bands + b] = acc;
        acc += v.band_count[b];
    }
}

// Tasks of one problem: view-major, spatial bands inside a view (segments
// near each other run near each other in time), label blocks innermost.
// The order inside a band depends on atomics; no result depends on it.
__global__ void k_task_fill(const Problem *__restrict__ P, int problem_index, Task *__restrict__ tasks)
{
    const int vi = blockIdx.y;
    const ViewDesc &v = P->views[vi];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= v.S) return;
    const int nb = P->n_lblocks;
    const int pos = atomicAdd(&v.band_count[v.n_bands + segment_band(v, s)], 1);
    Task *t = tasks + (v.row0 + pos) * nb;
    for (int b = 0; b < nb; ++b) {
        Task tk;
        tk.problem = problem_index;
        tk.view = vi;
        tk.seg = s;
        tk.lblock = b;
        t[b] = tk;
    }
}

// ------------------------------------------------------------------ sweep
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

// a * b + c on the 24-bit multiplier (operands below 2^24)
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// One task: labels [64 J b, 64 J (b + 1)) of row (view, seg).
template <int J, bool BIL, bool TEXF32, bool F16OUT>
__device__ __forceinline__ void sweep_task(const Problem *__restrict__ P, const Task task)
{
    constexpr int kTexB = TEXF32 ? 16 : 8;
    const int lane = lane_id();
    const int c = task.view, s = task.seg;
    const int L = ldu(&P->L), n = ldu(&P->n_views);
    const ViewDesc *views = ldu(&P->views);
    const PairConst *pairs = ldu(&P->pairs);
    const float *sigma = ldu(&P->sigma);
    const float norm = ldu(&P->norm);
    void *cost = ldu(&P->cost);
    const ViewDesc *vc = views + c;
    const int32_t *offsets = ldu(&vc->offsets);
    const int p0 = ldu(offsets + s), p1 = ldu(offsets + s + 1);
    const float *pix = ldu(&vc->pixrec);
    const int nt = ldu(&vc->n_targets);
    const int64_t row0 = ldu(&vc->row0);

    int lab[J];
    float sig[J], best[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        lab[j] = task.lblock * (kWave * J) + j * kWave + lane;
        sig[j] = lab[j] < L ? sigma[c * L + lab[j]] : 0.f;
        best[j] = __builtin_inff();
    }

    for (int ti = 0; ti < nt; ++ti) {
        const int c2 = ldu(&vc->targets[ti]);
        const ViewDesc *vt = views + c2;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(ldu(&vt->tex), ldu(&vt->tex_bytes));
        const int tW = ldu(&vt->W), tH = ldu(&vt->H);
        const float Wm1 = (float)(tW - 1), Hm1 = (float)(tH - 1);
        const uint32_t tp = (uint32_t)ldu(&vt->tex_pitch);
        const int rowB = (int)tp * kTexB;
        const float *pc = reinterpret_cast<const float *>(pairs + c * n + c2);
        const f32x4 ha = ldu4(pc), hb = ldu4(pc + 4), hc = ldu4(pc + 8);
        const float H0 = ha.x, H1 = ha.y, H2 = ha.z, H3 = ha.w;
        const float H4 = hb.x, H5 = hb.y, H6 = hb.z, H7 = hb.w;
        const float H8 = hc.x, e0 = hc.y, e1 = hc.z, e2 = hc.w;

        float acc[J];
        uint64_t acci[J];
        int cnt[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            acc[j] = 0.f;
            acci[j] = 0;
            cnt[j] = 0;
        }

        for (int i = p0; i < p1; ++i) {
            const f32x4 r0 = ldu4(pix + 8 * (int64_t)i);
            const f32x4 r1 = ldu4(pix + 8 * (int64_t)i + 4);
            const float x = r0.x, y = r0.y, gp = r0.z;
            const float ry = r0.w, ru = r1.x, rv = r1.y;
            const float qx = fmaf(H0, x, fmaf(H1, y, H2));
            const float qy = fmaf(H3, x, fmaf(H4, y, H5));
            const float qz = fmaf(H6, x, fmaf(H7, y, H8));
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const float w = sig[j] * gp;          // 1 / tau: positive in front of view c
                const float hx = fmaf(w, e0, qx);
                const float hy = fmaf(w, e1, qy);
                const float hz = fmaf(w, e2, qz);
                const float r = __builtin_amdgcn_rcpf(hz);
                const float u = hx * r, v = hy * r;
                bool valid = (w > 0.f) & (hz > 0.f);
                if constexpr (BIL) {
                    const float uc = __builtin_amdgcn_fmed3f(u, 0.f, Wm1);
                    const float vc2 = __builtin_amdgcn_fmed3f(v, 0.f, Hm1);
                    valid &= (fabsf(u - uc) <= kEdge) & (fabsf(v - vc2) <= kEdge);
                    const uint32_t x0 = (uint32_t)(int)uc, y0 = (uint32_t)(int)vc2;
                    const float ax = __builtin_amdgcn_fractf(uc), ay = __builtin_amdgcn_fractf(vc2);
                    const float bx = 1.f - ax, by = 1.f - ay;
                    const float w00 = bx * by, w01 = ax * by, w10 = bx * ay, w11 = ax * ay;
                    const int off = (int)(mad_u24(y0, tp, x0) * kTexB);
                    float tY, tU, tV;
                    if constexpr (!TEXF32) {
                        // texels (x0, y0), (x0 + 1, y0) and the row below
                        const uint4 a = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
                        const uint4 bq = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, rowB, 0));
                        tY = fmaf(h_lo(a.x), w00, -ry);
                        tU = fmaf(h_hi(a.x), w00, -ru);
                        tV = fmaf(h_lo(a.y), w00, -rv);
                        tY = fmaf(h_lo(a.z), w01, tY);
                        tU = fmaf(h_hi(a.z), w01, tU);
                        tV = fmaf(h_lo(a.w), w01, tV);
                        tY = fmaf(h_lo(bq.x), w10, tY);
                        tU = fmaf(h_hi(bq.x), w10, tU);
                        tV = fmaf(h_lo(bq.y), w10, tV);
                        tY = fmaf(h_lo(bq.z), w11, tY);
                        tU = fmaf(h_hi(bq.z), w11, tU);
                        tV = fmaf(h_lo(bq.w), w11, tV);
                    } else {
                        const float4 a0 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
                        const float4 a1 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0));
                        const float4 b0 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, rowB, 0));
                        const float4 b1 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, rowB, 0));
                        tY = fmaf(a0.x, w00, -ry);
                        tU = fmaf(a0.y, w00, -ru);
                        tV = fmaf(a0.z, w00, -rv);
                        tY = fmaf(a1.x, w01, tY);
                        tU = fmaf(a1.y, w01, tU);
                        tV = fmaf(a1.z, w01, tV);
                        tY = fmaf(b0.x, w10, tY);
                        tU = fmaf(b0.y, w10, tU);
                        tV = fmaf(b0.z, w10, tV);
                        tY = fmaf(b1.x, w11, tY);
                        tU = fmaf(b1.y, w11, tU);
                        tV = fmaf(b1.z, w11, tV);
                    }
                    const float d = fabsf(tY) + fabsf(tU) + fabsf(tV);
                    acc[j] += valid ? d : 0.f;
                    cnt[j] += valid ? 1 : 0;
                } else {
                    const float fx = floorf(u + 0.5f), fy = floorf(v + 0.5f);
                    valid &= (fx >= 0.f) & (fx <= Wm1) & (fy >= 0.f) & (fy <= Hm1);
                    const uint32_t xi = (uint32_t)(int)fx, yi = (uint32_t)(int)fy;
                    const int off = (int)(mad_u24(yi, tp, xi) * kTexB);
                    float dY, dU, dV;
                    if constexpr (!TEXF32) {
                        const uint2 a = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
                        dY = h_lo(a.x) - ry;
                        dU = h_hi(a.x) - ru;
                        dV = h_lo(a.y) - rv;
                    } else {
                        const float4 a = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
                        dY = a.x - ry;
                        dU = a.y - ru;
                        dV = a.z - rv;
                    }
                    // integer code-value differences: exact in FP32, summed exactly
                    const uint32_t d = (uint32_t)(fabsf(dY) + fabsf(dU) + fabsf(dV));
                    acci[j] += valid ? d : 0u;
                    cnt[j] += valid ? 1 : 0;
                }
            }
        }
#pragma unroll
        for (int j = 0; j < J; ++j) {
            if (cnt[j] > 0) {
                const float sum = BIL ? acc[j] : (float)acci[j];
                const float m = sum / ((float)cnt[j] * norm);
                best[j] = fminf(best[j], m);
            }
        }
    }

    const int64_t row = row0 + s;
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (lab[j] < L) {
            const float o = best[j] == __builtin_inff() ? 1.0f : best[j];
            if constexpr (F16OUT)
                static_cast<__half *>(cost)[row * L + lab[j]] = __float2half_rn(o);
            else
                static_cast<float *>(cost)[row * L + lab[j]] = o;
        }
    }
}

// Plain launch: one wave per task.  Block b runs on XCD b mod 8; the
// remapping gives each XCD a contiguous stretch of the spatially ordered
// task list, so its L2 holds the image bands those tasks gather from.
template <int J, bool BIL, bool TEXF32, bool F16OUT>
__global__ __launch_bounds__(256) void k_sweep(const Problem *__restrict__ probs, const Task *__restrict__ tasks,
                                               int64_t n_tasks, int per_xcd)
{
    const int wpg = blockDim.x / kWave;
    const int b = blockIdx.x;
    const int64_t lb = (int64_t)(b & 7) * per_xcd + (b >> 3);
    const int64_t t = lb * wpg + uniform(threadIdx.x / kWave);
    if (t >= n_tasks) return;
    const Task task = ldu_task(tasks + t);
    sweep_task<J, BIL, TEXF32, F16OUT>(probs + task.problem, task);
}

// Persistent launch: waves pull tasks from a shared cursor until the device
// task count (written by an earlier kernel) is exhausted.
template <int J, bool BIL, bool TEXF32, bool F16OUT>
__global__ __launch_bounds__(256) void k_sweep_persistent(const Problem *__restrict__ probs,
                                                          const Task *__restrict__ tasks,
                                                          const int32_t *__restrict__ n_tasks,
                                                          int32_t *__restrict__ cursor, int64_t max_tasks)
{
    const int lane = lane_id();
    const int64_t limit = min((int64_t)ldu(n_tasks), max_tasks);
    for (;;) {
        int t = 0;
        if (lane == 0) t = atomicAdd(cursor, 1);
        t = uniform(__shfl(t, 0));
        if (t >= limit) break;
        const Task task = ldu_task(tasks + t);
        sweep_task<J, BIL, TEXF32, F16OUT>(probs + task.problem, task);
    }
}

// ------------------------------------------------------------------ argmin
template <bool F16>
__global__ void k_argmin(const void *__restrict__ cost, int64_t rows, int L, int32_t *__restrict__ out)
{
    const int lane = lane_id();
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (r >= rows) return;
    float bv = __builtin_inff();
    int bi = 0x7fffffff;
    for (int l = lane; l < L; l += kWave) {
        float x = F16 ? __half2float(static_cast<const __half *>(cost)[r * L + l])
                      : static_cast<const float *>(cost)[r * L + l];
        if (x != x) x = __builtin_inff();       // NaN never wins
        if (x < bv || (x == bv && l < bi)) {
            bv = x;
            bi = l;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const float ov = __shfl_xor(bv, d);
        const int oi = __shfl_xor(bi, d);
        if (ov < bv || (ov == bv && oi < bi)) {
            bv = ov;
            bi = oi;
        }
    }
    if (lane == 0) out[r] = bi == 0x7fffffff ? 0 : bi;
}

// ------------------------------------------------------------------ temporal
// Keep the tasks whose row is marked changed.  Order across waves follows
// the atomics; results do not depend on it.
__global__ void k_compact_tasks(const Problem *__restrict__ P, const Task *__restrict__ all, int64_t n_all,
                                const uint8_t *__restrict__ mask, Task *__restrict__ out,
                                int32_t *__restrict__ n_out)
{
    const int lane = lane_id();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool keep = false;
    Task t{};
    if (i < n_all) {
        t = all[i];
        keep = mask[P->views[t.view].row0 + t.seg] != 0;
    }
    const uint64_t bal = __ballot(keep);
    int base = 0;
    if (lane == 0 && bal) base = atomicAdd(n_out, __builtin_popcountll(bal));
    base = __shfl(base, 0);
    if (keep) out[base + __builtin_popcountll(bal & ((1ull << lane) - 1))] = t;
}

__global__ void k_copy_bytes(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n16)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const unsigned char *p = static_cast<const unsigned char *>(src);
    for (size_t off = 0; off < bytes; off += sizeof(UploadChunk)) {
        UploadChunk c;
        const int n = (int)((bytes - off) < sizeof(c.bytes) ? (bytes - off) : sizeof(c.bytes));
        __builtin_memcpy(c.bytes, p + off, n);
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, static_cast<unsigned char *>(dst) + off, c, n);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_prepare(const Problem *dprob, const Extents &ext, int tex_f32, hipStream_t s)
{
    const unsigned nv = (unsigned)ext.n_views;
    {
        const int n = ext.max_s > 2 * ext.max_bands ? ext.max_s : 2 * ext.max_bands;
        hipLaunchKernelGGL(k_index_init, dim3((unsigned)((n + 255) / 256), nv), dim3(256), 0, s, dprob);
    }
    {
        dim3 blk(64, 4);
        dim3 grd((unsigned)((ext.max_w + 1 + 63) / 64), (unsigned)((ext.max_h + 1 + 3) / 4), nv);
        if (tex_f32)
            hipLaunchKernelGGL(k_pack<float4>, grd, blk, 0, s, dprob);
        else
            hipLaunchKernelGGL(k_pack<uint2>, grd, blk, 0, s, dprob);
    }
    {
        dim3 blk(64, 4);
        dim3 grd((unsigned)((ext.max_w + 63) / 64), (unsigned)((ext.max_h + 3) / 4), nv);
        hipLaunchKernelGGL(k_seg_count, grd, blk, 0, s, dprob);
    }
    hipLaunchKernelGGL(k_scan, dim3(nv), dim3(1024), 0, s, dprob);
    hipLaunchKernelGGL(k_seg_fill, dim3((unsigned)((ext.max_s + 3) / 4), nv), dim3(256), 0, s, dprob);
    return hipGetLastError();
}

hipError_t launch_worklist(const Problem *dprob, const Extents &ext, int problem_index, Task *tasks,
                           hipStream_t s)
{
    const unsigned nv = (unsigned)ext.n_views;
    const unsigned gs = (unsigned)((ext.max_s + 255) / 256);
    hipLaunchKernelGGL(k_band_count, dim3(gs, nv), dim3(256), 0, s, dprob);
    hipLaunchKernelGGL(k_band_scan, dim3(1), dim3(64), 0, s, dprob);
    hipLaunchKernelGGL(k_task_fill, dim3(gs, nv), dim3(256), 0, s, dprob, problem_index, tasks);
    return hipGetLastError();
}

template <int J, bool BIL, bool TEXF32, bool F16OUT>
static hipError_t sweep_plain(const Problem *dprobs, const Task *tasks, int64_t n_tasks, int wpg, hipStream_t s)
{
    const int64_t groups = (n_tasks + wpg - 1) / wpg;
    const int64_t per_xcd = (groups + 7) / 8;
    const int64_t grid = per_xcd * 8;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_sweep<J, BIL, TEXF32, F16OUT>), dim3((unsigned)grid), dim3(64 * wpg), 0, s, dprobs,
                       tasks, n_tasks, (int)per_xcd);
    return hipGetLastError();
}

template <int J, bool BIL, bool TEXF32, bool F16OUT>
static hipError_t sweep_pers(const Problem *dprobs, const Task *tasks, const int32_t *n_tasks, int32_t *cursor,
                             int64_t max_tasks, int wpg, int n_groups, hipStream_t s)
{
    hipLaunchKernelGGL((k_sweep_persistent<J, BIL, TEXF32, F16OUT>), dim3((unsigned)n_groups), dim3(64 * wpg), 0, s,
                       dprobs, tasks, n_tasks, cursor, max_tasks);
    return hipGetLastError();
}

#define IVDE_DISPATCH_FLAGS(FN, J, ...)                                                      \
    do {                                                                                     \
        if (bilinear) {                                                                      \
            if (tex_f32) {                                                                   \
                return f16out ? FN<J, true, true, true>(__VA_ARGS__) : FN<J, true, true, false>(__VA_ARGS__); \
            }                                                                                \
            return f16out ? FN<J, true, false, true>(__VA_ARGS__) : FN<J, true, false, false>(__VA_ARGS__); \
        }                                                                                    \
        if (tex_f32) {                                                                       \
            return f16out ? FN<J, false, true, true>(__VA_ARGS__) : FN<J, false, true, false>(__VA_ARGS__); \
        }                                                                                    \
        return f16out ? FN<J, false, false, true>(__VA_ARGS__) : FN<J, false, false, false>(__VA_ARGS__); \
    } while (0)

hipError_t launch_sweep(const Problem *dprobs, const Task *tasks, int64_t n_tasks, int J, int bilinear,
                        int tex_f32, int f16out, int wpg, hipStream_t s)
{
    if (n_tasks <= 0) return hipSuccess;
    switch (J) {
    case 1: IVDE_DISPATCH_FLAGS(sweep_plain, 1, dprobs, tasks, n_tasks, wpg, s);
    case 2: IVDE_DISPATCH_FLAGS(sweep_plain, 2, dprobs, tasks, n_tasks, wpg, s);
    case 4: IVDE_DISPATCH_FLAGS(sweep_plain, 4, dprobs, tasks, n_tasks, wpg, s);
    case 8: IVDE_DISPATCH_FLAGS(sweep_plain, 8, dprobs, tasks, n_tasks, wpg, s);
    default: return hipErrorInvalidValue;
    }
}

template <int J, bool BIL, bool TEXF32, bool F16OUT>
static hipError_t occ(int wpg, int *per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sweep_persistent<J, BIL, TEXF32, F16OUT>,
                                                        64 * wpg, 0);
}

hipError_t sweep_persistent_occupancy(int J, int bilinear, int tex_f32, int f16out, int wpg, int *per_cu)
{
    const int f16 = f16out;
#define IVDE_OCC(JJ)                                                                                   \
    do {                                                                                              \
        if (bilinear) {                                                                               \
            if (tex_f32) return f16 ? occ<JJ, true, true, true>(wpg, per_cu) : occ<JJ, true, true, false>(wpg, per_cu); \
            return f16 ? occ<JJ, true, false, true>(wpg, per_cu) : occ<JJ, true, false, false>(wpg, per_cu); \
        }                                                                                             \
        if (tex_f32) return f16 ? occ<JJ, false, true, true>(wpg, per_cu) : occ<JJ, false, true, false>(wpg, per_cu); \
        return f16 ? occ<JJ, false, false, true>(wpg, per_cu) : occ<JJ, false, false, false>(wpg, per_cu); \
    } while (0)
    switch (J) {
    case 1: IVDE_OCC(1);
    case 2: IVDE_OCC(2);
    case 4: IVDE_OCC(4);
    case 8: IVDE_OCC(8);
    default: return hipErrorInvalidValue;
    }
#undef IVDE_OCC
}

hipError_t launch_sweep_persistent(const Problem *dprobs, const Task *tasks, const int32_t *n_tasks_dev,
                                   int32_t *cursor, int64_t max_tasks, int J, int bilinear, int tex_f32,
                                   int f16out, int wpg, int n_groups, hipStream_t s)
{
    switch (J) {
    case 1: IVDE_DISPATCH_FLAGS(sweep_pers, 1, dprobs, tasks, n_tasks_dev, cursor, max_tasks, wpg, n_groups, s);
    case 2: IVDE_DISPATCH_FLAGS(sweep_pers, 2, dprobs, tasks, n_tasks_dev, cursor, max_tasks, wpg, n_groups, s);
    case 4: IVDE_DISPATCH_FLAGS(sweep_pers, 4, dprobs, tasks, n_tasks_dev, cursor, max_tasks, wpg, n_groups, s);
    case 8: IVDE_DISPATCH_FLAGS(sweep_pers, 8, dprobs, tasks, n_tasks_dev, cursor, max_tasks, wpg, n_groups, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_argmin(const void *cost, int f16, int64_t rows, int L, int32_t *out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    const int64_t blocks = (rows + 3) / 4;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (f16)
        hipLaunchKernelGGL(k_argmin<true>, dim3((unsigned)blocks), dim3(256), 0, s, cost, rows, L, out);
    else
        hipLaunchKernelGGL(k_argmin<false>, dim3((unsigned)blocks), dim3(256), 0, s, cost, rows, L, out);
    return hipGetLastError();
}

hipError_t launch_compact_tasks(const Problem *dprob, const Task *all, int64_t n_all, const uint8_t *mask,
                                Task *out, int32_t *n_out, hipStream_t s)
{
    if (n_all <= 0) return hipSuccess;
    const int64_t blocks = (n_all + 255) / 256;
    hipLaunchKernelGGL(k_compact_tasks, dim3((unsigned)blocks), dim3(256), 0, s, dprob, all, n_all, mask, out,
                       n_out);
    return hipGetLastError();
}

hipError_t launch_copy_rows(const void *src, void *dst, int64_t bytes, hipStream_t s)
{
    if (bytes <= 0) return hipSuccess;
    if (bytes % 16) return hipErrorInvalidValue;
    const int64_t n16 = bytes / 16;
    int64_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_copy_bytes, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst), n16);
    return hipGetLastError();
}

}  // namespace ivde
