// gfx950 kernels of libivde: image packing, segment index, spatial work
// list, the plane-sweep cost kernel (one persistent launch with per-XCD task
// cursors), argmin and the temporal task compaction.
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
// order, so single-frame, batched and served calls give bitwise equal costs.
#include <algorithm>
#include <type_traits>

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "ivde_internal.h"

namespace ivde {

namespace {

// gathers each wave keeps in flight in the sweep's inner loop
#ifndef IVDE_INFLIGHT
#define IVDE_INFLIGHT 4
#endif

// LDS texels each wave of the one-label-per-lane sweep may stage a target
// footprint into (0: none, the default).  32 waves per CU share 160 KB, so
// 624 is the most that keeps full occupancy; on the 8-view 1080p workload
// about 11% of (task, target) footprints fit that and the staged sweep was
// measured slower than the gathers it replaces, so it is built only for
// measurement (build.py's stage_texels).
#ifndef IVDE_STAGE_TEXELS
#define IVDE_STAGE_TEXELS 0
#endif

constexpr uint32_t kRsrcWord3 = 0x00020000u;   // raw buffer, gfx9 family

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             (int)kRsrcWord3);
}

// A descriptor over 8-byte texel cells (stride 8, the cell count as its
// range) for loads that address cells by index: the hardware forms the byte
// address from the index, so the sweep spends no shift on it.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc_cells(const void *base, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)8, (int)(bytes / 8), (int)kRsrcWord3);
}

// Structured buffer load of 16 bytes at cell vindex (+ voffset + soffset
// bytes), range-checked by cell index against the descriptor.
typedef int ivde_i32x4v __attribute__((ext_vector_type(4)));
__device__ ivde_i32x4v struct_load_b128(__amdgpu_buffer_rsrc_t rsrc, int vindex, int voffset, int soffset,
                                        int aux) __asm("llvm.amdgcn.struct.ptr.buffer.load.v4i32");

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

// Packed texels: (W + 2) x (H + 2) of {Y, Cb, Cr, 0} in 16-bit channels
// (8 bytes a texel), chroma replicated to full resolution (pixel (x, y) owns
// chroma (x >> k, y >> k)).  Channels are halves for bit depths up to 11
// and the 16-bit code values themselves (U16) above, exact either way.
// Texel (X, Y) holds pixel (clamp(X - 1), clamp(Y - 1)): a one-texel border
// that repeats the edge, so a bilinear sample up to one pixel outside the
// image reads the edge value, which is the clamped sample.  A thread packs
// kPackRows texels of one column (rows blockDim.y apart), its loads issued
// together.
constexpr int kPackRows = 4;

template <bool U16>
__global__ __launch_bounds__(256) void k_pack(const Problem *__restrict__ P)
{
    const ViewDesc *vd = ldu(&P->views) + blockIdx.z;
    const int W = ldu(&vd->W), H = ldu(&vd->H);
    const int X = blockIdx.x * blockDim.x + threadIdx.x;
    if (X > W + 1) return;
    const Planes pl = planes_of(P, vd);
    uint2 *tex = static_cast<uint2 *>(ldu(&vd->tex));
    const int64_t tp = ldu(&vd->tex_pitch);
    const int x = min(max(X - 1, 0), W - 1);
    const int Y0 = blockIdx.y * (blockDim.y * kPackRows) + threadIdx.y;
    float c0[kPackRows], c1[kPackRows], c2[kPackRows];
#pragma unroll
    for (int q = 0; q < kPackRows; ++q) {
        const int Y = min(Y0 + q * (int)blockDim.y, H + 1);   // rows past the end repeat the last
        yuv_at(pl, x, min(max(Y - 1, 0), H - 1), c0[q], c1[q], c2[q]);
    }
#pragma unroll
    for (int q = 0; q < kPackRows; ++q) {
        const int Y = Y0 + q * (int)blockDim.y;
        if (Y > H + 1) break;
        uint2 w;
        if constexpr (U16) {
            // code values below 2^16, held exactly by the FP32 colours
            w.x = (uint32_t)c0[q] | ((uint32_t)c1[q] << 16);
            w.y = (uint32_t)c2[q];
        } else {
            w.x = __builtin_bit_cast(uint32_t, __floats2half2_rn(c0[q], c1[q]));
            w.y = __builtin_bit_cast(uint32_t, __floats2half2_rn(c2[q], 0.f));
        }
        stg(tex + (int64_t)Y * tp + X, w);
    }
}

// Pixel counts and boxes.  A block covers a tile of 64 x 16 pixels, a wave
// four of its rows.  Runs of equal ids in a row are merged so one lane per
// run records it, first in a small table in LDS (segment id -> count and
// box, linear probing), which the block then adds to the global arrays with
// one set of atomics per distinct segment.  Runs that find the table full
// go to the global arrays directly.
constexpr int kCountTileRows = 16;
constexpr int kCountSlots = 128;

__device__ __forceinline__ void count_global(int32_t *counts, int32_t *bbox, int id, int n, int x0, int y0, int x1,
                                             int y1)
{
    atomicAdd(&counts[id], n);
    atomicMin(&bbox[4 * id + 0], x0);
    atomicMin(&bbox[4 * id + 1], y0);
    atomicMax(&bbox[4 * id + 2], x1);
    atomicMax(&bbox[4 * id + 3], y1);
}

__global__ __launch_bounds__(256) void k_seg_count(const Problem *__restrict__ P)
{
    __shared__ int key[kCountSlots];
    __shared__ int cnt[kCountSlots], bx0[kCountSlots], by0[kCountSlots], bx1[kCountSlots], by1[kCountSlots];
    const ViewDesc *vd = ldu(&P->views) + blockIdx.z;
    const int W = ldu(&vd->W), H = ldu(&vd->H), S = ldu(&vd->S);
    const int32_t *seg = ldu(&vd->seg);
    const int64_t sp = ldu(&vd->seg_pitch);
    int32_t *counts = ldu(&vd->counts);
    int32_t *bbox = ldu(&vd->bbox);
    int32_t *flag = ldu(&P->flag);
    const int tid = threadIdx.y * kWave + threadIdx.x;
    if (tid < kCountSlots) {
        key[tid] = -1;
        cnt[tid] = 0;
        bx0[tid] = by0[tid] = 0x7fffffff;
        bx1[tid] = by1[tid] = -1;
    }
    __syncthreads();
    const int lane = threadIdx.x;
    const int x = blockIdx.x * kWave + lane;
    constexpr int kRowsPerWave = kCountTileRows / 4;
    int ids[kRowsPerWave];
#pragma unroll
    for (int k = 0; k < kRowsPerWave; ++k) {
        const int y = blockIdx.y * kCountTileRows + 4 * k + threadIdx.y;
        ids[k] = x < W && y < H ? ldg(seg + (int64_t)y * sp + x) : -1;
    }
    for (int k = 0; k < kRowsPerWave; ++k) {
        const int y = blockIdx.y * kCountTileRows + 4 * k + threadIdx.y;
        const bool in = x < W && y < H;
        int id = ids[k];
        if (in && (id < 0 || id >= S)) {
            atomicOr(flag, 1);
            id = -1;
        }
        const int prev = __shfl_up(id, 1);
        const int next = __shfl_down(id, 1);
        const bool head = id >= 0 && (lane == 0 || prev != id);
        const bool tail = id >= 0 && (lane == kWave - 1 || next != id);
        const uint64_t tails = __ballot(tail);
        if (head) {
            const uint64_t after = tails & (~0ull << lane);
            const int len = __builtin_ctzll(after) - lane + 1;
            int slot = id & (kCountSlots - 1), probe = 0;
            for (; probe < kCountSlots; ++probe) {
                const int k0 = atomicCAS(&key[slot], -1, id);
                if (k0 == -1 || k0 == id) break;
                slot = (slot + 1) & (kCountSlots - 1);
            }
            if (probe < kCountSlots) {
                atomicAdd(&cnt[slot], len);
                atomicMin(&bx0[slot], x);
                atomicMin(&by0[slot], y);
                atomicMax(&bx1[slot], x + len - 1);
                atomicMax(&by1[slot], y);
            } else {
                count_global(counts, bbox, id, len, x, y, x + len - 1, y);
            }
        }
    }
    __syncthreads();
    if (tid < kCountSlots && key[tid] >= 0)
        count_global(counts, bbox, key[tid], cnt[tid], bx0[tid], by0[tid], bx1[tid], by1[tid]);
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

// One wave per segment scans its box in raster order and writes the pixel
// records in that order.  A box at most half a wave wide is covered several
// rows per step (lane order is still raster order); wider boxes row by row
// in 64-pixel chunks.  A pixel record is (x, y, g . p~, Y) (Cb, Cr, 0, 0).
// The ids and colours of the next step are loaded while the current step's
// records are written.
__global__ __launch_bounds__(256) void k_seg_fill(const Problem *__restrict__ P)
{
    const ViewDesc *vd = ldu(&P->views) + blockIdx.y;
    const int lane = lane_id();
    const int s = uniform(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    if (s >= ldu(&vd->S)) return;
    const int32_t *bbox = ldu(&vd->bbox) + 4 * s;
    const int x0 = ldu(bbox + 0), y0 = ldu(bbox + 1), x1 = ldu(bbox + 2), y1 = ldu(bbox + 3);
    if (x1 < x0) return;   // empty segment
    const int32_t *offs = ldu(&vd->offsets);
    const int base = ldu(offs + s), cap = ldu(offs + s + 1);
    const Planes pl = planes_of(P, vd);
    const float g0 = ldu(&vd->g[0]), g1 = ldu(&vd->g[1]), g2 = ldu(&vd->g[2]);
    const int32_t *seg = ldu(&vd->seg);
    const int64_t sp = ldu(&vd->seg_pitch);
    float *rec = ldu(&vd->pixrec);
    const int bw = x1 - x0 + 1;
    // step t covers box rows y0 + t rows .. and columns x0 + lc (small boxes),
    // or row y0 + t / chunks, columns from 64 (t % chunks) (wide boxes)
    const bool small = bw <= kWave / 2;
    const int rows = small ? kWave / bw : 1;
    const int lr = small ? lane / bw : 0, lc = small ? lane - lr * bw : lane;
    const int chunks = small ? 1 : (bw + kWave - 1) / kWave;
    const int steps = small ? (y1 - y0 + rows) / rows : (y1 - y0 + 1) * chunks;
    int r = 0, ci = 0;   // row group and chunk of the next step
    auto next_pixel = [&](int &x, int &y) {
        y = y0 + r * rows + lr;
        x = x0 + ci * kWave + lc;
        if (++ci == chunks) {
            ci = 0;
            ++r;
        }
        return lr < rows && y <= y1 && x <= x1;
    };
    // a step's id and colour loads are issued together, one step ahead
    int xn, yn, id = -1;
    float cy = 0.f, cu = 0.f, cv = 0.f;
    auto fetch = [&]() {
        const bool in = next_pixel(xn, yn);
        if (in) {
            id = ldg(seg + (int64_t)yn * sp + xn);
            yuv_at(pl, xn, yn, cy, cu, cv);
        } else {
            id = -1;
        }
    };
    fetch();
    int run = 0;
    for (int t = 0; t < steps; ++t) {
        const int x = xn, y = yn;
        const bool m = id == s;
        float4 r0, r1;
        r0.x = (float)x;
        r0.y = (float)y;
        r0.z = fmaf(g0, r0.x, fmaf(g1, r0.y, g2));
        r0.w = cy;
        r1 = make_float4(cu, cv, 0.f, 0.f);
        if (t + 1 < steps) fetch();
        const uint64_t bal = __ballot(m);
        const int pos = base + run + __builtin_popcountll(bal & ((1ull << lane) - 1));
        if (m && pos < cap) {
            float4 *dst = reinterpret_cast<float4 *>(rec) + 2 * (int64_t)pos;
            stg(dst, r0);
            stg(dst + 1, r1);
        }
        run += __builtin_popcountll(bal);
    }
}

// A new frame of the same segmentation: record positions and g . p~ stay,
// the colours are read again (the same samples a full fill would write).
__global__ __launch_bounds__(256) void k_seg_colour(const Problem *__restrict__ P)
{
    const ViewDesc *vd = ldu(&P->views) + blockIdx.y;
    const int64_t n = ldu(ldu(&vd->offsets) + ldu(&vd->S));
    const Planes pl = planes_of(P, vd);
    float4 *recs = reinterpret_cast<float4 *>(ldu(&vd->pixrec));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float4 *rec = recs + 2 * i;
        float4 r0 = ldg(rec);
        float4 r1;
        yuv_at(pl, (int)r0.x, (int)r0.y, r0.w, r1.x, r1.y);
        r1.z = 0.f;
        r1.w = 0.f;
        stg(rec, r0);
        stg(rec + 1, r1);
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

// counter[key] += 1 for every active lane, one atomic per distinct key in
// the wave (neighbouring segments mostly share a band, and one atomic per
// lane on one address serialises); returns the counter's old value plus the
// lane's rank among the active lanes with its key.
__device__ __forceinline__ int wave_increment(int *counter, int key)
{
    const int lane = lane_id();
    uint64_t pending = __ballot(1);
    int out = 0;
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const int k = __shfl(key, leader);
        const uint64_t group = __ballot(key == k) & pending;
        int base = 0;
        if (lane == leader) base = atomicAdd(&counter[k], (int)__popcll(group));
        base = __shfl(base, leader);
        if ((group >> lane) & 1) out = base + (int)__popcll(group & ((1ull << lane) - 1));
        pending &= ~group;
    }
    return out;
}

__global__ void k_band_count(const Problem *__restrict__ P)
{
    const ViewDesc &v = P->views[blockIdx.y];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= v.S) return;
    wave_increment(v.band_count, segment_band(v, s));
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
// The order of waves inside a band depends on atomics (inside a wave it is
// segment order); no result depends on it.
__global__ void k_task_fill(const Problem *__restrict__ P, int problem_index, Task *__restrict__ tasks)
{
    const int vi = blockIdx.y;
    const ViewDesc &v = P->views[vi];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= v.S) return;
    const int nb = P->n_lblocks;
    const int pos = wave_increment(v.band_count + v.n_bands, segment_band(v, s));
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
// a * b + c on the 24-bit multiplier (operands below 2^24)
__device__ __forceinline__ uint32_t mad_u24(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

#define IVDE_AS3 __attribute__((address_space(3)))

// Byte address of an LDS object in the LDS aperture.
[[maybe_unused]] __device__ __forceinline__ uint32_t lds_addr(const void *p) { return (uint32_t)(uintptr_t)(const IVDE_AS3 void *)p; }

// Two consecutive 8-byte texels at LDS byte address a (8-byte aligned).
[[maybe_unused]] __device__ __forceinline__ uint4 lds_pair(uint32_t a)
{
    const IVDE_AS3 u32x2 *t = (const IVDE_AS3 u32x2 *)(uintptr_t)a;
    const u32x2 x = t[0], y = t[1];
    return make_uint4(x.x, x.y, y.x, y.y);
}

// Target samples of one evaluation, as loaded (8-byte texels).
template <bool BIL>
struct Sample;
template <>
struct Sample<true> {   // texels (x0, y0), (x0 + 1, y0) and the row below
    uint4 a, b;
};
template <>
struct Sample<false> {
    uint2 a;
};

struct Weights {
    float w00, w01, w10, w11;
};

// Per-target constants of the projection h = q + w e.  Coordinates are in
// the bordered texel frame (pixel + 1).  Bilinear samples are valid in
// [1 - edge, W + edge] x [1 - edge, H + edge]; nearest ones when the rounded
// position is a pixel, [1, W] x [1, H].
struct Target {
    __amdgpu_buffer_rsrc_t rs;
    float lo, hi_x, hi_y;
    uint32_t tp;
    uint32_t rowB;        // bytes per texel row
    float e0, e1, e2;
    // staged footprint (half texels in LDS): byte address of texel (0, 0)
    // of the target image relative to the stage, and bytes per stage row
    uint32_t sbase, srowB;
};

// Projects one (pixel, label) into the target, decides validity and issues
// the texel loads: h = q + w e with w = sigma (g . p~) = 1 / tau.  FRONT
// says what the host has shown: 0 nothing (test w > 0, the point in front of
// the source camera, and h_z > 0, in front of the target), 1 every pixel and
// label of the view lies in front of the source camera (test h_z > 0 only),
// 2 and also in front of this target (no test).  Out-of-image
// coordinates are clamped, so every load is in bounds; the buffer
// descriptor bounds them again.
template <bool BIL, int FRONT, bool STAGED = false>
__device__ __forceinline__ void project_issue(const Target &T, float qx, float qy, float qz, float w,
                                              Sample<BIL> &smp, Weights &wt, bool &valid)
{
    constexpr int kTexB = 8;
    const float hx = fmaf(w, T.e0, qx);
    const float hy = fmaf(w, T.e1, qy);
    const float hz = fmaf(w, T.e2, qz);
    const float r = __builtin_amdgcn_rcpf(hz);
    const float u = hx * r, v = hy * r;
    valid = FRONT == 2 ? true : FRONT == 1 ? (hz > 0.f) : ((w > 0.f) & (hz > 0.f));
    if constexpr (BIL) {
        // clamp into the valid band; the sample is valid iff nothing moved.
        // Clamped coordinates are positive (truncation is floor) and keep
        // invalid lanes' reads next to the image border.
        const float uc = __builtin_amdgcn_fmed3f(u, T.lo, T.hi_x);
        const float vc = __builtin_amdgcn_fmed3f(v, T.lo, T.hi_y);
        valid &= (uc == u) & (vc == v);
        const uint32_t x0 = (uint32_t)(int)uc, y0 = (uint32_t)(int)vc;
        const float ax = __builtin_amdgcn_fractf(uc), ay = __builtin_amdgcn_fractf(vc);
        wt.w11 = ax * ay;
        wt.w01 = ax - wt.w11;
        wt.w10 = ay - wt.w11;
        wt.w00 = (1.f - ax) - wt.w10;
        if constexpr (STAGED) {
            // the footprint staged in LDS, rows of srowB bytes
            const uint32_t a = mad_u24(x0, (uint32_t)kTexB, mad_u24(y0, T.srowB, T.sbase));
            smp.a = lds_pair(a);
            smp.b = lds_pair(a + T.srowB);
            return;
        }
        const int off = (int)(mad_u24(y0, T.tp, x0) * kTexB);
        smp.a = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(T.rs, off, 0, 0));
        smp.b = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(T.rs, off, (int)T.rowB, 0));
    } else {
        const float fx = floorf(u + 0.5f), fy = floorf(v + 0.5f);
        valid &= (fx >= 1.f) & (fx <= T.hi_x - kEdge) & (fy >= 1.f) & (fy <= T.hi_y - kEdge);
        const uint32_t xi = (uint32_t)(int)fx, yi = (uint32_t)(int)fy;
        const int off = valid ? (int)(mad_u24(yi, T.tp, xi) * kTexB) : 0;
        smp.a = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(T.rs, off, 0, 0));
    }
}

// |dY| + |dCb| + |dCr| of one evaluation in code values.
template <bool BIL, bool U16>
__device__ __forceinline__ float consume(const Sample<BIL> &smp, const Weights &wt, float ry, float ru, float rv)
{
    float tY, tU, tV;
    if constexpr (BIL) {
        tY = fmaf(ch_lo<U16>(smp.a.x), wt.w00, -ry);
        tU = fmaf(ch_hi<U16>(smp.a.x), wt.w00, -ru);
        tV = fmaf(ch_lo<U16>(smp.a.y), wt.w00, -rv);
        tY = fmaf(ch_lo<U16>(smp.a.z), wt.w01, tY);
        tU = fmaf(ch_hi<U16>(smp.a.z), wt.w01, tU);
        tV = fmaf(ch_lo<U16>(smp.a.w), wt.w01, tV);
        tY = fmaf(ch_lo<U16>(smp.b.x), wt.w10, tY);
        tU = fmaf(ch_hi<U16>(smp.b.x), wt.w10, tU);
        tV = fmaf(ch_lo<U16>(smp.b.y), wt.w10, tV);
        tY = fmaf(ch_lo<U16>(smp.b.z), wt.w11, tY);
        tU = fmaf(ch_hi<U16>(smp.b.z), wt.w11, tU);
        tV = fmaf(ch_lo<U16>(smp.b.w), wt.w11, tV);
    } else {
        tY = ch_lo<U16>(smp.a.x) - ry;
        tU = ch_hi<U16>(smp.a.x) - ru;
        tV = ch_lo<U16>(smp.a.y) - rv;
    }
    return fabsf(tY) + fabsf(tU) + fabsf(tV);
}

// PU pixels x J labels per step: all gathers of the step are issued before
// the first is consumed, so a wave keeps PU J of them in flight.  The
// accumulation order per label is the pixel order either way.
template <int J, int PU, bool BIL, bool U16, int FRONT, bool STAGED = false>
__device__ __forceinline__ void sweep_pixels(const float *__restrict__ pix, int i0, int i1, const float (&H)[9],
                                             const Target &T, const float (&sig)[J], float (&acc)[J],
                                             uint64_t (&acci)[J], int (&cnt)[J])
{
    int i = i0;
    for (; i + PU <= i1; i += PU) {
        Sample<BIL> smp[PU][J];
        Weights wt[PU][J];
        bool val[PU][J];
        float ry[PU], ru[PU], rv[PU];
#pragma unroll
        for (int p = 0; p < PU; ++p) {
            const f32x4 r0 = ldu4(pix + 8 * (int64_t)(i + p));
            const f32x4 r1 = ldu4(pix + 8 * (int64_t)(i + p) + 4);
            const float x = r0.x, y = r0.y, gp = r0.z;
            ry[p] = r0.w;
            ru[p] = r1.x;
            rv[p] = r1.y;
            const float qx = fmaf(H[0], x, fmaf(H[1], y, H[2]));
            const float qy = fmaf(H[3], x, fmaf(H[4], y, H[5]));
            const float qz = fmaf(H[6], x, fmaf(H[7], y, H[8]));
#pragma unroll
            for (int j = 0; j < J; ++j)
                project_issue<BIL, FRONT, STAGED>(T, qx, qy, qz, sig[j] * gp, smp[p][j], wt[p][j], val[p][j]);
        }
        // keep the scheduler from sinking the loads back next to their uses
        if constexpr (PU > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int p = 0; p < PU; ++p) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const float d = consume<BIL, U16>(smp[p][j], wt[p][j], ry[p], ru[p], rv[p]);
                if constexpr (BIL) {
                    acc[j] += val[p][j] ? d : 0.f;
                } else {
                    // integer code-value differences: exact in FP32, summed exactly
                    acci[j] += val[p][j] ? (uint32_t)d : 0u;
                }
                cnt[j] += val[p][j] ? 1 : 0;
            }
        }
    }
    if constexpr (PU > 1) sweep_pixels<J, 1, BIL, U16, FRONT, STAGED>(pix, i, i1, H, T, sig, acc, acci, cnt);
}

// One task: labels [64 J b, 64 J (b + 1)) of row (view, seg).
// The box of target texels that one task's samples can touch in target c2,
// when every level point of the view lies in front of both cameras: the
// points of the segment's pixel box between the task's first and last level
// fill a convex solid (the box's viewing frustum between two level planes)
// whose eight corners are the box corners at those two levels; a projection
// with positive depth keeps it convex, so the projected corners bound every
// sample, and clamping to the validity band (monotone) keeps them in the box.
// One texel of margin covers FP32 rounding, one more the second bilinear
// tap.  If the box fits `budget` texels, the wave copies it (rows of bw
// texels) into its LDS stage and returns true.
template <int J>
__device__ __forceinline__ bool stage_footprint(const ViewDesc *vc, const ViewDesc *vt, int s, int l_lo, int l_hi,
                                                const float *sigma_row, const float (&H)[9], Target &T,
                                                uint2 *stage, int budget)
{
    const int lane = lane_id();
    const int32_t *bb = ldu(&vc->bbox) + 4 * s;
    const int bx0 = ldu(bb), by0 = ldu(bb + 1), bx1 = ldu(bb + 2), by1 = ldu(bb + 3);
    if (bx1 < bx0) return false;   // empty segment
    const int k = lane & 7;
    const float cx = (float)((k & 1) ? bx1 : bx0), cy = (float)((k & 2) ? by1 : by0);
    const float gp = fmaf(ldu(&vc->g[0]), cx, fmaf(ldu(&vc->g[1]), cy, ldu(&vc->g[2])));
    const float w = sigma_row[(k & 4) ? l_hi : l_lo] * gp;
    const float hx = fmaf(w, T.e0, fmaf(H[0], cx, fmaf(H[1], cy, H[2])));
    const float hy = fmaf(w, T.e1, fmaf(H[3], cx, fmaf(H[4], cy, H[5])));
    const float hz = fmaf(w, T.e2, fmaf(H[6], cx, fmaf(H[7], cy, H[8])));
    const float r = __builtin_amdgcn_rcpf(hz);
    const int ix = (int)floorf(__builtin_amdgcn_fmed3f(hx * r, T.lo, T.hi_x));
    const int iy = (int)floorf(__builtin_amdgcn_fmed3f(hy * r, T.lo, T.hi_y));
    const bool corner = lane < 8;
    const int xmin = wave_min_i32(corner ? ix : 0x7fffffff), xmax = -wave_min_i32(corner ? -ix : 0x7fffffff);
    const int ymin = wave_min_i32(corner ? iy : 0x7fffffff), ymax = -wave_min_i32(corner ? -iy : 0x7fffffff);
    const int W = ldu(&vt->W), Ht = ldu(&vt->H);
    const int X0 = max(xmin - 1, 0), X1 = min(xmax + 2, W + 1);
    const int Y0 = max(ymin - 1, 0), Y1 = min(ymax + 2, Ht + 1);
    const int bw = X1 - X0 + 1, area = bw * (Y1 - Y0 + 1);
    if (area > budget) return false;
    // copy, row-major with pitch bw; stage index t = row * bw + column
    const uint2 *src = static_cast<const uint2 *>(ldu(&vt->tex)) + (int64_t)Y0 * T.tp + X0;
    const float inv_bw = __builtin_amdgcn_rcpf((float)bw);
    for (int t0 = 0; t0 < area; t0 += 4 * kWave) {
        uint2 val[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = t0 + q * kWave + lane;
            // t < 2^10: the product is within 1e-4 of row + (column + 1/2) / bw
            const int row = (int)(((float)t + 0.5f) * inv_bw);
            val[q] = t < area ? ldg2u(src + (int64_t)row * T.tp + (t - row * bw)) : make_uint2(0u, 0u);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = t0 + q * kWave + lane;
            if (t < area) stage[t] = val[q];
        }
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);    // lgkmcnt(0): the stage is written before it is read
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    T.srowB = (uint32_t)bw * 8u;
    T.sbase = lds_addr(stage) - (uint32_t)(Y0 * bw + X0) * 8u;
    return true;
}

template <int J, bool BIL, bool U16, bool F16OUT, int STAGE = 0>
__device__ __forceinline__ void sweep_task(const Problem *__restrict__ P, const Task task, uint2 *stage = nullptr)
{
    constexpr int PU = IVDE_INFLIGHT / J > 0 ? IVDE_INFLIGHT / J : 1;
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

    const int front_all = ldu(&vc->front_all);
    const uint32_t front_targets = ldu(&vc->front_targets);

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
        Target T;
        T.rs = make_rsrc(ldu(&vt->tex), ldu(&vt->tex_bytes));
        T.lo = 1.f - kEdge;
        T.hi_x = (float)ldu(&vt->W) + kEdge;
        T.hi_y = (float)ldu(&vt->H) + kEdge;
        T.tp = (uint32_t)ldu(&vt->tex_pitch);
        T.rowB = (int)T.tp * 8;
        const float *pc = reinterpret_cast<const float *>(pairs + c * n + c2);
        const f32x4 ha = ldu4(pc), hb = ldu4(pc + 4), hc = ldu4(pc + 8);
        const float H[9] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y, hb.z, hb.w, hc.x};
        T.e0 = hc.y;
        T.e1 = hc.z;
        T.e2 = hc.w;

        float acc[J];
        uint64_t acci[J];
        int cnt[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            acc[j] = 0.f;
            acci[j] = 0;
            cnt[j] = 0;
        }
        bool staged = false;
        if constexpr (STAGE > 0 && J == 1 && BIL && !U16) {
            if (front_all && ((front_targets >> c2) & 1u) && p1 > p0) {
                const int l_lo = task.lblock * kWave, l_hi = min(l_lo + kWave - 1, L - 1);
                staged = stage_footprint<J>(vc, vt, s, l_lo, l_hi, sigma + c * L, H, T, stage, STAGE);
                if (staged) sweep_pixels<J, PU, BIL, U16, 2, true>(pix, p0, p1, H, T, sig, acc, acci, cnt);
            }
        }
        if (staged) {
        } else if (front_all && ((front_targets >> c2) & 1u))
            sweep_pixels<J, PU, BIL, U16, 2>(pix, p0, p1, H, T, sig, acc, acci, cnt);
        else if (front_all)
            sweep_pixels<J, PU, BIL, U16, 1>(pix, p0, p1, H, T, sig, acc, acci, cnt);
        else
            sweep_pixels<J, PU, BIL, U16, 0>(pix, p0, p1, H, T, sig, acc, acci, cnt);
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

// The sweep launch: a grid that fits on the GPU at once, whose waves pull
// tasks from per-XCD cursors until the device task count (written by an
// earlier kernel) is exhausted.  A wave whose home range is empty helps with
// the others, so no XCD idles while another has work (with one XCD per view
// in a view-major task list, views whose gathers cost more no longer set
// the kernel's end).
template <int J, bool BIL, bool U16, bool F16OUT, int STAGE = 0>
__device__ __forceinline__ void sweep_persistent_body(const Problem *__restrict__ probs,
                                                      const Task *__restrict__ tasks,
                                                      const int32_t *__restrict__ n_tasks,
                                                      int32_t *__restrict__ cursors, int64_t max_tasks,
                                                      uint2 *stage = nullptr)
{
    const int lane = lane_id();
    const int64_t limit = min((int64_t)ldu(n_tasks), max_tasks);
    // The task list is cut into kXcds contiguous ranges with a cursor each.
    // Block b runs on XCD b mod kXcds: its waves drain their own XCD's range
    // first (so that XCD's L2 holds the image bands those tasks gather
    // from), then help with the other ranges in turn.  Every wave tries
    // every range until it is empty, so all waves end.
    const int home = (int)(blockIdx.x % kXcds);
    for (int k = 0; k < kXcds; ++k) {
        const int x = (home + k) % kXcds;
        const int64_t lo = limit * x / kXcds, n = limit * (x + 1) / kXcds - lo;
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&cursors[x], 1);
            t = uniform(__shfl(t, 0));
            if (t >= n) break;
            const Task task = ldu_task(tasks + lo + t);
            sweep_task<J, BIL, U16, F16OUT, STAGE>(probs + task.problem, task, stage);
        }
    }
}

template <int J, bool BIL, bool U16, bool F16OUT>
__global__ __launch_bounds__(256) void k_sweep_persistent(const Problem *__restrict__ probs,
                                                          const Task *__restrict__ tasks,
                                                          const int32_t *__restrict__ n_tasks,
                                                          int32_t *__restrict__ cursors, int64_t max_tasks)
{
    sweep_persistent_body<J, BIL, U16, F16OUT>(probs, tasks, n_tasks, cursors, max_tasks);
}

// One label per lane fits 64 VGPRs; at 8 waves per SIMD it hides gather
// latency best (measured on the 8-view 1080p workload).
template <bool BIL, bool F16OUT, bool U16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_sweep_persistent_j1(
    const Problem *__restrict__ probs, const Task *__restrict__ tasks, const int32_t *__restrict__ n_tasks,
    int32_t *__restrict__ cursors, int64_t max_tasks)
{
#if IVDE_STAGE_TEXELS > 0
    __shared__ uint2 stage[4][IVDE_STAGE_TEXELS];
    sweep_persistent_body<1, BIL, U16, F16OUT, IVDE_STAGE_TEXELS>(probs, tasks, n_tasks, cursors, max_tasks,
                                                                  stage[threadIdx.x / kWave]);
#else
    sweep_persistent_body<1, BIL, U16, F16OUT>(probs, tasks, n_tasks, cursors, max_tasks);
#endif
}

// ------------------------------------------------------------------ pixel-pair sweep
// The same (view, segment, 64-level block) tasks, with each wave step
// covering two pixels of the segment at 32 levels instead of one pixel at
// 64: lanes 0-31 take the even records of the segment, lanes 32-63 the odd
// ones, and lane k of either half the levels 64 b + k (first pass) and
// 64 b + 32 + k (second pass).  The 64 gathers of one instruction then span
// the epipolar stretch of 32 levels at two neighbouring pixels, which touch
// almost the same texels, instead of the stretch of 64 levels: half the
// cache lines per gather.  The segment's pixel records are staged in the
// wave's slice of LDS per (target, chunk of up to 256 records), read back by
// each lane for its own pixel, and both 32-level passes run over a chunk
// while it is staged.  For a target proven in front of every level point
// the stage holds the projection base already divided by g . p~ (see
// stage_projected), so a step forms h with three multiply-adds; otherwise
// it holds {x, y, Y | Cb, Cr} and a step forms q = H p~ and g . p~ as the
// one-pixel sweep does.  Reference colours use the texels' 16-bit channels
// (halves up to 11 bits, code values above), exact either way.
// The two halves' sums and counts meet through one cross-lane exchange per
// (target, pass).
constexpr int kPairStage = 256;   // records one wave stages at a time (16 B + 2 B, or 16 B + 8 B, each)

// What the stage keeps beside each 16-byte projected record: Cr as an FP16
// channel, or, with 16-bit code values, Cb and Cr as FP32 (the record's
// fourth word then holds Y as FP32), so that the sweep converts no
// reference colour per step.
template <bool U16>
using PairSide = std::conditional_t<U16, uint2, uint16_t>;

// Two reference colours (code values) in the 16-bit channels the texels use.
template <bool U16>
__device__ __forceinline__ uint32_t pack_ch(float a, float b)
{
    if constexpr (U16)
        return (uint32_t)a | ((uint32_t)b << 16);
    else
        return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a, b));
}

// Records [i0, i0 + n) of the view into the stage (n <= kPairStage).
template <bool U16>
__device__ __forceinline__ void stage_records(const float *__restrict__ pix, int i0, int n, uint4 *st)
{
    const int lane = lane_id();
    __builtin_amdgcn_wave_barrier();   // earlier reads of the stage come first
    for (int t0 = 0; t0 < n; t0 += kWave) {
        const int t = t0 + lane;
        if (t < n) {
            const float *r = pix + 8 * (int64_t)(i0 + t);
            const float4 r0 = ldg(reinterpret_cast<const float4 *>(r));
            const float2 r1 = ldg(reinterpret_cast<const float2 *>(r + 4));
            st[t] = make_uint4(__float_as_uint(r0.x), __float_as_uint(r0.y), pack_ch<U16>(r0.w, r1.x),
                               pack_ch<U16>(r1.y, 0.f));
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Records [i0, i0 + n) of the view towards a target proven in front of every
// level point (n <= kPairStage).  The homogeneous target point of a pixel at
// level sigma is h = q + sigma (g . p~) e with q = H p~; dividing by g . p~
// (non-zero there, since the level point has finite positive depth) gives
// q' + sigma e with q' = q / (g . p~), which projects to the same pixel, and
// the target's validity needs no sign test.  The stage holds {q'x, q'y,
// q'z, Y | Cb} and the Cr channel beside it, in cr; with 16-bit code values
// {q'x, q'y, q'z, Y} and {Cb, Cr}, all FP32.
//
// Returns true (wave-uniform) when every staged record's samples at levels
// sig_a .. sig_b lie inside the validity band.  The level points of one
// pixel between two levels form a segment of its viewing ray in front of
// the target, so their projections form the segment between the two end
// projections, and the band is convex: both ends inside it, with a margin
// of kInside pixels far above the FP32 error of any projected coordinate,
// put every level's sample inside, as the sweep computes it.
constexpr float kInside = 1.0f / 16.0f;

template <bool U16>
__device__ __forceinline__ bool stage_projected(const float *__restrict__ pix, int i0, int n, const float (&H)[9],
                                                const Target &T, float sig_a, float sig_b, uint4 *st,
                                                PairSide<U16> *cr)
{
    const int lane = lane_id();
    bool outside = false;
    __builtin_amdgcn_wave_barrier();   // earlier reads of the stage come first
    for (int t0 = 0; t0 < n; t0 += kWave) {
        const int t = t0 + lane;
        if (t < n) {
            const float *r = pix + 8 * (int64_t)(i0 + t);
            const float4 r0 = ldg(reinterpret_cast<const float4 *>(r));
            const float2 r1 = ldg(reinterpret_cast<const float2 *>(r + 4));
            const float x = r0.x, y = r0.y, rg = 1.0f / r0.z;   // r0.z = g . p~ of the index build
            const float qx = fmaf(H[0], x, fmaf(H[1], y, H[2])) * rg;
            const float qy = fmaf(H[3], x, fmaf(H[4], y, H[5])) * rg;
            const float qz = fmaf(H[6], x, fmaf(H[7], y, H[8])) * rg;
            if constexpr (U16) {
                st[t] = make_uint4(__float_as_uint(qx), __float_as_uint(qy), __float_as_uint(qz),
                                   __float_as_uint(r0.w));
                cr[t] = make_uint2(__float_as_uint(r1.x), __float_as_uint(r1.y));
            } else {
                st[t] = make_uint4(__float_as_uint(qx), __float_as_uint(qy), __float_as_uint(qz),
                                   pack_ch<false>(r0.w, r1.x));
                cr[t] = (uint16_t)pack_ch<false>(r1.y, 0.f);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const float w = k ? sig_b : sig_a;
                const float rz = __builtin_amdgcn_rcpf(fmaf(w, T.e2, qz));
                const float u = fmaf(w, T.e0, qx) * rz, v = fmaf(w, T.e1, qy) * rz;
                outside |= !((u >= T.lo + kInside) & (u <= T.hi_x - kInside) & (v >= T.lo + kInside) &
                             (v <= T.hi_y - kInside));
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return __ballot(outside) == 0;
}

// Projection and gathers of one (pixel, label) for the pixel-pair sweep: as
// project_issue, but the bilinear fractions are returned
// instead of the four weights, which consume_pair forms (the same
// operations, later), so fewer registers stay live across the gathers.
// FRONT 3: as 2, and the sample is known to lie inside the validity band
// (stage_projected), so it is neither clamped nor tested.  CELLS: T.rs is a
// cell descriptor (make_rsrc_cells) and bilinear gathers address texels by
// index (with 16-bit code-value texels, whose sweep is limited by VALU issue
// as much as by the texture path: 1-2% faster there, and 0.2-0.4% slower
// with FP16 texels, where the texture path alone binds).
template <bool BIL, int FRONT, bool CELLS = false>
__device__ __forceinline__ void project_pair(const Target &T, float qx, float qy, float qz, float w,
                                             Sample<BIL> &smp, float &ax, float &ay, bool &valid)
{
    const float hx = fmaf(w, T.e0, qx);
    const float hy = fmaf(w, T.e1, qy);
    const float hz = fmaf(w, T.e2, qz);
    const float r = __builtin_amdgcn_rcpf(hz);
    const float u = hx * r, v = hy * r;
    valid = FRONT >= 2 ? true : FRONT == 1 ? (hz > 0.f) : ((w > 0.f) & (hz > 0.f));
    if constexpr (BIL) {
        float uc = u, vc = v;
        if constexpr (FRONT != 3) {
            uc = __builtin_amdgcn_fmed3f(u, T.lo, T.hi_x);
            vc = __builtin_amdgcn_fmed3f(v, T.lo, T.hi_y);
            valid &= (uc == u) & (vc == v);
        }
        const uint32_t x0 = (uint32_t)(int)uc, y0 = (uint32_t)(int)vc;
        ax = __builtin_amdgcn_fractf(uc);
        ay = __builtin_amdgcn_fractf(vc);
        if constexpr (CELLS) {
            const int cell = (int)mad_u24(y0, T.tp, x0);
            smp.a = __builtin_bit_cast(uint4, struct_load_b128(T.rs, cell, 0, 0, 0));
            smp.b = __builtin_bit_cast(uint4, struct_load_b128(T.rs, cell, 0, (int)T.rowB, 0));
        } else {
            const int off = (int)(mad_u24(y0, T.tp, x0) * 8u);
            smp.a = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(T.rs, off, 0, 0));
            smp.b = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(T.rs, off, (int)T.rowB, 0));
        }
    } else {
        const float fx = floorf(u + 0.5f), fy = floorf(v + 0.5f);
        if constexpr (FRONT != 3)
            valid &= (fx >= 1.f) & (fx <= T.hi_x - kEdge) & (fy >= 1.f) & (fy <= T.hi_y - kEdge);
        const uint32_t xi = (uint32_t)(int)fx, yi = (uint32_t)(int)fy;
        const int off = (FRONT == 3 || valid) ? (int)(mad_u24(yi, T.tp, xi) * 8u) : 0;
        smp.a = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(T.rs, off, 0, 0));
        ax = ay = 0.f;
    }
}

// |dY| + |dCb| + |dCr| of one evaluation against reference colours
// (ry, ru, rv), with the weights formed from the bilinear fractions as
// project_issue forms them.
template <bool BIL, bool U16>
__device__ __forceinline__ float consume_pair(const Sample<BIL> &smp, float ax, float ay, float ry, float ru,
                                              float rv)
{
    float tY, tU, tV;
    if constexpr (BIL) {
        Weights wt;
        wt.w11 = ax * ay;
        wt.w01 = ax - wt.w11;
        wt.w10 = ay - wt.w11;
        wt.w00 = (1.f - ax) - wt.w10;
        tY = fmaf(ch_lo<U16>(smp.a.x), wt.w00, -ry);
        tU = fmaf(ch_hi<U16>(smp.a.x), wt.w00, -ru);
        tV = fmaf(ch_lo<U16>(smp.a.y), wt.w00, -rv);
        tY = fmaf(ch_lo<U16>(smp.a.z), wt.w01, tY);
        tU = fmaf(ch_hi<U16>(smp.a.z), wt.w01, tU);
        tV = fmaf(ch_lo<U16>(smp.a.w), wt.w01, tV);
        tY = fmaf(ch_lo<U16>(smp.b.x), wt.w10, tY);
        tU = fmaf(ch_hi<U16>(smp.b.x), wt.w10, tU);
        tV = fmaf(ch_lo<U16>(smp.b.y), wt.w10, tV);
        tY = fmaf(ch_lo<U16>(smp.b.z), wt.w11, tY);
        tU = fmaf(ch_hi<U16>(smp.b.z), wt.w11, tU);
        tV = fmaf(ch_lo<U16>(smp.b.w), wt.w11, tV);
    } else {
        tY = ch_lo<U16>(smp.a.x) - ry;
        tU = ch_hi<U16>(smp.a.x) - ru;
        tV = ch_lo<U16>(smp.a.y) - rv;
    }
    return fabsf(tY) + fabsf(tU) + fabsf(tV);
}

// The same against reference colours packed in the texels' 16-bit channels
// (rz = Y | Cb, rw = Cr).
template <bool BIL, bool U16>
__device__ __forceinline__ float consume_pair(const Sample<BIL> &smp, float ax, float ay, uint32_t rz, uint32_t rw)
{
    return consume_pair<BIL, U16>(smp, ax, ay, ch_lo<U16>(rz), ch_hi<U16>(rz), ch_lo<U16>(rw));
}

// Pairs of staged records [0, m) towards one target at one pass (lane k of
// either half at level sig): PU pairs per step with every gather issued
// before the first is consumed, then the remaining pairs one at a time (the
// last possibly with one pixel).
template <int PU, bool BIL, int FRONT, int G, bool U16>
__device__ __forceinline__ void sweep_pair_records(const uint4 *st, int m, int h, const float (&H)[9],
                                                   const float (&g)[3], const Target &T, float sig, float &acc,
                                                   uint64_t &acci, int &cnt)
{
    int i = 0;
    for (; i + G * PU <= m; i += G * PU) {
        Sample<BIL> smp[PU];
        float ax[PU], ay[PU];
        bool val[PU];
        uint32_t rz[PU], rw[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const uint4 r = st[i + G * u + h];
            const float x = __uint_as_float(r.x), y = __uint_as_float(r.y);
            rz[u] = r.z;
            rw[u] = r.w;
            const float qx = fmaf(H[0], x, fmaf(H[1], y, H[2]));
            const float qy = fmaf(H[3], x, fmaf(H[4], y, H[5]));
            const float qz = fmaf(H[6], x, fmaf(H[7], y, H[8]));
            const float gp = fmaf(g[0], x, fmaf(g[1], y, g[2]));
            project_pair<BIL, FRONT, U16 && BIL>(T, qx, qy, qz, sig * gp, smp[u], ax[u], ay[u], val[u]);
        }
        if constexpr (PU > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const float d = consume_pair<BIL, U16>(smp[u], ax[u], ay[u], rz[u], rw[u]);
            if constexpr (BIL)
                acc += val[u] ? d : 0.f;
            else
                acci += val[u] ? (uint32_t)d : 0u;
            cnt += val[u] ? 1 : 0;
        }
    }
    for (; i < m; i += G) {
        const int j = i + h;
        const bool here = j < m;
        const uint4 r = st[here ? j : m - 1];
        const float x = __uint_as_float(r.x), y = __uint_as_float(r.y);
        const float qx = fmaf(H[0], x, fmaf(H[1], y, H[2]));
        const float qy = fmaf(H[3], x, fmaf(H[4], y, H[5]));
        const float qz = fmaf(H[6], x, fmaf(H[7], y, H[8]));
        const float gp = fmaf(g[0], x, fmaf(g[1], y, g[2]));
        Sample<BIL> smp;
        float ax, ay;
        bool val;
        project_pair<BIL, FRONT, U16 && BIL>(T, qx, qy, qz, sig * gp, smp, ax, ay, val);
        val &= here;
        const float d = consume_pair<BIL, U16>(smp, ax, ay, r.z, r.w);
        if constexpr (BIL)
            acc += val ? d : 0.f;
        else
            acci += val ? (uint32_t)d : 0u;
        cnt += val ? 1 : 0;
    }
}

// One evaluation against a projected record's colours: the record's fourth
// word and what the stage keeps beside it (PairSide).
template <bool BIL, bool U16>
__device__ __forceinline__ float consume_projected(const Sample<BIL> &smp, float ax, float ay, uint32_t rw4,
                                                   PairSide<U16> side)
{
    if constexpr (U16)
        return consume_pair<BIL, true>(smp, ax, ay, __uint_as_float(rw4), __uint_as_float(side.x),
                                       __uint_as_float(side.y));
    else
        return consume_pair<BIL, false>(smp, ax, ay, rw4, (uint32_t)side);
}

// Pairs of projected records [0, m) (stage_projected) towards a target
// proven in front of every level point, at one pass (lane k of either half
// at level sig): as sweep_pair_records with h = q' + sig e; FRONT 3 when
// every sample of the chunk lies inside the validity band.
template <int PU, bool BIL, int FRONT, int G, bool U16>
__device__ __forceinline__ void sweep_pair_projected(const uint4 *st, const PairSide<U16> *cr, int m, int h,
                                                     const Target &T, float sig, float &acc, uint64_t &acci,
                                                     int &cnt)
{
    int i = 0;
    for (; i + G * PU <= m; i += G * PU) {
        Sample<BIL> smp[PU];
        float ax[PU], ay[PU];
        bool val[PU];
        uint32_t rz[PU];
        PairSide<U16> rw[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const uint4 r = st[i + G * u + h];
            rz[u] = r.w;
            rw[u] = cr[i + G * u + h];
            project_pair<BIL, FRONT, U16 && BIL>(T, __uint_as_float(r.x), __uint_as_float(r.y), __uint_as_float(r.z),
                                                 sig, smp[u], ax[u], ay[u], val[u]);
        }
        if constexpr (PU > 1) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            const float d = consume_projected<BIL, U16>(smp[u], ax[u], ay[u], rz[u], rw[u]);
            if constexpr (BIL)
                acc += val[u] ? d : 0.f;
            else
                acci += val[u] ? (uint32_t)d : 0u;
            if constexpr (FRONT != 3) cnt += val[u] ? 1 : 0;
        }
    }
    for (; i < m; i += G) {
        const int j = i + h;
        const bool here = j < m;
        const int jj = here ? j : m - 1;
        const uint4 r = st[jj];
        Sample<BIL> smp;
        float ax, ay;
        bool val;
        project_pair<BIL, FRONT, U16 && BIL>(T, __uint_as_float(r.x), __uint_as_float(r.y), __uint_as_float(r.z), sig,
                                             smp, ax, ay, val);
        val &= here;
        const float d = consume_projected<BIL, U16>(smp, ax, ay, r.w, cr[jj]);
        if constexpr (BIL)
            acc += val ? d : 0.f;
        else
            acci += val ? (uint32_t)d : 0u;
        if constexpr (FRONT != 3) cnt += val ? 1 : 0;
    }
    if constexpr (FRONT == 3) cnt += (m - h + G - 1) / G;   // every record of this group, every sample valid
}

// Pairs each wave keeps in flight in the pixel-pair sweep, and the waves per
// SIMD its kernel is compiled for.  Three pairs at six waves take 76 VGPRs
// with nothing spilled; on the 8-view 1080p arc rig they beat eight waves
// (64 VGPRs, spills outside the pixel loop) by 3-6% at 128, 256 and 512
// levels, and two or four pairs at four to six waves by up to 2%.
// Evaluating both of a lane's levels per pixel (the projection base formed
// once for both) fits only one pixel in flight and was slower.
#ifndef IVDE_PAIR_INFLIGHT
#define IVDE_PAIR_INFLIGHT 3
#endif
// With texels of 16-bit code values the two-pixel sweep keeps two pairs in
// flight (75 VGPRs at six waves): 3-4% faster than three at 256 and 512
// levels on the 8-view 1080p arc scene at 12 bits; the four-pixel sweep
// keeps three (two were 2% slower at 128 levels), as do both with halves.
#define IVDE_PAIR16_INFLIGHT 2
#define IVDE_PAIR_WAVES_PER_SIMD 6
// Four pixels per step keep four passes' sums, counts and levels live: at
// six waves per SIMD they spilled 68 bytes outside the pixel loops; at five
// (95 VGPRs, nothing spilled) the four-pixel sweep ran 2-6% faster on the
// 8-view 1080p arc rig at 64 to 512 levels.
#define IVDE_QUAD_WAVES_PER_SIMD 5
// 0 (a measurement build): chunks inside the validity band run the tested
// loop as well, which must give bitwise the same volume.
#ifndef IVDE_PAIR_INSIDE
#define IVDE_PAIR_INSIDE 1
#endif

// Wave steps of the pixel-pair sweep a wave has taken since its last flush
// (wave-uniform): all, on projected records, on chunks inside the band.
struct PairSteps {
    uint32_t all = 0, projected = 0, inside = 0;
};

// G pixels per wave step (2: pairs, 4: quads): lane group h = lane / (64 / G)
// takes records h, h + G, ...; lane k of a group takes level
// 64 b + (64 / G) q + k in pass q.
template <bool BIL, bool F16OUT, int G, bool U16>
__device__ __forceinline__ void sweep_task_pairs(const Problem *__restrict__ P, const Task task, uint4 *st,
                                                 PairSide<U16> *cr, PairSteps &ns)
{
    constexpr int PU = (U16 && G == 2) ? IVDE_PAIR16_INFLIGHT : IVDE_PAIR_INFLIGHT;
    constexpr int PW = kWave / G;   // lanes per group = levels per pass
    const int lane = lane_id();
    const int h = lane / PW, k = lane % PW;
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
    const int front_all = ldu(&vc->front_all);
    const uint32_t front_targets = ldu(&vc->front_targets);
    const float g[3] = {ldu(&vc->g[0]), ldu(&vc->g[1]), ldu(&vc->g[2])};

    const int lbase = task.lblock * kWave;
    const int passes = min(G, (L - lbase + PW - 1) / PW);
    int lab[G];
    float sig[G], best[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        lab[q] = lbase + q * PW + k;
        // lanes past the last level repeat it (their sums are never stored)
        sig[q] = sigma[c * L + min(lab[q], L - 1)];
        best[q] = __builtin_inff();
    }
    const int np = p1 - p0;
    // the task's first and last levels
    const float sig_a = ldu(sigma + c * L + lbase), sig_b = ldu(sigma + c * L + min(lbase + kWave, L) - 1);

    for (int ti = 0; ti < nt; ++ti) {
        const int c2 = ldu(&vc->targets[ti]);
        const ViewDesc *vt = views + c2;
        Target T;
        T.rs = U16 && BIL ? make_rsrc_cells(ldu(&vt->tex), ldu(&vt->tex_bytes))   // see project_pair
                         : make_rsrc(ldu(&vt->tex), ldu(&vt->tex_bytes));
        T.lo = 1.f - kEdge;
        T.hi_x = (float)ldu(&vt->W) + kEdge;
        T.hi_y = (float)ldu(&vt->H) + kEdge;
        T.tp = (uint32_t)ldu(&vt->tex_pitch);
        T.rowB = (int)T.tp * 8;
        const float *pc = reinterpret_cast<const float *>(pairs + c * n + c2);
        const f32x4 ha = ldu4(pc), hb = ldu4(pc + 4), hc = ldu4(pc + 8);
        const float H[9] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y, hb.z, hb.w, hc.x};
        T.e0 = hc.y;
        T.e1 = hc.z;
        T.e2 = hc.w;
        const int front = front_all ? (((front_targets >> c2) & 1u) ? 2 : 1) : 0;
        float acc[G];
        uint64_t acci[G];
        int cnt[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            acc[q] = 0.f;
            acci[q] = 0;
            cnt[q] = 0;
        }
        for (int b0 = 0; b0 < np; b0 += kPairStage) {
            const int m = min(kPairStage, np - b0);
            const uint32_t steps = (uint32_t)(passes * ((m + G - 1) / G));
            ns.all += steps;
            if (front == 2) {
                ns.projected += steps;
                const bool inside = stage_projected<U16>(pix, p0 + b0, m, H, T, sig_a, sig_b, st, cr);
                if (IVDE_PAIR_INSIDE && inside) {
                    ns.inside += steps;
#pragma unroll
                    for (int q = 0; q < G; ++q)
                        if (q < passes)
                            sweep_pair_projected<PU, BIL, 3, G, U16>(st, cr, m, h, T, sig[q], acc[q], acci[q], cnt[q]);
                } else {
#pragma unroll
                    for (int q = 0; q < G; ++q)
                        if (q < passes)
                            sweep_pair_projected<PU, BIL, 2, G, U16>(st, cr, m, h, T, sig[q], acc[q], acci[q], cnt[q]);
                }
            } else {
                stage_records<U16>(pix, p0 + b0, m, st);
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (q >= passes) continue;
                    if (front == 1)
                        sweep_pair_records<PU, BIL, 1, G, U16>(st, m, h, H, g, T, sig[q], acc[q], acci[q], cnt[q]);
                    else
                        sweep_pair_records<PU, BIL, 0, G, U16>(st, m, h, H, g, T, sig[q], acc[q], acci[q], cnt[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            if (q >= passes) continue;
            // the groups' sums and counts: log2 G exchanges across the groups
            int c_all = cnt[q];
            float sum = acc[q];
            uint64_t sumi = acci[q];
#pragma unroll
            for (int o = PW; o < kWave; o <<= 1) {
                c_all += __shfl_xor(c_all, o);
                if constexpr (BIL) {
                    sum += __shfl_xor(sum, o);
                } else {
                    const uint32_t lo = (uint32_t)sumi, hi = (uint32_t)(sumi >> 32);
                    sumi += ((uint64_t)(uint32_t)__shfl_xor((int)hi, o) << 32) | (uint32_t)__shfl_xor((int)lo, o);
                }
            }
            if constexpr (!BIL) sum = (float)sumi;
            if (c_all > 0) best[q] = fminf(best[q], sum / ((float)c_all * norm));
        }
    }

    const int64_t row = row0 + s;
#pragma unroll
    for (int q = 0; q < G; ++q) {
        if (h == 0 && lab[q] < L) {
            const float o = best[q] == __builtin_inff() ? 1.0f : best[q];
            if constexpr (F16OUT)
                static_cast<__half *>(cost)[row * L + lab[q]] = __float2half_rn(o);
            else
                static_cast<float *>(cost)[row * L + lab[q]] = o;
        }
    }
}

template <bool BIL, bool F16OUT, int G, bool U16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    G == 4 ? IVDE_QUAD_WAVES_PER_SIMD : IVDE_PAIR_WAVES_PER_SIMD, G == 4 ? IVDE_QUAD_WAVES_PER_SIMD : IVDE_PAIR_WAVES_PER_SIMD))) void k_sweep_pairs(
    const Problem *__restrict__ probs, const Task *__restrict__ tasks, const int32_t *__restrict__ n_tasks,
    int32_t *__restrict__ cursors, int64_t max_tasks)
{
    extern __shared__ uint4 pair_stage[];
    const int wave = (int)(threadIdx.x / kWave), wpg = (int)(blockDim.x / kWave);
    uint4 *st = pair_stage + wave * kPairStage;
    PairSide<U16> *cr = reinterpret_cast<PairSide<U16> *>(pair_stage + wpg * kPairStage) + wave * kPairStage;
    const int lane = lane_id();
    const int64_t limit = min((int64_t)ldu(n_tasks), max_tasks);
    // per-XCD ranges and work stealing as in sweep_persistent_body
    const int home = (int)(blockIdx.x % kXcds);
    // step counts go to the problem of the tasks they came from, one flush
    // per change of problem and one at the end
    PairSteps ns;
    int cur = -1;
    auto flush = [&]() {
        if (cur >= 0 && lane == 0 && ns.all) {
            unsigned long long *d = ldu(&probs[cur].steps);
            atomicAdd(d, (unsigned long long)ns.all);
            atomicAdd(d + 1, (unsigned long long)ns.projected);
            atomicAdd(d + 2, (unsigned long long)ns.inside);
        }
        ns = PairSteps{};
    };
    for (int k = 0; k < kXcds; ++k) {
        const int x = (home + k) % kXcds;
        const int64_t lo = limit * x / kXcds, n = limit * (x + 1) / kXcds - lo;
        for (;;) {
            int t = 0;
            if (lane == 0) t = atomicAdd(&cursors[x], 1);
            t = uniform(__shfl(t, 0));
            if (t >= n) break;
            const Task task = ldu_task(tasks + lo + t);
            if (task.problem != cur) {
                flush();
                cur = task.problem;
            }
            sweep_task_pairs<BIL, F16OUT, G, U16>(probs + task.problem, task, st, cr, ns);
        }
    }
    flush();
}

// Cursors of the sweep to zero, then the task count.
__global__ void k_sweep_counters(int32_t *__restrict__ counters, int32_t n_tasks)
{
    if (threadIdx.x < kXcds) counters[threadIdx.x] = 0;
    if (threadIdx.x == kXcds) counters[kXcds] = n_tasks;
}

// ------------------------------------------------------------------ argmin
// V consecutive costs of one row as FP32 (V = 4: one 16- or 8-byte load).
template <bool F16, int V>
__device__ __forceinline__ void load_costs(const void *__restrict__ cost, int64_t i, float (&x)[V])
{
    if constexpr (V == 4) {
        if constexpr (F16) {
            const uint2 w = *reinterpret_cast<const uint2 *>(static_cast<const __half *>(cost) + i);
            x[0] = h_lo(w.x);
            x[1] = h_hi(w.x);
            x[2] = h_lo(w.y);
            x[3] = h_hi(w.y);
        } else {
            const float4 w = *reinterpret_cast<const float4 *>(static_cast<const float *>(cost) + i);
            x[0] = w.x;
            x[1] = w.y;
            x[2] = w.z;
            x[3] = w.w;
        }
    } else {
        x[0] = F16 ? __half2float(static_cast<const __half *>(cost)[i]) : static_cast<const float *>(cost)[i];
    }
}

// (value, label) keeps the lowest label among equal minima; NaN never wins.
__device__ __forceinline__ void argmin_take(float x, int l, float &bv, int &bi)
{
    if (x != x) x = __builtin_inff();
    if (x < bv || (x == bv && l < bi)) {
        bv = x;
        bi = l;
    }
}

// One wave per kRowsPerWave rows: lane k holds labels V k + 64 V i, and the
// loads of all the wave's rows are issued before the first comparison, so
// a wave keeps several rows of reads in flight.  V = 4 needs L % 4 == 0 and
// a 4-element-aligned base (checked on the host).
constexpr int kArgminRows = 4;

template <bool F16, int V>
__global__ __launch_bounds__(256) void k_argmin(const void *__restrict__ cost, int64_t rows, int L,
                                                int32_t *__restrict__ out)
{
    const int lane = lane_id();
    const int64_t r0 = ((int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kArgminRows;
    if (r0 >= rows) return;
    float bv[kArgminRows];
    int bi[kArgminRows];
#pragma unroll
    for (int q = 0; q < kArgminRows; ++q) {
        bv[q] = __builtin_inff();
        bi[q] = 0x7fffffff;
    }
    for (int l0 = lane * V; l0 < L; l0 += kWave * V) {
        float x[kArgminRows][V];
#pragma unroll
        for (int q = 0; q < kArgminRows; ++q) {
            const int64_t r = min(r0 + q, rows - 1);     // rows past the end repeat the last
            load_costs<F16, V>(cost, r * L + l0, x[q]);
        }
#pragma unroll
        for (int q = 0; q < kArgminRows; ++q)
#pragma unroll
            for (int k = 0; k < V; ++k) argmin_take(x[q][k], l0 + k, bv[q], bi[q]);
    }
#pragma unroll
    for (int q = 0; q < kArgminRows; ++q) {
        for (int d = 32; d >= 1; d >>= 1) {
            const float ov = __shfl_xor(bv[q], d);
            const int oi = __shfl_xor(bi[q], d);
            argmin_take(ov, oi, bv[q], bi[q]);
        }
        if (lane == 0 && r0 + q < rows) out[r0 + q] = bi[q] == 0x7fffffff ? 0 : bi[q];
    }
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

__global__ void k_copy_words(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, int64_t n4)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_copy_halves(const uint16_t *__restrict__ src, uint16_t *__restrict__ dst, int64_t n2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
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

hipError_t launch_pack(const Problem *dprob, const Extents &ext, int tex_u16, hipStream_t s)
{
    dim3 blk(64, 4);
    const int rows = 4 * kPackRows;
    dim3 grd((unsigned)((ext.max_w + 2 + 63) / 64), (unsigned)((ext.max_h + 2 + rows - 1) / rows), (unsigned)ext.n_views);
    if (tex_u16)
        hipLaunchKernelGGL(k_pack<true>, grd, blk, 0, s, dprob);
    else
        hipLaunchKernelGGL(k_pack<false>, grd, blk, 0, s, dprob);
    return hipGetLastError();
}

hipError_t launch_prepare(const Problem *dprob, const Extents &ext, int tex_u16, hipStream_t s, bool pack)
{
    const unsigned nv = (unsigned)ext.n_views;
    {
        const int n = ext.max_s > 2 * ext.max_bands ? ext.max_s : 2 * ext.max_bands;
        hipLaunchKernelGGL(k_index_init, dim3((unsigned)((n + 255) / 256), nv), dim3(256), 0, s, dprob);
    }
    if (pack) {
        const hipError_t e = launch_pack(dprob, ext, tex_u16, s);
        if (e != hipSuccess) return e;
    }
    {
        dim3 blk(64, 4);
        dim3 grd((unsigned)((ext.max_w + 63) / 64), (unsigned)((ext.max_h + kCountTileRows - 1) / kCountTileRows), nv);
        hipLaunchKernelGGL(k_seg_count, grd, blk, 0, s, dprob);
    }
    hipLaunchKernelGGL(k_scan, dim3(nv), dim3(1024), 0, s, dprob);
    hipLaunchKernelGGL(k_seg_fill, dim3((unsigned)((ext.max_s + 3) / 4), nv), dim3(256), 0, s, dprob);
    return hipGetLastError();
}

hipError_t launch_refresh(const Problem *dprob, const Extents &ext, int tex_u16, hipStream_t s)
{
    const unsigned nv = (unsigned)ext.n_views;
    {
        const hipError_t e = launch_pack(dprob, ext, tex_u16, s);
        if (e != hipSuccess) return e;
    }
    const int64_t px = (int64_t)ext.max_w * ext.max_h;
    const unsigned bx = (unsigned)std::min<int64_t>((px + 255) / 256, 4096);
    hipLaunchKernelGGL(k_seg_colour, dim3(bx, nv), dim3(256), 0, s, dprob);
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

// Dynamic LDS of the pixel-pair sweep: one record stage per wave (16-byte
// records, then what the projected form keeps beside each, PairSide).
static size_t pair_stage_bytes(int wpg, bool u16)
{
    return (size_t)wpg * kPairStage * (sizeof(uint4) + (u16 ? sizeof(uint2) : sizeof(uint16_t)));
}

template <int J, bool BIL, bool U16, bool F16OUT>
static hipError_t sweep_pers(const Problem *dprobs, const Task *tasks, const int32_t *n_tasks, int32_t *cursors,
                             int64_t max_tasks, int px, int wpg, int n_groups, hipStream_t s)
{
    if constexpr (J == 1) {
        if (px == 4)
            hipLaunchKernelGGL((k_sweep_pairs<BIL, F16OUT, 4, U16>), dim3((unsigned)n_groups), dim3(64 * wpg),
                               pair_stage_bytes(wpg, U16), s, dprobs, tasks, n_tasks, cursors, max_tasks);
        else if (px == 2)
            hipLaunchKernelGGL((k_sweep_pairs<BIL, F16OUT, 2, U16>), dim3((unsigned)n_groups), dim3(64 * wpg),
                               pair_stage_bytes(wpg, U16), s, dprobs, tasks, n_tasks, cursors, max_tasks);
        else
            hipLaunchKernelGGL((k_sweep_persistent_j1<BIL, F16OUT, U16>), dim3((unsigned)n_groups), dim3(64 * wpg), 0,
                               s, dprobs, tasks, n_tasks, cursors, max_tasks);
    } else
        hipLaunchKernelGGL((k_sweep_persistent<J, BIL, U16, F16OUT>), dim3((unsigned)n_groups), dim3(64 * wpg), 0,
                           s, dprobs, tasks, n_tasks, cursors, max_tasks);
    return hipGetLastError();
}

#define IVDE_DISPATCH_FLAGS(FN, J, ...)                                                      \
    do {                                                                                     \
        if (bilinear) {                                                                      \
            if (tex_u16) {                                                                   \
                return f16out ? FN<J, true, true, true>(__VA_ARGS__) : FN<J, true, true, false>(__VA_ARGS__); \
            }                                                                                \
            return f16out ? FN<J, true, false, true>(__VA_ARGS__) : FN<J, true, false, false>(__VA_ARGS__); \
        }                                                                                    \
        if (tex_u16) {                                                                       \
            return f16out ? FN<J, false, true, true>(__VA_ARGS__) : FN<J, false, true, false>(__VA_ARGS__); \
        }                                                                                    \
        return f16out ? FN<J, false, false, true>(__VA_ARGS__) : FN<J, false, false, false>(__VA_ARGS__); \
    } while (0)

template <int J, bool BIL, bool U16, bool F16OUT>
static hipError_t occ(int px, int wpg, int *per_cu)
{
    if constexpr (J == 1) {
        if (px == 4)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sweep_pairs<BIL, F16OUT, 4, U16>, 64 * wpg,
                                                                pair_stage_bytes(wpg, U16));
        if (px == 2)
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sweep_pairs<BIL, F16OUT, 2, U16>, 64 * wpg,
                                                                pair_stage_bytes(wpg, U16));
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sweep_persistent_j1<BIL, F16OUT, U16>, 64 * wpg,
                                                            0);
    } else
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_sweep_persistent<J, BIL, U16, F16OUT>,
                                                            64 * wpg, 0);
}

hipError_t sweep_persistent_occupancy(int J, int px, int bilinear, int tex_u16, int f16out, int wpg, int *per_cu)
{
    const int f16 = f16out;
#define IVDE_OCC(JJ)                                                                                   \
    do {                                                                                              \
        if (bilinear) {                                                                               \
            if (tex_u16) return f16 ? occ<JJ, true, true, true>(px, wpg, per_cu) : occ<JJ, true, true, false>(px, wpg, per_cu); \
            return f16 ? occ<JJ, true, false, true>(px, wpg, per_cu) : occ<JJ, true, false, false>(px, wpg, per_cu); \
        }                                                                                             \
        if (tex_u16) return f16 ? occ<JJ, false, true, true>(px, wpg, per_cu) : occ<JJ, false, true, false>(px, wpg, per_cu); \
        return f16 ? occ<JJ, false, false, true>(px, wpg, per_cu) : occ<JJ, false, false, false>(px, wpg, per_cu); \
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
                                   int32_t *cursors, int64_t max_tasks, int J, int px, int bilinear, int tex_u16,
                                   int f16out, int wpg, int n_groups, hipStream_t s)
{
    switch (J) {
    case 1: IVDE_DISPATCH_FLAGS(sweep_pers, 1, dprobs, tasks, n_tasks_dev, cursors, max_tasks, px, wpg, n_groups, s);
    case 2: IVDE_DISPATCH_FLAGS(sweep_pers, 2, dprobs, tasks, n_tasks_dev, cursors, max_tasks, px, wpg, n_groups, s);
    case 4: IVDE_DISPATCH_FLAGS(sweep_pers, 4, dprobs, tasks, n_tasks_dev, cursors, max_tasks, px, wpg, n_groups, s);
    case 8: IVDE_DISPATCH_FLAGS(sweep_pers, 8, dprobs, tasks, n_tasks_dev, cursors, max_tasks, px, wpg, n_groups, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(const Problem *dprobs, const Task *tasks, int64_t n_tasks, int J, int px, int bilinear,
                        int tex_u16, int f16out, int wpg, int32_t *counters, hipStream_t s)
{
    if (n_tasks <= 0) return hipSuccess;
    if (n_tasks > 0x7fffffff) return hipErrorInvalidValue;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = sweep_persistent_occupancy(J, px, bilinear, tex_u16, f16out, wpg, &per_cu)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sweep_counters, dim3(1), dim3(64), 0, s, counters, (int32_t)n_tasks);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int n_groups = std::max(1, cus) * std::max(1, per_cu);
    return launch_sweep_persistent(dprobs, tasks, counters + kXcds, counters, n_tasks, J, px, bilinear, tex_u16,
                                   f16out, wpg, n_groups, s);
}

hipError_t launch_argmin(const void *cost, int f16, int64_t rows, int L, int32_t *out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    const int64_t per_block = 4 * kArgminRows;
    const int64_t blocks = (rows + per_block - 1) / per_block;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const size_t esz = f16 ? 2 : 4;
    const bool vec = L % 4 == 0 && reinterpret_cast<uintptr_t>(cost) % (4 * esz) == 0;
    const dim3 g((unsigned)blocks), b(256);
    if (f16 && vec)
        hipLaunchKernelGGL((k_argmin<true, 4>), g, b, 0, s, cost, rows, L, out);
    else if (f16)
        hipLaunchKernelGGL((k_argmin<true, 1>), g, b, 0, s, cost, rows, L, out);
    else if (vec)
        hipLaunchKernelGGL((k_argmin<false, 4>), g, b, 0, s, cost, rows, L, out);
    else
        hipLaunchKernelGGL((k_argmin<false, 1>), g, b, 0, s, cost, rows, L, out);
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
    const uintptr_t a = reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst);
    if (bytes % 2 || a % 2) return hipErrorInvalidValue;
    if (bytes % 16 == 0 && a % 16 == 0) {
        const int64_t n16 = bytes / 16;
        int64_t blocks = (n16 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_copy_bytes, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint4 *>(src),
                           static_cast<uint4 *>(dst), n16);
    } else if (bytes % 4 == 0 && a % 4 == 0) {
        const int64_t n4 = bytes / 4;
        int64_t blocks = (n4 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_copy_words, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint32_t *>(src),
                           static_cast<uint32_t *>(dst), n4);
    } else {
        // half-precision volumes with an odd number of entries
        const int64_t n2 = bytes / 2;
        int64_t blocks = (n2 + 255) / 256;
        if (blocks > 8192) blocks = 8192;
        hipLaunchKernelGGL(k_copy_halves, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const uint16_t *>(src),
                           static_cast<uint16_t *>(dst), n2);
    }
    return hipGetLastError();
}

}  // namespace ivde
