// gfx950 kernels of the energy terms around the matching cost: segment
// statistics (centre and mean colour), the window matching core of
// Sec. III-C (Eqs. (4), (5)) and the temporal rule of Sec. III-E.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "ivde_internal.h"

namespace ivde {

namespace {

// ------------------------------------------------------------------ segment statistics
// Count, centre (centroid rounded half up) and mean colour of every segment,
// one wave per segment over its pixel records; integer sums, so the result
// does not depend on the summation order.
__global__ void k_seg_stats(const Problem *__restrict__ P, int32_t *__restrict__ count_flat)
{
    const ViewDesc &v = P->views[blockIdx.y];
    const int lane = lane_id();
    const int s = uniform(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    if (s >= v.S) return;
    const int p0 = v.offsets[s], p1 = v.offsets[s + 1];
    unsigned long long sx = 0, sy = 0, sc[3] = {0, 0, 0};
    const float4 *rec = reinterpret_cast<const float4 *>(v.pixrec);
    for (int i = p0 + lane; i < p1; i += kWave) {
        const float4 r0 = rec[2 * (int64_t)i], r1 = rec[2 * (int64_t)i + 1];
        sx += (unsigned long long)r0.x;
        sy += (unsigned long long)r0.y;
        sc[0] += (unsigned long long)r0.w;
        sc[1] += (unsigned long long)r1.x;
        sc[2] += (unsigned long long)r1.y;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        sx += __shfl_xor(sx, d);
        sy += __shfl_xor(sy, d);
        for (int c = 0; c < 3; ++c) sc[c] += __shfl_xor(sc[c], d);
    }
    if (lane == 0) {
        const int n = p1 - p0;
        if (count_flat) count_flat[v.row0 + s] = n;
        if (n == 0) {
            v.centre[2 * s] = v.centre[2 * s + 1] = -1;
            for (int c = 0; c < 4; ++c) v.mean[4 * s + c] = 0.f;
        } else {
            const double dn = (double)n;
            v.centre[2 * s] = (int)floor((double)sx / dn + 0.5);
            v.centre[2 * s + 1] = (int)floor((double)sy / dn + 0.5);
            for (int c = 0; c < 3; ++c) v.mean[4 * s + c] = (float)((double)sc[c] / dn);
            v.mean[4 * s + 3] = 0.f;
        }
    }
}

// ------------------------------------------------------------------ window matching core
template <bool TEXF32>
__device__ __forceinline__ void texel_at(const void *tex, uint32_t tp, int X, int Y, float &y, float &u, float &v)
{
    if constexpr (TEXF32) {
        const float4 t = static_cast<const float4 *>(tex)[(int64_t)Y * tp + X];
        y = t.x;
        u = t.y;
        v = t.z;
    } else {
        const uint2 t = static_cast<const uint2 *>(tex)[(int64_t)Y * tp + X];
        y = h_lo(t.x);
        u = h_hi(t.x);
        v = h_lo(t.y);
    }
}

// The paper's matching core at the segment centre (Sec. III-C, Eq. (4))
// towards the neighbouring views c - 1 (slot 0) and c + 1 (slot 1) of
// Sec. III-B.  Lanes are labels: each projects the centre to its level,
// rounds to the nearest pixel of the target and compares the (2r+1)^2
// windows (taps clamped to the images).  m is in 8-bit code values; hit is
// the volume row of the target segment under the projected centre.
template <bool TEXF32>
__global__ __launch_bounds__(256) void k_window(const Problem *__restrict__ P, const Task *__restrict__ tasks,
                                                int64_t n_tasks, int radius, float *__restrict__ m_out,
                                                int32_t *__restrict__ hit_out)
{
    const int lane = lane_id();
    const int64_t t = (int64_t)blockIdx.x * (blockDim.x / kWave) + uniform(threadIdx.x / kWave);
    if (t >= n_tasks) return;
    const Task task = ldu_task(tasks + t);
    const int c = task.view, s = task.seg;
    const int L = ldu(&P->L), n = ldu(&P->n_views);
    const ViewDesc *views = ldu(&P->views);
    const PairConst *pairs = ldu(&P->pairs);
    const float scale = (float)(1 << (ldu(&P->bit_depth) - 8));
    const ViewDesc *vc = views + c;
    const int *cen = ldu(&vc->centre);
    const int cx = ldu(cen + 2 * s), cy = ldu(cen + 2 * s + 1);
    const int Wc = ldu(&vc->W), Hc = ldu(&vc->H);
    const void *stex = ldu(&vc->tex);
    const uint32_t stp = (uint32_t)ldu(&vc->tex_pitch);
    const int64_t row = ldu(&vc->row0) + s;
    const int l = task.lblock * kWave + lane;
    const float sig = l < L ? ldu(&P->sigma)[c * L + l] : 0.f;
    const float taps = (float)((2 * radius + 1) * (2 * radius + 1));
    for (int slot = 0; slot < 2; ++slot) {
        const int c2 = slot == 0 ? c - 1 : c + 1;
        float m = __builtin_nanf("");
        int hit = -1;
        if (c2 >= 0 && c2 < n && cx >= 0) {
            const ViewDesc *vt = views + c2;
            const float *pc = reinterpret_cast<const float *>(pairs + c * n + c2);
            const f32x4 ha = ldu4(pc), hb = ldu4(pc + 4), hc = ldu4(pc + 8);
            const float x = (float)cx, y = (float)cy;
            const float gp = fmaf(ldu(&vc->g[0]), x, fmaf(ldu(&vc->g[1]), y, ldu(&vc->g[2])));
            const float w = sig * gp;
            const float hx = fmaf(w, hc.y, fmaf(ha.x, x, fmaf(ha.y, y, ha.z)));
            const float hy = fmaf(w, hc.z, fmaf(ha.w, x, fmaf(hb.x, y, hb.y)));
            const float hz = fmaf(w, hc.w, fmaf(hb.z, x, fmaf(hb.w, y, hc.x)));
            const float r = __builtin_amdgcn_rcpf(hz);
            // bordered texel frame: pixel (x, y) is texel (x + 1, y + 1)
            const float fx = floorf(hx * r + 0.5f), fy = floorf(hy * r + 0.5f);
            const int W2 = ldu(&vt->W), H2 = ldu(&vt->H);
            const bool valid = (w > 0.f) & (hz > 0.f) & (fx >= 1.f) & (fx <= (float)W2) & (fy >= 1.f) &
                               (fy <= (float)H2) & (l < L);
            if (valid) {
                const int tx = (int)fx - 1, ty = (int)fy - 1;
                const void *ttex = ldu(&vt->tex);
                const uint32_t ttp = (uint32_t)ldu(&vt->tex_pitch);
                float sum = 0.f;
                for (int dy = -radius; dy <= radius; ++dy)
                    for (int dx = -radius; dx <= radius; ++dx) {
                        float ay, au, av, by, bu, bv;
                        texel_at<TEXF32>(stex, stp, min(max(cx + dx, 0), Wc - 1) + 1, min(max(cy + dy, 0), Hc - 1) + 1,
                                         ay, au, av);
                        texel_at<TEXF32>(ttex, ttp, min(max(tx + dx, 0), W2 - 1) + 1, min(max(ty + dy, 0), H2 - 1) + 1,
                                         by, bu, bv);
                        sum += fabsf(ay - by) + fabsf(au - bu) + fabsf(av - bv);
                    }
                m = sum / (taps * scale);
                const int32_t *seg2 = ldu(&vt->seg);
                hit = (int)ldu(&vt->row0) + seg2[(int64_t)ty * ldu(&vt->seg_pitch) + tx];
            }
        }
        if (l < L) {
            const int64_t o = (row * 2 + slot) * L + l;
            m_out[o] = m;
            hit_out[o] = hit;
        }
    }
}

// Eq. (5) summed over the two neighbours for a fixed labelling.
__global__ void k_window_energy(int64_t rows, int L, const float *__restrict__ m, const int32_t *__restrict__ hit,
                                const int32_t *__restrict__ labelling, float K, float *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * L) return;
    const int64_t r = i / L;
    const int l = (int)(i - r * L);
    float e = 0.f;
    for (int slot = 0; slot < 2; ++slot) {
        const int64_t o = (r * 2 + slot) * L + l;
        const int h = hit[o];
        if (h >= 0 && h < rows && labelling[h] == l) e += fminf(0.f, m[o] - K);
    }
    out[i] = e;
}

// ------------------------------------------------------------------ temporal rule
// Sec. III-E: a segment is unchanged when every mean colour component moved
// by less than t_i since the I frame (it then adopts the I frame's result,
// source 2) or by less than t_p since the previous frame (source 1);
// otherwise it is recomputed (source 0).  The stricter I-frame test is taken
// first.  counts[k] += number of rows with source k.
__global__ void k_temporal_rule(int64_t rows, const float *__restrict__ mean, const float *__restrict__ prev,
                                const float *__restrict__ iframe, float t_p, float t_i, uint8_t *__restrict__ source,
                                uint8_t *__restrict__ changed, int32_t *__restrict__ counts)
{
    const int lane = lane_id();
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int src = -1;
    if (r < rows) {
        const float4 m = reinterpret_cast<const float4 *>(mean)[r];
        const float4 p = reinterpret_cast<const float4 *>(prev)[r];
        const float dp = fmaxf(fabsf(m.x - p.x), fmaxf(fabsf(m.y - p.y), fabsf(m.z - p.z)));
        bool from_i = false;
        if (iframe) {
            const float4 q = reinterpret_cast<const float4 *>(iframe)[r];
            const float di = fmaxf(fabsf(m.x - q.x), fmaxf(fabsf(m.y - q.y), fabsf(m.z - q.z)));
            from_i = di < t_i;
        }
        src = from_i ? 2 : (dp < t_p ? 1 : 0);
        source[r] = (uint8_t)src;
        if (changed) changed[r] = src == 0;
    }
    if (counts) {
        for (int k = 0; k < 3; ++k) {
            const uint64_t b = __ballot(src == k);
            if (lane == 0 && b) atomicAdd(&counts[k], __builtin_popcountll(b));
        }
    }
}

// Copy the rows whose source is `which` from one volume to another.
__global__ void k_copy_rows_where(int64_t rows, int row_bytes, const uint8_t *__restrict__ source, int which,
                                  const uint8_t *__restrict__ from, uint8_t *__restrict__ to)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // one 4-byte word per thread
    const int words = row_bytes / 4;
    if (i >= rows * words) return;
    const int64_t r = i / words;
    if (source[r] != which) return;
    reinterpret_cast<uint32_t *>(to)[i] = reinterpret_cast<const uint32_t *>(from)[i];
}

}  // namespace

hipError_t launch_segment_stats(const Problem *dprob, const Extents &ext, int32_t *count_flat, hipStream_t s)
{
    hipLaunchKernelGGL(k_seg_stats, dim3((unsigned)((ext.max_s + 3) / 4), (unsigned)ext.n_views), dim3(256), 0, s,
                       dprob, count_flat);
    return hipGetLastError();
}

hipError_t launch_temporal_rule(int64_t rows, const float *mean, const float *prev, const float *iframe, float t_p,
                                float t_i, uint8_t *source, uint8_t *changed, int32_t *counts, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    const int64_t blocks = (rows + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_temporal_rule, dim3((unsigned)blocks), dim3(256), 0, s, rows, mean, prev, iframe, t_p, t_i,
                       source, changed, counts);
    return hipGetLastError();
}

hipError_t launch_copy_rows_where(int64_t rows, int row_bytes, const uint8_t *source, int which, const void *from,
                                  void *to, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    if (row_bytes % 4) return hipErrorInvalidValue;
    const int64_t n = rows * (row_bytes / 4);
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy_rows_where, dim3((unsigned)blocks), dim3(256), 0, s, rows, row_bytes, source, which,
                       static_cast<const uint8_t *>(from), static_cast<uint8_t *>(to));
    return hipGetLastError();
}

hipError_t launch_window(const Problem *dprob, const Task *tasks, int64_t n_tasks, int radius, int tex_f32,
                         float *m_out, int32_t *hit_out, hipStream_t s)
{
    if (n_tasks <= 0) return hipSuccess;
    const int64_t blocks = (n_tasks + 3) / 4;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (tex_f32)
        hipLaunchKernelGGL(k_window<true>, dim3((unsigned)blocks), dim3(256), 0, s, dprob, tasks, n_tasks, radius, m_out,
                           hit_out);
    else
        hipLaunchKernelGGL(k_window<false>, dim3((unsigned)blocks), dim3(256), 0, s, dprob, tasks, n_tasks, radius,
                           m_out, hit_out);
    return hipGetLastError();
}

hipError_t launch_window_energy(int64_t rows, int L, const float *m, const int32_t *hit, const int32_t *labelling,
                                float K, float *out, hipStream_t s)
{
    const int64_t n = rows * L;
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_window_energy, dim3((unsigned)blocks), dim3(256), 0, s, rows, L, m, hit, labelling, K, out);
    return hipGetLastError();
}

}  // namespace ivde
