// gfx950 kernels of the energy terms around the matching cost: segment
// statistics (centre and mean colour), the window matching core of
// Sec. III-C (Eqs. (4), (5)), the temporal rule of Sec. III-E and the
// intra-view term of Sec. III-D (Eqs. (2), (3)).
#include <algorithm>

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
// x, y, Y, Cb, Cr summed over records [p0, p1), across the wave; integer
// sums, exact in T as long as they fit.
template <typename T>
__device__ __forceinline__ void record_sums(const float4 *rec, int p0, int p1, int lane, unsigned long long (&out)[5])
{
    T acc[5] = {0, 0, 0, 0, 0};
    for (int i = p0 + lane; i < p1; i += kWave) {
        const float4 r0 = ldg(rec + 2 * (int64_t)i), r1 = ldg(rec + 2 * (int64_t)i + 1);
        acc[0] += (T)r0.x;
        acc[1] += (T)r0.y;
        acc[2] += (T)r0.w;
        acc[3] += (T)r1.x;
        acc[4] += (T)r1.y;
    }
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int c = 0; c < 5; ++c) out[c] = wave_sum_u32(acc[c]);
    } else {
        for (int d = 32; d >= 1; d >>= 1)
#pragma unroll
            for (int c = 0; c < 5; ++c) acc[c] += __shfl_xor(acc[c], d);
#pragma unroll
        for (int c = 0; c < 5; ++c) out[c] = (unsigned long long)acc[c];
    }
}

__global__ __launch_bounds__(256) void k_seg_stats(const Problem *__restrict__ P, int32_t *__restrict__ count_flat)
{
    const ViewDesc *vd = ldu(&P->views) + blockIdx.y;
    const int lane = lane_id();
    const int s = uniform(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    if (s >= ldu(&vd->S)) return;
    const int32_t *offs = ldu(&vd->offsets);
    const int p0 = ldu(offs + s), p1 = ldu(offs + s + 1);
    const float4 *rec = reinterpret_cast<const float4 *>(ldu(&vd->pixrec));
    unsigned long long sum[5];
    // coordinates and samples are below 2^16, so sums over at most 2^16
    // pixels fit 32 bits (half the cross-lane traffic of 64-bit sums)
    if (p1 - p0 <= 65536)
        record_sums<uint32_t>(rec, p0, p1, lane, sum);
    else
        record_sums<unsigned long long>(rec, p0, p1, lane, sum);
    const unsigned long long sx = sum[0], sy = sum[1], sc[3] = {sum[2], sum[3], sum[4]};
    if (lane == 0) {
        const int n = p1 - p0;
        int32_t *centre = ldu(&vd->centre) + 2 * s;
        float *mean = ldu(&vd->mean) + 4 * s;
        if (count_flat) stg(count_flat + ldu(&vd->row0) + s, (int32_t)n);
        if (n == 0) {
            stg(centre, -1);
            stg(centre + 1, -1);
            stg(reinterpret_cast<float4 *>(mean), make_float4(0.f, 0.f, 0.f, 0.f));
        } else {
            const double dn = (double)n;
            stg(centre, (int)floor((double)sx / dn + 0.5));
            stg(centre + 1, (int)floor((double)sy / dn + 0.5));
            stg(reinterpret_cast<float4 *>(mean), make_float4((float)((double)sc[0] / dn), (float)((double)sc[1] / dn),
                                                              (float)((double)sc[2] / dn), 0.f));
        }
    }
}

// Pixel sums of every segment straight from the segment map, without the
// segment index: count, sum x, sum y and the sums of Y, Cb, Cr (chroma at
// (x >> k, y >> k)), in 64-bit integers at [row][6].  A 256-thread block
// covers a 64 x kSumRows tile; each wave row is split into runs of equal id,
// a run's colour sums are differences of wave prefix sums, and the runs of a
// tile meet in an LDS table before one set of global atomics per distinct
// segment.  Integer sums do not depend on the order of the additions.
constexpr int kSumRows = 16;
constexpr int kSumSlots = 128;

__device__ __forceinline__ void sums_global(unsigned long long *row, uint32_t n, uint32_t sx, uint32_t sy,
                                            uint32_t c0, uint32_t c1, uint32_t c2)
{
    atomicAdd(row + 0, (unsigned long long)n);
    atomicAdd(row + 1, (unsigned long long)sx);
    atomicAdd(row + 2, (unsigned long long)sy);
    atomicAdd(row + 3, (unsigned long long)c0);
    atomicAdd(row + 4, (unsigned long long)c1);
    atomicAdd(row + 5, (unsigned long long)c2);
}

__global__ __launch_bounds__(256) void k_seg_sums(const Problem *__restrict__ P, unsigned long long *__restrict__ sums)
{
    __shared__ int key[kSumSlots];
    __shared__ uint32_t acc[6][kSumSlots];
    const ViewDesc *vd = ldu(&P->views) + blockIdx.z;
    const int W = ldu(&vd->W), H = ldu(&vd->H), S = ldu(&vd->S);
    const int32_t *seg = ldu(&vd->seg);
    const int64_t sp = ldu(&vd->seg_pitch);
    int32_t *flag = ldu(&P->flag);
    const Planes pl = planes_of(P, vd);
    const int k = pl.k;
    const int tid = threadIdx.y * kWave + threadIdx.x;
    if (tid < kSumSlots) {
        key[tid] = -1;
        for (int c = 0; c < 6; ++c) acc[c][tid] = 0;
    }
    __syncthreads();
    const int lane = threadIdx.x;
    const int x = blockIdx.x * kWave + lane;
    unsigned long long *rows = sums + 6 * ldu(&vd->row0);
    constexpr int kRowsPerWave = kSumRows / 4;
    int ids[kRowsPerWave];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int y = blockIdx.y * kSumRows + 4 * r + threadIdx.y;
        ids[r] = x < W && y < H ? ldg(seg + (int64_t)y * sp + x) : -1;
    }
    for (int r = 0; r < kRowsPerWave; ++r) {
        const int y = blockIdx.y * kSumRows + 4 * r + threadIdx.y;
        const bool in = x < W && y < H;
        int id = ids[r];
        if (in && (id < 0 || id >= S)) {
            atomicOr(flag, 1);
            id = -1;
        }
        uint32_t col[3] = {0, 0, 0};
        if (id >= 0) {
            col[0] = plane_u(pl, 0, (int64_t)y * pl.pitch[0] + x);
            col[1] = plane_u(pl, 1, (int64_t)(y >> k) * pl.pitch[1] + (x >> k));
            col[2] = plane_u(pl, 2, (int64_t)(y >> k) * pl.pitch[2] + (x >> k));
        }
        // inclusive prefix sums over the wave row (at most 64 x 65535 each)
        uint32_t pre[3] = {col[0], col[1], col[2]};
        for (int d = 1; d < kWave; d <<= 1)
            for (int c = 0; c < 3; ++c) {
                const uint32_t t = __shfl_up(pre[c], d);
                if (lane >= d) pre[c] += t;
            }
        const int prev = __shfl_up(id, 1);
        const int next = __shfl_down(id, 1);
        const bool head = id >= 0 && (lane == 0 || prev != id);
        const bool tail = id >= 0 && (lane == kWave - 1 || next != id);
        const uint64_t tails = __ballot(tail);
        // the run of a head lane ends at the first tail at or after it
        const int end = head ? __builtin_ctzll(tails & (~0ull << lane)) : lane;
        uint32_t before[3], upto[3];
        for (int c = 0; c < 3; ++c) {
            before[c] = __shfl_up(pre[c], 1);
            upto[c] = __shfl(pre[c], end);
        }
        if (head) {
            const uint32_t len = (uint32_t)(end - lane + 1);
            uint32_t cs[3];
            for (int c = 0; c < 3; ++c) cs[c] = upto[c] - (lane > 0 ? before[c] : 0u);
            const uint32_t sx = len * (uint32_t)x + len * (len - 1) / 2, sy = len * (uint32_t)y;
            int slot = id & (kSumSlots - 1), probe = 0;
            for (; probe < kSumSlots; ++probe) {
                const int k0 = atomicCAS(&key[slot], -1, id);
                if (k0 == -1 || k0 == id) break;
                slot = (slot + 1) & (kSumSlots - 1);
            }
            if (probe < kSumSlots) {
                atomicAdd(&acc[0][slot], len);
                atomicAdd(&acc[1][slot], sx);
                atomicAdd(&acc[2][slot], sy);
                for (int c = 0; c < 3; ++c) atomicAdd(&acc[3 + c][slot], cs[c]);
            } else {
                sums_global(rows + 6 * (int64_t)id, len, sx, sy, cs[0], cs[1], cs[2]);
            }
        }
    }
    __syncthreads();
    if (tid < kSumSlots && key[tid] >= 0)
        sums_global(rows + 6 * (int64_t)key[tid], acc[0][tid], acc[1][tid], acc[2][tid], acc[3][tid], acc[4][tid],
                    acc[5][tid]);
}

// Count, centre (centroid rounded half up) and mean colour from the sums,
// one thread per segment (the same formulas as k_seg_stats).
__global__ void k_seg_finish(const Problem *__restrict__ P, const unsigned long long *__restrict__ sums,
                             int32_t *__restrict__ count_flat)
{
    const ViewDesc *vd = ldu(&P->views) + blockIdx.y;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ldu(&vd->S)) return;
    const int64_t row0 = ldu(&vd->row0);
    int32_t *centre = ldu(&vd->centre) + 2 * s;
    float *mean = ldu(&vd->mean) + 4 * s;
    const unsigned long long *r = sums + 6 * (row0 + s);
    const unsigned long long n = r[0];
    if (count_flat) count_flat[row0 + s] = (int32_t)n;
    if (n == 0) {
        stg(centre, -1);
        stg(centre + 1, -1);
        stg(reinterpret_cast<float4 *>(mean), make_float4(0.f, 0.f, 0.f, 0.f));
        return;
    }
    const double dn = (double)n;
    stg(centre, (int)floor((double)r[1] / dn + 0.5));
    stg(centre + 1, (int)floor((double)r[2] / dn + 0.5));
    stg(reinterpret_cast<float4 *>(mean), make_float4((float)((double)r[3] / dn), (float)((double)r[4] / dn),
                                                      (float)((double)r[5] / dn), 0.f));
}

// Tasks in row order (view, segment, label block), for kernels that need no
// spatial ordering of their work.
__global__ void k_row_tasks(const Problem *__restrict__ P, Task *__restrict__ tasks)
{
    const ViewDesc &v = P->views[blockIdx.y];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= v.S) return;
    const int nb = P->n_lblocks;
    Task *t = tasks + (v.row0 + s) * nb;
    for (int b = 0; b < nb; ++b) {
        Task tk;
        tk.problem = 0;
        tk.view = blockIdx.y;
        tk.seg = s;
        tk.lblock = b;
        t[b] = tk;
    }
}

// ------------------------------------------------------------------ window matching core
template <bool U16>
__device__ __forceinline__ void texel_at(const void *tex, uint32_t tp, int X, int Y, float &y, float &u, float &v)
{
    const uint2 t = static_cast<const uint2 *>(tex)[(int64_t)Y * tp + X];
    y = ch_lo<U16>(t.x);
    u = ch_hi<U16>(t.x);
    v = ch_lo<U16>(t.y);
}

// The paper's matching core at the segment centre (Sec. III-C, Eq. (4))
// towards the neighbouring views c - 1 (slot 0) and c + 1 (slot 1) of
// Sec. III-B.  Lanes are labels: each projects the centre to its level,
// rounds to the nearest pixel of the target and compares the (2r+1)^2
// windows (taps clamped to the images).  m is in 8-bit code values; hit is
// the volume row of the target segment under the projected centre.
// R > 0 fixes the radius at compile time: the source window (the same for
// every lane) is read once per wave and all target taps are issued before
// the first is used.  R == 0 takes any radius at run time.
template <bool U16, int R>
__global__ __launch_bounds__(256) void k_window(const Problem *__restrict__ P, const Task *__restrict__ tasks,
                                                int64_t n_tasks, int radius, float *__restrict__ m_out,
                                                int32_t *__restrict__ hit_out)
{
    constexpr int kTexB = 8;
    constexpr int kSide = 2 * R + 1;
    constexpr int kTaps = R > 0 ? kSide * kSide : 1;
    const int lane = lane_id();
    const int64_t t = (int64_t)blockIdx.x * (blockDim.x / kWave) + uniform(threadIdx.x / kWave);
    if (t >= n_tasks) return;
    if constexpr (R > 0) radius = R;
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
    float sy[kTaps], su[kTaps], sv[kTaps];
    if constexpr (R > 0) {
        if (cx >= 0) {
#pragma unroll
            for (int dy = 0; dy < kSide; ++dy)
#pragma unroll
                for (int dx = 0; dx < kSide; ++dx)
                    texel_at<U16>(stex, stp, min(max(cx + dx - R, 0), Wc - 1) + 1,
                                     min(max(cy + dy - R, 0), Hc - 1) + 1, sy[dy * kSide + dx], su[dy * kSide + dx],
                                     sv[dy * kSide + dx]);
        }
    }
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
                if constexpr (R > 0) {
                    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                        const_cast<void *>(ttex), (short)0, (int)ldu(&vt->tex_bytes), (int)0x00020000);
                    int colo[kSide], rowo[kSide];
#pragma unroll
                    for (int k = 0; k < kSide; ++k) {
                        colo[k] = (min(max(tx + k - R, 0), W2 - 1) + 1) * kTexB;
                        rowo[k] = (min(max(ty + k - R, 0), H2 - 1) + 1) * (int)ttp * kTexB;
                    }
                    if constexpr (R == 1) {
                        // the one-texel border repeats the edge pixels, so the
                        // taps of a row are the three texels from (tx, ty + k),
                        // and no clamp is needed: one 16-byte and one 8-byte load
                        uint2 tv[kTaps];
#pragma unroll
                        for (int k = 0; k < kSide; ++k) {
                            const int o = (ty + k) * (int)ttp * kTexB + tx * kTexB;
                            const uint4 ab = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
                            tv[3 * k] = make_uint2(ab.x, ab.y);
                            tv[3 * k + 1] = make_uint2(ab.z, ab.w);
                            tv[3 * k + 2] = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, o + 16, 0, 0));
                        }
#pragma unroll
                        for (int k = 0; k < kTaps; ++k)
                            sum += fabsf(sy[k] - ch_lo<U16>(tv[k].x)) + fabsf(su[k] - ch_hi<U16>(tv[k].x)) +
                                   fabsf(sv[k] - ch_lo<U16>(tv[k].y));
                    } else {
                        uint2 tv[kTaps];
#pragma unroll
                        for (int k = 0; k < kTaps; ++k)
                            tv[k] = __builtin_bit_cast(uint2, __builtin_amdgcn_raw_buffer_load_b64(
                                                                  rs, rowo[k / kSide] + colo[k % kSide], 0, 0));
#pragma unroll
                        for (int k = 0; k < kTaps; ++k)
                            sum += fabsf(sy[k] - ch_lo<U16>(tv[k].x)) + fabsf(su[k] - ch_hi<U16>(tv[k].x)) +
                                   fabsf(sv[k] - ch_lo<U16>(tv[k].y));
                    }
                } else {
                    for (int dy = -radius; dy <= radius; ++dy)
                        for (int dx = -radius; dx <= radius; ++dx) {
                            float ay, au, av, by, bu, bv;
                            texel_at<U16>(stex, stp, min(max(cx + dx, 0), Wc - 1) + 1,
                                             min(max(cy + dy, 0), Hc - 1) + 1, ay, au, av);
                            texel_at<U16>(ttex, ttp, min(max(tx + dx, 0), W2 - 1) + 1,
                                             min(max(ty + dy, 0), H2 - 1) + 1, by, bu, bv);
                            sum += fabsf(ay - by) + fabsf(au - bu) + fabsf(av - bv);
                        }
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

// Copy the rows whose source is `which` from one volume to another, one
// element of T (4 bytes, or 2 for half-precision rows of odd length) per
// thread.
template <typename T>
__global__ void k_copy_rows_where(int64_t rows, int row_elems, const uint8_t *__restrict__ source, int which,
                                  const T *__restrict__ from, T *__restrict__ to)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * row_elems) return;
    const int64_t r = i / row_elems;
    if (source[r] != which) return;
    to[i] = from[i];
}


// ------------------------------------------------------------------ intra-view term
// Sec. III-D: segments of one view are adjacent when a pixel of one is a
// 4-neighbour of a pixel of the other.  One wave per segment reads, for each
// of its pixels, the segment ids left, right, above and below, and extracts
// the distinct ids in increasing order by repeated wave minima; the lists
// are therefore sorted and independent of any scheduling.
constexpr int kAdjCache = 4;            // pixel batches whose neighbour ids stay in registers
constexpr int kNoSeg = 0x7fffffff;

__device__ __forceinline__ int wave_min(int v) { return wave_min_i32(v); }

// A view's segment map, read once per wave into scalar registers.
struct SegMap {
    const int32_t *seg;
    int64_t pitch;
    int W, H, S;
};

// Segment ids around pixel record i; kNoSeg outside the image, for the
// segment itself and for ids out of range (reported by the index kernels).
__device__ __forceinline__ void neighbours4(const SegMap &v, const float *rec, int i, int s, int (&c)[4])
{
    const float2 xy = ldg(reinterpret_cast<const float2 *>(rec + 8 * (int64_t)i));
    const int x = (int)xy.x, y = (int)xy.y;
    const int32_t *row = v.seg + (int64_t)y * v.pitch;
    const int t0 = x > 0 ? ldg(row + x - 1) : kNoSeg;
    const int t1 = x + 1 < v.W ? ldg(row + x + 1) : kNoSeg;
    const int t2 = y > 0 ? ldg(row + x - v.pitch) : kNoSeg;
    const int t3 = y + 1 < v.H ? ldg(row + x + v.pitch) : kNoSeg;
    c[0] = (t0 != s && t0 >= 0 && t0 < v.S) ? t0 : kNoSeg;
    c[1] = (t1 != s && t1 >= 0 && t1 < v.S) ? t1 : kNoSeg;
    c[2] = (t2 != s && t2 >= 0 && t2 < v.S) ? t2 : kNoSeg;
    c[3] = (t3 != s && t3 >= 0 && t3 < v.S) ? t3 : kNoSeg;
}

__device__ __forceinline__ int min_above(const int (&c)[4], int last, int m)
{
    for (int d = 0; d < 4; ++d)
        if (c[d] > last) m = min(m, c[d]);
    return m;
}

// WRITE = false: offsets[row + 1] = number of neighbours, and the first
// kAdjKeep neighbour ids in kept[row].  WRITE = true (after the scan): the
// neighbour rows and their Eq. (3) weights from offsets[row], entries at or
// beyond `capacity` skipped; rows with at most kAdjKeep neighbours copy them
// from kept (one lane each), longer lists are extracted again.
template <bool WRITE>
__global__ __launch_bounds__(256) void k_adjacency(const Problem *__restrict__ P, int64_t *__restrict__ offsets,
                                                   int32_t *__restrict__ index, float *__restrict__ beta,
                                                   int64_t capacity, float beta0, float eps, float inv_scale,
                                                   int32_t *__restrict__ kept)
{
    const ViewDesc *vd = ldu(&P->views) + blockIdx.y;
    const int lane = lane_id();
    const int s = uniform(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
    SegMap v;
    v.S = ldu(&vd->S);
    if (s >= v.S) return;
    const int64_t row0 = ldu(&vd->row0);
    const int64_t row = row0 + s;
    const float4 *mean = reinterpret_cast<const float4 *>(ldu(&vd->mean));
    int32_t *keep = kept + row * kAdjKeep;
    if (WRITE) {
        const int64_t o = offsets[row], n = offsets[row + 1] - o;
        if (n <= kAdjKeep) {
            if (lane < n && o + lane < capacity) {
                const int m = keep[lane];
                const float4 ms = ldg(mean + s);
                const float4 mt = ldg(mean + m);
                const float d = (fabsf(ms.x - mt.x) + fabsf(ms.y - mt.y) + fabsf(ms.z - mt.z)) * inv_scale;
                index[o + lane] = (int32_t)(row0 + m);
                beta[o + lane] = beta0 / (d + eps);
            }
            return;
        }
    }
    v.seg = ldu(&vd->seg);
    v.pitch = ldu(&vd->seg_pitch);
    v.W = ldu(&vd->W);
    v.H = ldu(&vd->H);
    const int32_t *voffs = ldu(&vd->offsets);
    const int p0 = ldu(voffs + s), p1 = ldu(voffs + s + 1);
    const float *rec = ldu(&vd->pixrec);
    const bool cached = p1 - p0 <= kAdjCache * kWave;
    int c[kAdjCache][4];
#pragma unroll
    for (int b = 0; b < kAdjCache; ++b) {
        const int i = p0 + b * kWave + lane;
        if (cached && i < p1)
            neighbours4(v, rec, i, s, c[b]);
        else
            c[b][0] = c[b][1] = c[b][2] = c[b][3] = kNoSeg;
    }
    const int64_t out = WRITE ? offsets[row] : 0;
    float4 ms = make_float4(0.f, 0.f, 0.f, 0.f);
    if (WRITE) ms = ldg(mean + s);
    int last = -1, k = 0;
    for (;;) {
        int m = kNoSeg;
        if (cached) {
#pragma unroll
            for (int b = 0; b < kAdjCache; ++b) m = min_above(c[b], last, m);
        } else {
            for (int i0 = p0; i0 < p1; i0 += kWave) {
                int cc[4] = {kNoSeg, kNoSeg, kNoSeg, kNoSeg};
                if (i0 + lane < p1) neighbours4(v, rec, i0 + lane, s, cc);
                m = min_above(cc, last, m);
            }
        }
        m = wave_min(m);
        if (m == kNoSeg) break;
        if (WRITE && lane == 0 && out + k < capacity) {
            index[out + k] = (int32_t)(row0 + m);
            const float4 mt = ldg(mean + m);
            const float d = (fabsf(ms.x - mt.x) + fabsf(ms.y - mt.y) + fabsf(ms.z - mt.z)) * inv_scale;
            beta[out + k] = beta0 / (d + eps);
        }
        if (!WRITE && lane == 0 && k < kAdjKeep) keep[k] = m;
        ++k;
        last = m;
    }
    if (!WRITE && lane == 0) offsets[row + 1] = k;
}

// In-place inclusive scan of a[1..n], a[0] = 0, in three phases: sums of
// 256-element blocks, a scan of those sums, then each block's own scan.
__device__ __forceinline__ int64_t wave_inclusive_scan(int64_t v)
{
    const int lane = lane_id();
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t u = __shfl_up(v, d);
        if (lane >= d) v += u;
    }
    return v;
}

// Inclusive scan over a 256-thread block; `total` receives the block sum.
__device__ __forceinline__ int64_t block_inclusive_scan(int64_t v, int64_t &total)
{
    __shared__ int64_t wsum[4];
    const int w = threadIdx.x / kWave;
    v = wave_inclusive_scan(v);
    if (lane_id() == kWave - 1) wsum[w] = v;
    __syncthreads();
    int64_t before = 0;
    for (int k = 0; k < w; ++k) before += wsum[k];
    total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return v + before;
}

__global__ __launch_bounds__(256) void k_scan_block_sums(const int64_t *__restrict__ a, int64_t n,
                                                         int64_t *__restrict__ sums)
{
    const int64_t i = 1 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t total;
    block_inclusive_scan(i <= n ? a[i] : 0, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the block sums in place (one workgroup, 256 at a time).
__global__ __launch_bounds__(256) void k_scan_sums(int64_t *__restrict__ sums, int64_t nb)
{
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < nb ? sums[i] : 0;
        int64_t total;
        const int64_t inc = block_inclusive_scan(v, total);
        if (i < nb) sums[i] = carry + inc - v;
        carry += total;
    }
}

__global__ __launch_bounds__(256) void k_scan_apply(int64_t *__restrict__ a, int64_t n,
                                                    const int64_t *__restrict__ sums)
{
    const int64_t i = 1 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    int64_t total;
    const int64_t inc = block_inclusive_scan(i <= n ? a[i] : 0, total);
    if (i <= n) a[i] = sums[blockIdx.x] + inc;
    if (blockIdx.x == 0 && threadIdx.x == 0) a[0] = 0;
}

// Eq. (2) with the neighbours' labels held: out[r][l] = sum over entries
// (r, t) of beta * |l - d_t|, only over t with fixed[t] != 0 when a mask is
// given.  One wave per row: the lanes load up to 64 of the row's entries at
// once (weight and neighbour label), then every entry is read back from its
// lane and applied to kIntraBlocks 64-label blocks, lanes being labels.
// Each label accumulates the entries in order, as a plain loop would.
constexpr int kIntraBlocks = 4;

__global__ __launch_bounds__(256) void k_intra_cost(int64_t rows, int L, int n_lblocks,
                                                    const int64_t *__restrict__ offsets,
                                                    const int32_t *__restrict__ index, const float *__restrict__ beta,
                                                    const int32_t *__restrict__ labelling,
                                                    const uint8_t *__restrict__ fixed, float *__restrict__ out)
{
    const int lane = lane_id();
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / kWave) + uniform(threadIdx.x / kWave);
    if (r >= rows) return;
    const int64_t e0 = ldu(offsets + r), e1 = ldu(offsets + r + 1);
    for (int b0 = 0; b0 < n_lblocks; b0 += kIntraBlocks) {
        float acc[kIntraBlocks];
#pragma unroll
        for (int k = 0; k < kIntraBlocks; ++k) acc[k] = 0.f;
        for (int64_t c = e0; c < e1; c += kWave) {
            const int64_t e = c + lane;
            float bj = 0.f;
            int dj = 0;
            bool ok = false;
            if (e < e1) {
                const int t = index[e];
                ok = t >= 0 && t < rows && (!fixed || fixed[t]);
                if (ok) {
                    bj = beta[e];
                    dj = labelling[t];
                }
            }
            const uint64_t use = __ballot(ok);
            const int n = (int)min((int64_t)kWave, e1 - c);
            for (int j = 0; j < n; ++j) {
                if (!((use >> j) & 1)) continue;
                const float bb = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bj), j));
                const int dd = __builtin_amdgcn_readlane(dj, j);
#pragma unroll
                for (int k = 0; k < kIntraBlocks; ++k) {
                    const int l = (b0 + k) * kWave + lane;
                    acc[k] = fmaf(bb, fabsf((float)(l - dd)), acc[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kIntraBlocks; ++k) {
            const int l = (b0 + k) * kWave + lane;
            if (b0 + k < n_lblocks && l < L) out[r * L + l] = acc[k];
        }
    }
}

// ------------------------------------------------------------------ depth maps
// Sec. III-B: each pixel takes the depth of its segment's level, read from
// the level-depth table the host composed in FP64; NaN marks an out-of-range
// segment id or level.
__global__ __launch_bounds__(256) void k_paint_depth(PaintViews pv, const int32_t *__restrict__ labels, int L,
                                                     const float *__restrict__ level_depth, float *__restrict__ out)
{
    const int v = blockIdx.y;
    const int W = pv.W[v], H = pv.H[v], S = pv.S[v];
    const int64_t n = (int64_t)W * H;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t y = i / W, x = i - y * W;
        const int s = pv.seg[v][y * pv.pitch[v] + x];
        float z = __builtin_nanf("");
        if (s >= 0 && s < S) {
            const int l = labels[pv.row0[v] + s];
            if (l >= 0 && l < L) z = level_depth[l];
        }
        out[pv.out0[v] + i] = z;
    }
}

}  // namespace

hipError_t launch_segment_stats(const Problem *dprob, const Extents &ext, int32_t *count_flat, hipStream_t s)
{
    hipLaunchKernelGGL(k_seg_stats, dim3((unsigned)((ext.max_s + 3) / 4), (unsigned)ext.n_views), dim3(256), 0, s,
                       dprob, count_flat);
    return hipGetLastError();
}

hipError_t launch_segment_sums(const Problem *dprob, const Extents &ext, unsigned long long *sums, int64_t rows,
                               int32_t *count_flat, Task *tasks, hipStream_t s)
{
    hipError_t e = launch_fill_i32(reinterpret_cast<int32_t *>(sums), 0, 12 * rows, s);
    if (e != hipSuccess) return e;
    const unsigned nv = (unsigned)ext.n_views;
    {
        dim3 blk(64, 4);
        dim3 grd((unsigned)((ext.max_w + 63) / 64), (unsigned)((ext.max_h + kSumRows - 1) / kSumRows), nv);
        hipLaunchKernelGGL(k_seg_sums, grd, blk, 0, s, dprob, sums);
    }
    const unsigned gs = (unsigned)((ext.max_s + 255) / 256);
    hipLaunchKernelGGL(k_seg_finish, dim3(gs, nv), dim3(256), 0, s, dprob, sums, count_flat);
    if (tasks) hipLaunchKernelGGL(k_row_tasks, dim3(gs, nv), dim3(256), 0, s, dprob, tasks);
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
    const uintptr_t a = reinterpret_cast<uintptr_t>(from) | reinterpret_cast<uintptr_t>(to);
    if (row_bytes <= 0 || row_bytes % 2 || a % 2) return hipErrorInvalidValue;
    const bool words = row_bytes % 4 == 0 && a % 4 == 0;
    const int elems = words ? row_bytes / 4 : row_bytes / 2;
    const int64_t n = rows * elems;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (words)
        hipLaunchKernelGGL(k_copy_rows_where<uint32_t>, dim3((unsigned)blocks), dim3(256), 0, s, rows, elems, source,
                           which, static_cast<const uint32_t *>(from), static_cast<uint32_t *>(to));
    else
        hipLaunchKernelGGL(k_copy_rows_where<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, s, rows, elems, source,
                           which, static_cast<const uint16_t *>(from), static_cast<uint16_t *>(to));
    return hipGetLastError();
}

hipError_t launch_window(const Problem *dprob, const Task *tasks, int64_t n_tasks, int radius, int tex_u16,
                         float *m_out, int32_t *hit_out, hipStream_t s)
{
    if (n_tasks <= 0) return hipSuccess;
    const int64_t blocks = (n_tasks + 3) / 4;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((unsigned)blocks), b(256);
    if (tex_u16) {
        if (radius == 1)
            hipLaunchKernelGGL((k_window<true, 1>), g, b, 0, s, dprob, tasks, n_tasks, radius, m_out, hit_out);
        else
            hipLaunchKernelGGL((k_window<true, 0>), g, b, 0, s, dprob, tasks, n_tasks, radius, m_out, hit_out);
    } else {
        if (radius == 1)
            hipLaunchKernelGGL((k_window<false, 1>), g, b, 0, s, dprob, tasks, n_tasks, radius, m_out, hit_out);
        else
            hipLaunchKernelGGL((k_window<false, 0>), g, b, 0, s, dprob, tasks, n_tasks, radius, m_out, hit_out);
    }
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

hipError_t launch_adjacency(const Problem *dprob, const Extents &ext, int write, int64_t *offsets, int32_t *index,
                            float *beta, int64_t capacity, float beta0, float eps, float inv_scale, int32_t *kept,
                            hipStream_t s)
{
    const dim3 grid((unsigned)((ext.max_s + 3) / 4), (unsigned)ext.n_views);
    if (write)
        hipLaunchKernelGGL(k_adjacency<true>, grid, dim3(256), 0, s, dprob, offsets, index, beta, capacity, beta0, eps,
                           inv_scale, kept);
    else
        hipLaunchKernelGGL(k_adjacency<false>, grid, dim3(256), 0, s, dprob, offsets, index, beta, capacity, beta0,
                           eps, inv_scale, kept);
    return hipGetLastError();
}

hipError_t launch_scan_rows(int64_t *a, int64_t n, int64_t *block_sums, hipStream_t s)
{
    const int64_t nb = (n + 255) / 256;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(256), 0, s, a, n, block_sums);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_block_sums, dim3((unsigned)nb), dim3(256), 0, s, a, n, block_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, block_sums, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, s, a, n, block_sums);
    return hipGetLastError();
}

hipError_t launch_intra_cost(int64_t rows, int L, const int64_t *offsets, const int32_t *index, const float *beta,
                             const int32_t *labelling, const uint8_t *fixed, float *out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    const int nb = (L + 63) / 64;
    const int64_t blocks = (rows + 3) / 4;      // one wave per row
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_intra_cost, dim3((unsigned)blocks), dim3(256), 0, s, rows, L, nb, offsets, index, beta,
                       labelling, fixed, out);
    return hipGetLastError();
}

hipError_t launch_paint_depth(const PaintViews &pv, int n_views, int max_pixels, const int32_t *labels, int L,
                              const float *level_depth, float *out, hipStream_t s)
{
    if (n_views <= 0 || max_pixels <= 0) return hipSuccess;
    const unsigned bx = (unsigned)std::min<int64_t>(((int64_t)max_pixels + 255) / 256, 4096);
    hipLaunchKernelGGL(k_paint_depth, dim3(bx, (unsigned)n_views), dim3(256), 0, s, pv, labels, L, level_depth, out);
    return hipGetLastError();
}

}  // namespace ivde
