// Internal types shared by the host code and the gfx950 kernels of libivde.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ivde {

constexpr int kMaxViews = 32;          // views per problem (pair table is n x n)
constexpr int kBand = 32;              // rows per spatial band of the work list
constexpr int kXcds = 8;               // XCDs of the MI355X; consecutive blocks go to consecutive XCDs
constexpr int kFlagWords = 8;          // workspace flag area: error flag, padding, 3 x 64-bit step counts
constexpr float kEdge = 1.0f / 64.0f;  // bilinear margin outside the outer pixel centres

// Per-view device descriptor.  Everything a kernel needs about one view:
// the caller's planes, the packed texels, the segment index and the
// per-view constant of the reference plane.
struct ViewDesc {
    const void *plane[3];      // caller's Y, Cb, Cr planes (uint8 or uint16)
    int64_t pitch[3];          // their row pitches in samples
    const int32_t *seg;        // caller's segment map
    int64_t seg_pitch;
    void *tex;                 // packed texels, (W + 2) x (H + 2), edge-replicating border
    int64_t tex_bytes;
    int32_t W, H;
    int32_t tex_pitch;         // texels per row = W + 2
    int32_t S;                 // segments
    int64_t row0;              // first cost-volume row of this view
    int32_t *counts;           // [S] pixels per segment
    int32_t *offsets;          // [S + 1] exclusive scan of counts
    int32_t *bbox;             // [4 S] x0, y0, x1, y1 (inclusive)
    float *pixrec;             // [W H][8] x, y, g.p, Y, Cb, Cr, 0, 0 in segment order
    int32_t *band_count;       // [n_bands] segments per band, then band cursors
    int32_t *centre;           // [2 S] segment centre (centroid rounded half up), -1 if empty
    float *mean;               // [4 S] mean Y, Cb, Cr of the segment, 0
    int32_t n_bands;
    int32_t front_all;         // every pixel at every label lies in front of this camera
    uint32_t front_targets;    // bit c2: with front_all, every such point also lies in front of view c2
    int32_t n_targets;
    int32_t targets[kMaxViews];
    float g[4];                // g_c = K_c^-T R_c n_r (g . p~ = n_r . ray direction)
};

// Projection of view c into target c2 (FP64 on the host, cast to FP32):
// h = H p~ + sigma_{c,l} (g_c . p~) e,  u = h_x / h_z,  v = h_y / h_z, in the
// target's bordered texel coordinates (pixel coordinates plus one).
struct PairConst {
    float H[9];
    float e[3];
};

// One cost-volume problem in device memory.
struct Problem {
    int32_t n_views;
    int32_t L;                 // labels
    int32_t J;                 // labels per lane
    int32_t n_lblocks;         // ceil(L / (64 J))
    int32_t bilinear;
    int32_t f16out;
    int32_t bit_depth;
    int32_t chroma_shift;
    float norm;                // 3 (2^b - 1)
    int32_t tex_u16;           // texel channels are 16-bit code values (bit depth > 11) instead of halves
    int64_t total_rows;
    ViewDesc *views;           // [n_views]
    PairConst *pairs;          // [n_views * n_views], [c * n + c2]
    float *sigma;              // [n_views * L], 1 / (z_l - delta_c) or 0 when undefined
    void *cost;                // [total_rows * L] float or half
    int32_t *flag;             // device error flag (segment id out of range)
    // wave steps of the pixel-pair sweep: [0] all, [1] on projected records,
    // [2] on chunks whose every sample lies inside the validity band
    unsigned long long *steps;
};

// A unit of sweep work: one wave computes labels [64 J b, 64 J (b + 1)) of
// one cost-volume row.
struct Task {
    int32_t problem;           // index into the problem table
    int32_t view;
    int32_t seg;
    int32_t lblock;
};

// ---------------------------------------------------------------- launchers
// All return hipSuccess or the launch error.
hipError_t launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s);
// Sizes of the largest view of a problem, for grid shapes.
struct Extents {
    int n_views;
    int max_w, max_h, max_s, max_bands;
};
// segment index (counts, offsets, boxes, pixel records) and, with pack, the texels
hipError_t launch_prepare(const Problem *dprob, const Extents &ext, int tex_u16, hipStream_t s, bool pack = true);
// the bordered texel image of every view
hipError_t launch_pack(const Problem *dprob, const Extents &ext, int tex_u16, hipStream_t s);
// a new frame over an index already built for the same segmentation:
// repack the texels and refresh the records' colours
hipError_t launch_refresh(const Problem *dprob, const Extents &ext, int tex_u16, hipStream_t s);
hipError_t launch_worklist(const Problem *dprob, const Extents &ext, int problem_index, Task *tasks,
                           hipStream_t s);
// The sweep over tasks[0, n_tasks): enough resident groups to fill every CU
// take tasks from per-XCD cursors.  counters: kXcds + 1 device ints of
// scratch (the cursors, then the task count), set by this call.
// px: pixels per wave step (2: the pixel-pair sweep, which exists for one
// label per lane and half texels; 1: the one-pixel sweep).
hipError_t launch_sweep(const Problem *dprobs, const Task *tasks, int64_t n_tasks, int J, int px,
                        int bilinear, int tex_u16, int f16out, int waves_per_group, int32_t *counters,
                        hipStream_t s);
// cursors: kXcds zeroed counters, one per contiguous range of the task list
hipError_t launch_sweep_persistent(const Problem *dprobs, const Task *tasks, const int32_t *n_tasks_dev,
                                   int32_t *cursors, int64_t max_tasks, int J, int px, int bilinear, int tex_u16,
                                   int f16out, int waves_per_group, int n_groups, hipStream_t s);
// Resident groups per CU of the persistent sweep for this launch shape.
hipError_t sweep_persistent_occupancy(int J, int px, int bilinear, int tex_u16, int f16out, int waves_per_group,
                                      int *groups_per_cu);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_argmin(const void *cost, int f16, int64_t rows, int L, int32_t *out, hipStream_t s);
hipError_t launch_compact_tasks(const Problem *dprob, const Task *all, int64_t n_all, const uint8_t *mask,
                                Task *out, int32_t *n_out, hipStream_t s);
hipError_t launch_copy_rows(const void *src, void *dst, int64_t bytes, hipStream_t s);
// Per-segment count, centre and mean colour (needs the segment index);
// count_flat [rows] may be null.
hipError_t launch_segment_stats(const Problem *dprob, const Extents &ext, int32_t *count_flat, hipStream_t s);
// segment statistics from the segment map alone (no segment index): clears
// and fills sums [rows][6], then counts, centres and means; with tasks, also
// the work list in row order
hipError_t launch_segment_sums(const Problem *dprob, const Extents &ext, unsigned long long *sums, int64_t rows,
                               int32_t *count_flat, Task *tasks, hipStream_t s);
hipError_t launch_temporal_rule(int64_t rows, const float *mean, const float *prev, const float *iframe, float t_p,
                                float t_i, uint8_t *source, uint8_t *changed, int32_t *counts, hipStream_t s);
hipError_t launch_copy_rows_where(int64_t rows, int row_bytes, const uint8_t *source, int which, const void *from,
                                  void *to, hipStream_t s);
// Window matching core towards views c - 1 and c + 1 for every task.
// kept: [rows][kAdjKeep] neighbour ids written by the count pass and copied
// by the fill pass for rows with at most kAdjKeep neighbours
constexpr int kAdjKeep = 32;
hipError_t launch_adjacency(const Problem *dprob, const Extents &ext, int write, int64_t *offsets, int32_t *index,
                            float *beta, int64_t capacity, float beta0, float eps, float inv_scale, int32_t *kept,
                            hipStream_t s);
// In-place inclusive scan of a[1..n] with a[0] = 0; block_sums holds
// ceil(n / 256) (at least 1) int64 of scratch.
hipError_t launch_scan_rows(int64_t *a, int64_t n, int64_t *block_sums, hipStream_t s);
hipError_t launch_intra_cost(int64_t rows, int L, const int64_t *offsets, const int32_t *index, const float *beta,
                             const int32_t *labelling, const uint8_t *fixed, float *out, hipStream_t s);
// Views of a depth painting: caller's segment maps and output offsets.
struct PaintViews {
    const int32_t *seg[kMaxViews];
    int64_t pitch[kMaxViews];
    int64_t row0[kMaxViews];
    int64_t out0[kMaxViews];
    int32_t W[kMaxViews], H[kMaxViews], S[kMaxViews];
};
hipError_t launch_paint_depth(const PaintViews &pv, int n_views, int max_pixels, const int32_t *labels, int L,
                              const float *level_depth, float *out, hipStream_t s);
hipError_t launch_window(const Problem *dprob, const Task *tasks, int64_t n_tasks, int radius, int tex_u16,
                         float *m_out, int32_t *hit_out, hipStream_t s);
hipError_t launch_window_energy(int64_t rows, int L, const float *m, const int32_t *hit, const int32_t *labelling,
                                float K, float *out, hipStream_t s);

}  // namespace ivde
