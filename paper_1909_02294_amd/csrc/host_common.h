// Host-side helpers shared by the plain, batched and serving entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

#include "../../include/ivde.h"
#include "ivde_internal.h"

namespace ivde {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct ViewLayout {
    int64_t row0;
    int32_t n_bands;
    int64_t tex_bytes;
    size_t off_tex, off_counts, off_offsets, off_bbox, off_pixrec, off_bands;
};

// Byte offsets of everything one problem keeps in its workspace.
struct Layout {
    int n, L, J, wpg, n_lblocks, tex_u16, f16;
    int px;                            // pixels per wave step of the sweep (1 or 2)
    int max_w, max_h, max_s, max_bands;
    int64_t total_rows, n_tasks;
    size_t off_problem, off_views, off_pairs, off_sigma, off_flag, off_tasks;   // off_flag: kFlagWords words
    size_t off_centre, off_mean;       // [rows][2] int32 and [rows][4] float over all views
    size_t off_sums;                   // [rows][6] uint64 pixel sums (statistics without the index)
    size_t off_cursors;                // kXcds + 1 int32: sweep cursors and task count
    size_t workspace_bytes, cost_bytes;
    ViewLayout views[kMaxViews];
};

struct HostConstants {
    Problem problem;
    std::vector<ViewDesc> views;
    std::vector<PairConst> pairs;
    std::vector<float> sigma;
};

void set_error(const char *fmt, ...);
const char *last_error();
ivde_status hip_fail(hipError_t e, const char *what);

ivde_status validate_problem(int32_t n, const ivde_camera *cams, const ivde_image *views,
                             const ivde_segmentation *segs, const ivde_label_range *labels,
                             const ivde_options *opt, bool need_images);
int default_labels_per_lane(int L);
Layout plan_layout(int32_t n, const ivde_camera *cams, const ivde_segmentation *segs, const ivde_label_range *labels,
                   const ivde_options *opt, int bit_depth);
ivde_status compose(int32_t n, const ivde_camera *cams, const ivde_image *views, const ivde_segmentation *segs,
                    const ivde_label_range *labels, const ivde_options *opt, const Layout &ly, char *ws_base,
                    void *cost_out, HostConstants &hc);
hipError_t upload_constants(const HostConstants &hc, const Layout &ly, char *ws_base, hipStream_t s);
Extents extents_of(const Layout &ly);
// Constants, segment statistics from the segment map alone (no segment
// index) and, with texels, the packed texel images; with tasks, the work list
// in row order.
ivde_status enqueue_stats(int32_t n, const ivde_camera *cams, const ivde_image *views,
                          const ivde_segmentation *segs, const ivde_label_range *labels, const ivde_options *opt,
                          const Layout &ly, char *ws, Task *tasks, int32_t *count_flat, hipStream_t s,
                          bool texels = true);
// index_ready: the workspace already holds the segment index and work list
// of this segmentation and layout; only the frame's images are taken in.
// texels / worklist = false skip the packed texels / the work list for
// callers that read only the index.
ivde_status enqueue_front(int32_t n, const ivde_camera *cams, const ivde_image *views,
                          const ivde_segmentation *segs, const ivde_label_range *labels, const ivde_options *opt,
                          const Layout &ly, char *ws, void *cost_out, int problem_index, Task *tasks,
                          hipStream_t s,
                          bool index_ready = false, bool texels = true, bool worklist = true);
ivde_status check_workspace(const void *workspace, size_t have, size_t need);
// The plain cost volume into a validated workspace `ws` laid out as `ly`:
// constants, segment index, work list and the sweep, enqueued on `s`.
ivde_status enqueue_cost_volume(int32_t n, const ivde_camera *cams, const ivde_image *views,
                                const ivde_segmentation *segs, const ivde_label_range *labels,
                                const ivde_options *opt, const Layout &ly, char *ws, void *cost_out, hipStream_t s);
ivde_status check_tex_limits(const Layout &ly);

}  // namespace ivde
