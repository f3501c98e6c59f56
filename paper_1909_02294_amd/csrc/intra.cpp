// The intra-view term of Sec. III-D: segment adjacency with the adaptive
// smoothing weights of Eq. (3), and the Eq. (2) costs that held neighbours
// impose on each segment at each label.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/ivde.h"
#include "host_common.h"
#include "ivde_internal.h"

using namespace ivde;

namespace {

// The segment index and statistics need no sweep: nearest sampling, one
// label, own-camera reference.
ivde_options index_options()
{
    ivde_options o{};
    o.sampling = IVDE_NEAREST;
    o.cost_dtype = IVDE_F32;
    o.targets = IVDE_TARGETS_ALL;
    o.labels_per_lane = 1;
    o.waves_per_group = 4;
    return o;
}

const ivde_label_range kIndexLabels{1.0, 2.0, 1, IVDE_REF_RIG_CENTER};

// The index workspace, the block sums of the offsets scan, then the first
// kAdjKeep neighbour ids of every row.
size_t adjacency_sums_bytes(const Layout &ly)
{
    return align_up(sizeof(int64_t) * (size_t)((ly.total_rows + 255) / 256 + 1), 256);
}

size_t adjacency_workspace(const Layout &ly)
{
    return align_up(ly.workspace_bytes, 256) + adjacency_sums_bytes(ly) +
           align_up(sizeof(int32_t) * kAdjKeep * (size_t)ly.total_rows, 256);
}

}  // namespace

extern "C" {

ivde_status ivde_adjacency_size(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                                int32_t bit_depth, size_t *workspace_bytes)
{
    const ivde_options o = index_options();
    ivde_status st = validate_problem(n_views, cams, nullptr, segs, &kIndexLabels, &o, false);
    if (st != IVDE_OK) return st;
    if (bit_depth < 8 || bit_depth > 16) {
        set_error("bit_depth must be 8..16");
        return IVDE_EINVAL;
    }
    const Layout ly = plan_layout(n_views, cams, segs, &kIndexLabels, &o, bit_depth);
    if (workspace_bytes) *workspace_bytes = adjacency_workspace(ly);
    return IVDE_OK;
}

ivde_status ivde_adjacency(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                           const ivde_segmentation *segs, float beta0, float eps, void *workspace,
                           size_t workspace_bytes, int64_t *offsets, int32_t *index, float *beta, int64_t capacity,
                           ivde_stream stream)
{
    const ivde_options o = index_options();
    ivde_status st = validate_problem(n_views, cams, views, segs, &kIndexLabels, &o, true);
    if (st != IVDE_OK) return st;
    if (!offsets || capacity < 0 || (capacity > 0 && (!index || !beta))) {
        set_error("adjacency: offsets is required, and index and beta when capacity > 0");
        return IVDE_EINVAL;
    }
    if (!(std::isfinite(beta0) && beta0 > 0.f && std::isfinite(eps) && eps > 0.f)) {
        set_error("adjacency: beta0 and eps must be finite and positive");
        return IVDE_EINVAL;
    }
    const Layout ly = plan_layout(n_views, cams, segs, &kIndexLabels, &o, views[0].bit_depth);
    if (ly.total_rows >= ((int64_t)1 << 31)) {
        set_error("adjacency: too many segments");
        return IVDE_EINVAL;
    }
    if ((st = check_workspace(workspace, workspace_bytes, adjacency_workspace(ly))) != IVDE_OK) return st;
    if ((st = check_tex_limits(ly)) != IVDE_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    int64_t *block_sums = reinterpret_cast<int64_t *>(ws + align_up(ly.workspace_bytes, 256));
    int32_t *kept = reinterpret_cast<int32_t *>(ws + align_up(ly.workspace_bytes, 256) + adjacency_sums_bytes(ly));
    Task *tasks = reinterpret_cast<Task *>(ws + ly.off_tasks);
    // the pixel records only: no texels, no work list
    st = enqueue_front(n_views, cams, views, segs, &kIndexLabels, &o, ly, ws, nullptr, 0, tasks, s, false, false, false);
    if (st != IVDE_OK) return st;
    const Problem *dp = reinterpret_cast<const Problem *>(ws + ly.off_problem);
    const Extents ext = extents_of(ly);
    const float inv_scale = 1.0f / (float)(1 << (views[0].bit_depth - 8));
    hipError_t e = launch_segment_stats(dp, ext, nullptr, s);
    if (e == hipSuccess) e = launch_adjacency(dp, ext, 0, offsets, nullptr, nullptr, 0, beta0, eps, inv_scale, kept, s);
    if (e == hipSuccess) e = launch_scan_rows(offsets, ly.total_rows, block_sums, s);
    if (e == hipSuccess && capacity > 0)
        e = launch_adjacency(dp, ext, 1, offsets, index, beta, capacity, beta0, eps, inv_scale, kept, s);
    if (e != hipSuccess) return hip_fail(e, "adjacency");
    return IVDE_OK;
}

ivde_status ivde_intra_cost(int64_t rows, int32_t num_labels, const int64_t *offsets, const int32_t *index,
                            const float *beta, const int32_t *labelling, const uint8_t *fixed, float *out,
                            ivde_stream stream)
{
    if (rows < 0 || num_labels < 1 || (rows > 0 && (!offsets || !index || !beta || !labelling || !out))) {
        set_error("intra_cost: rows >= 0, num_labels >= 1 and non-null offsets, index, beta, labelling, out");
        return IVDE_EINVAL;
    }
    hipError_t e = launch_intra_cost(rows, num_labels, offsets, index, beta, labelling, fixed, out,
                                     static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "intra cost");
    return IVDE_OK;
}

}  // extern "C"
