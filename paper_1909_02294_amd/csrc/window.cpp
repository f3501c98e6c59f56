// The paper's own data term (Sec. III-C, Eqs. (4) and (5)): the window
// matching core at each segment centre towards the neighbouring views, and
// the inter-view cost under a labelling.
#include <hip/hip_runtime.h>

#include "../../include/ivde.h"
#include "host_common.h"
#include "ivde_internal.h"

using namespace ivde;

namespace {

ivde_options window_options()
{
    ivde_options o{};
    o.sampling = IVDE_NEAREST;
    o.cost_dtype = IVDE_F32;
    o.targets = IVDE_TARGETS_NEAREST_LR;
    o.labels_per_lane = 1;     // one 64-label block per wave
    o.waves_per_group = 4;
    return o;
}

}  // namespace

extern "C" {

ivde_status ivde_window_cost_size(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                                  const ivde_label_range *labels, int32_t bit_depth, size_t *out_bytes,
                                  size_t *workspace_bytes)
{
    const ivde_options o = window_options();
    ivde_status st = validate_problem(n_views, cams, nullptr, segs, labels, &o, false);
    if (st != IVDE_OK) return st;
    if (bit_depth < 8 || bit_depth > 16) {
        set_error("bit_depth must be 8..16");
        return IVDE_EINVAL;
    }
    const Layout ly = plan_layout(n_views, cams, segs, labels, &o, bit_depth);
    if (out_bytes) *out_bytes = (size_t)ly.total_rows * 2 * ly.L * 4;
    if (workspace_bytes) *workspace_bytes = ly.workspace_bytes;
    return IVDE_OK;
}

ivde_status ivde_window_cost(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                             const ivde_segmentation *segs, const ivde_label_range *labels, int32_t radius,
                             void *workspace, size_t workspace_bytes, float *m_out, int32_t *hit_out,
                             ivde_stream stream)
{
    const ivde_options o = window_options();
    ivde_status st = validate_problem(n_views, cams, views, segs, labels, &o, true);
    if (st != IVDE_OK) return st;
    if (radius < 0 || radius > 8 || !m_out || !hit_out) {
        set_error("window_cost: radius must be 0..8 and both outputs given");
        return IVDE_EINVAL;
    }
    const Layout ly = plan_layout(n_views, cams, segs, labels, &o, views[0].bit_depth);
    if (ly.total_rows >= ((int64_t)1 << 31)) {
        set_error("window_cost: too many segments");
        return IVDE_EINVAL;
    }
    if ((st = check_workspace(workspace, workspace_bytes, ly.workspace_bytes)) != IVDE_OK) return st;
    if ((st = check_tex_limits(ly)) != IVDE_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    Task *tasks = reinterpret_cast<Task *>(ws + ly.off_tasks);
    st = enqueue_stats(n_views, cams, views, segs, labels, &o, ly, ws, tasks, nullptr, s);
    if (st != IVDE_OK) return st;
    const Problem *dp = reinterpret_cast<const Problem *>(ws + ly.off_problem);
    hipError_t e = launch_window(dp, tasks, ly.n_tasks, radius, ly.tex_u16, m_out, hit_out, s);
    if (e != hipSuccess) return hip_fail(e, "window matching");
    return IVDE_OK;
}

ivde_status ivde_window_energy(int64_t rows, int32_t num_labels, const float *m, const int32_t *hit,
                               const int32_t *labelling, float K, float *out, ivde_stream stream)
{
    if (rows < 0 || num_labels < 1 || (rows > 0 && (!m || !hit || !labelling || !out))) {
        set_error("window_energy: rows >= 0, num_labels >= 1 and non-null buffers are required");
        return IVDE_EINVAL;
    }
    hipError_t e = launch_window_energy(rows, num_labels, m, hit, labelling, K, out, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "window energy");
    return IVDE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- segment statistics and the temporal rule
extern "C" {

ivde_status ivde_segment_stats_size(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                                    int32_t bit_depth, size_t *workspace_bytes)
{
    ivde_label_range lr{1.0, 2.0, 1, IVDE_REF_RIG_CENTER};
    const ivde_options o = window_options();
    ivde_status st = validate_problem(n_views, cams, nullptr, segs, &lr, &o, false);
    if (st != IVDE_OK) return st;
    if (bit_depth < 8 || bit_depth > 16) {
        set_error("bit_depth must be 8..16");
        return IVDE_EINVAL;
    }
    const Layout ly = plan_layout(n_views, cams, segs, &lr, &o, bit_depth);
    if (workspace_bytes) *workspace_bytes = ly.workspace_bytes;
    return IVDE_OK;
}

ivde_status ivde_segment_stats(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                               const ivde_segmentation *segs, void *workspace, size_t workspace_bytes,
                               int32_t *count_out, int32_t *centre_out, float *mean_out, ivde_stream stream)
{
    ivde_label_range lr{1.0, 2.0, 1, IVDE_REF_RIG_CENTER};
    const ivde_options o = window_options();
    ivde_status st = validate_problem(n_views, cams, views, segs, &lr, &o, true);
    if (st != IVDE_OK) return st;
    const Layout ly = plan_layout(n_views, cams, segs, &lr, &o, views[0].bit_depth);
    if ((st = check_workspace(workspace, workspace_bytes, ly.workspace_bytes)) != IVDE_OK) return st;
    if ((st = check_tex_limits(ly)) != IVDE_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *ws = static_cast<char *>(workspace);
    st = enqueue_stats(n_views, cams, views, segs, &lr, &o, ly, ws, nullptr, count_out, s, false);
    if (st != IVDE_OK) return st;
    hipError_t e;
    if (centre_out &&
        (e = launch_copy_rows(ws + ly.off_centre, centre_out, (int64_t)ly.total_rows * 8, s)) != hipSuccess)
        return hip_fail(e, "centre copy");
    if (mean_out && (e = launch_copy_rows(ws + ly.off_mean, mean_out, (int64_t)ly.total_rows * 16, s)) != hipSuccess)
        return hip_fail(e, "mean copy");
    return IVDE_OK;
}

ivde_status ivde_temporal_rule(int64_t rows, const float *mean, const float *mean_prev, const float *mean_iframe,
                               float t_p, float t_i, int32_t bit_depth, uint8_t *source_out, ivde_stream stream)
{
    if (rows < 0 || (rows > 0 && (!mean || !mean_prev || !source_out)) || bit_depth < 8 || bit_depth > 16) {
        set_error("temporal_rule: rows >= 0, mean, mean_prev, source_out and a bit depth 8..16 are required");
        return IVDE_EINVAL;
    }
    const float scale = (float)(1 << (bit_depth - 8));
    hipError_t e = launch_temporal_rule(rows, mean, mean_prev, mean_iframe, t_p * scale, t_i * scale, source_out,
                                        nullptr, nullptr, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "temporal rule");
    return IVDE_OK;
}

}  // extern "C"
