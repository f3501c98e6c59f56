// Depth maps from segment labels (Sec. III-B: a segment's depth is painted
// onto its pixels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/ivde.h"
#include "host_common.h"
#include "ivde_internal.h"

using namespace ivde;

extern "C" {

ivde_status ivde_depth_map(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                           const ivde_label_range *labels, const int32_t *label_of_row, void *workspace,
                           size_t workspace_bytes, float *depth_out, ivde_stream stream)
{
    if (n_views < 1 || n_views > kMaxViews || !cams || !segs || !labels || !label_of_row || !depth_out) {
        set_error("depth_map: 1..%d views, cameras, segmentations, a label range, labels and an output", kMaxViews);
        return IVDE_EINVAL;
    }
    if (!(labels->z_near > 0 && labels->z_far > 0 && std::isfinite(labels->z_near) && std::isfinite(labels->z_far) &&
          labels->z_near != labels->z_far) ||
        labels->num_labels < 1 || labels->num_labels > 8192) {
        set_error("depth_map: positive, distinct, finite z_near and z_far and num_labels in [1, 8192] are required");
        return IVDE_EINVAL;
    }
    const int L = labels->num_labels;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 4) {
        set_error("depth_map: a 4-byte aligned workspace is required");
        return IVDE_EINVAL;
    }
    if (workspace_bytes < sizeof(float) * (size_t)L) {
        set_error("depth_map: workspace too small: %zu bytes given, %zu needed", workspace_bytes,
                  sizeof(float) * (size_t)L);
        return IVDE_ENOMEM;
    }
    PaintViews pv{};
    int64_t row0 = 0, out0 = 0;
    int max_px = 0;
    for (int v = 0; v < n_views; ++v) {
        const ivde_camera &c = cams[v];
        const ivde_segmentation &g = segs[v];
        if (c.width < 1 || c.height < 1 || !g.seg_map || g.num_segments < 1 || g.pitch < c.width ||
            (int64_t)c.width * c.height >= ((int64_t)1 << 31)) {
            set_error("depth_map: view %d needs a size, a map with pitch >= width and num_segments >= 1", v);
            return IVDE_EINVAL;
        }
        pv.seg[v] = g.seg_map;
        pv.pitch[v] = g.pitch;
        pv.row0[v] = row0;
        pv.out0[v] = out0;
        pv.W[v] = c.width;
        pv.H[v] = c.height;
        pv.S[v] = g.num_segments;
        row0 += g.num_segments;
        out0 += (int64_t)c.width * c.height;
        max_px = std::max(max_px, c.width * c.height);
    }
    // level depths in FP64, one rounding per operation (separate statements,
    // so no multiply-add is contracted), stored as FP32
    std::vector<float> depth(L);
    const double inv_far = 1.0 / labels->z_far;
    const double span = 1.0 / labels->z_near - inv_far;
    for (int l = 0; l < L; ++l) {
        const double frac = L > 1 ? (double)l / (double)(L - 1) : 0.0;
        const double step = frac * span;
        const double rho = inv_far + step;
        depth[l] = (float)(1.0 / rho);
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    float *table = static_cast<float *>(workspace);
    hipError_t e = launch_upload(table, depth.data(), sizeof(float) * (size_t)L, s);
    if (e != hipSuccess) return hip_fail(e, "level-depth upload");
    e = launch_paint_depth(pv, n_views, max_px, label_of_row, L, table, depth_out, s);
    if (e != hipSuccess) return hip_fail(e, "depth map");
    return IVDE_OK;
}

}  // extern "C"
