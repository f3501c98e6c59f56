// Launch-shape autotuner: times every (labels per lane, waves per group,
// pixels per step) shape of the sweep on a given problem and returns the
// fastest.  Labels per lane and waves per group change how labels map to
// lanes and waves to workgroups, never a result; the pixel-pair sweep adds a
// segment's pixels in another order (bitwise equal results only where the
// sums are integers).
#include <hip/hip_runtime.h>

#include <cfloat>

#include "../../include/ivde.h"
#include "host_common.h"
#include "ivde_internal.h"

using namespace ivde;

namespace {

struct Shape {
    int J, wpg, px;
};

constexpr Shape kShapes[] = {{1, 1, 1}, {1, 2, 1}, {1, 4, 1}, {2, 1, 1}, {2, 2, 1}, {2, 4, 1},
                             {4, 1, 1}, {4, 2, 1}, {4, 4, 1}, {8, 1, 1}, {8, 2, 1}, {8, 4, 1},
                             {1, 1, 2}, {1, 2, 2}, {1, 4, 2}, {1, 1, 4}, {1, 2, 4}, {1, 4, 4}};

}  // namespace

extern "C" ivde_status ivde_autotune(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                                     const ivde_segmentation *segs, const ivde_label_range *labels,
                                     const ivde_options *opt, void *workspace, size_t workspace_bytes,
                                     void *cost_out, ivde_stream stream, int32_t reps, ivde_options *opt_out,
                                     float *times_us, int32_t max_times)
{
    ivde_status st = validate_problem(n_views, cams, views, segs, labels, opt, true);
    if (st != IVDE_OK) return st;
    if (!opt_out || reps < 1 || !cost_out) {
        set_error("autotune: need opt_out, cost_out and reps >= 1");
        return IVDE_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t ev[2];
    hipError_t e = hipEventCreate(&ev[0]);
    if (e != hipSuccess) return hip_fail(e, "event create");
    if ((e = hipEventCreate(&ev[1])) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return hip_fail(e, "event create");
    }
    float best = FLT_MAX;
    ivde_options chosen = *opt;
    int i = 0;
    for (const Shape &sh : kShapes) {
        ivde_options o = *opt;
        o.labels_per_lane = sh.J;
        o.waves_per_group = sh.wpg;
        o.pixels_per_step = sh.px;
        o.sweep_events[0] = ev[0];
        o.sweep_events[1] = ev[1];
        const Layout ly = plan_layout(n_views, cams, segs, labels, &o, views[0].bit_depth);
        float us = -1.f;
        // a shape whose work list does not fit the given workspace is skipped,
        // and so is a pixel-pair shape where that sweep does not exist
        if (ly.workspace_bytes <= workspace_bytes && 64 * sh.J <= 2 * ((labels->num_labels + 63) / 64) * 64 &&
            ly.px == sh.px) {
            st = ivde_cost_volume(n_views, cams, views, segs, labels, &o, workspace, workspace_bytes, cost_out,
                                  stream);   // warm-up
            float total = 0.f;
            for (int r = 0; st == IVDE_OK && r < reps; ++r) {
                st = ivde_cost_volume(n_views, cams, views, segs, labels, &o, workspace, workspace_bytes, cost_out,
                                      stream);
                if (st != IVDE_OK) break;
                if ((e = hipEventSynchronize(ev[1])) != hipSuccess) {
                    st = hip_fail(e, "event synchronize");
                    break;
                }
                float ms = 0.f;
                if ((e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess) {
                    st = hip_fail(e, "event elapsed");
                    break;
                }
                total += ms;
            }
            if (st != IVDE_OK) break;
            us = 1e3f * total / reps;
            if (us < best) {
                best = us;
                chosen = *opt;
                chosen.labels_per_lane = sh.J;
                chosen.waves_per_group = sh.wpg;
                chosen.pixels_per_step = sh.px;
            }
        }
        if (times_us && i < max_times) times_us[i] = us;
        ++i;
    }
    if (st == IVDE_OK && (e = hipStreamSynchronize(s)) != hipSuccess) st = hip_fail(e, "stream synchronize");
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (st != IVDE_OK) return st;
    if (best == FLT_MAX) {
        set_error("autotune: no launch shape fits the workspace");
        return IVDE_ENOMEM;
    }
    chosen.sweep_events[0] = chosen.sweep_events[1] = nullptr;
    *opt_out = chosen;
    return IVDE_OK;
}
