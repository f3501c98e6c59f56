// Batched form: many frames with uneven view, segment and label counts in
// one persistent sweep launch, optionally replayed from a hipGraph.
//
// Every frame keeps its own region of the batch workspace (packed images,
// segment index, constants); their task lists are laid out back to back so
// that the concatenation is one queue.  Frames are ordered by decreasing
// work so the queue drains large tasks first.  The sweep kernel runs the
// same per-task code as ivde_cost_volume, so each frame's cost volume is
// bitwise equal to what ivde_cost_volume returns for it.  Frames whose
// levels lie far apart take the pixel-pair sweep (as ivde_cost_volume would
// choose for them): their tasks form the back of the queue, drained by a
// second persistent launch right after the first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/ivde.h"
#include "host_common.h"
#include "ivde_internal.h"

using namespace ivde;

// Sweep forms a batch can hold, by pixels per wave step, in queue order.
constexpr int kBatchForms = 3;
constexpr int kBatchFormPx[kBatchForms] = {1, 2, 4};
inline int form_index(int px) { return px == 1 ? 0 : px == 2 ? 1 : 2; }

struct ivde_batch {
    int n_frames = 0;
    std::vector<ivde_frame> frames;
    std::vector<std::vector<ivde_camera>> cams;
    std::vector<std::vector<ivde_image>> views;
    std::vector<std::vector<ivde_segmentation>> segs;
    std::vector<Layout> layouts;
    std::vector<size_t> frame_off;     // byte offset of each frame's region
    std::vector<int64_t> task_off;     // first task of each frame in the queue
    std::vector<int> order;            // frames by sweep form (1, 2, then 4 pixels per step), each by decreasing work
    ivde_options opt{};
    char *ws = nullptr;
    size_t off_probs = 0, off_tasks = 0, off_counters = 0, total_bytes = 0;
    int64_t n_tasks = 0;
    int64_t form_end[kBatchForms] = {0, 0, 0};   // end of each sweep form's range of the queue
    int J = 4, wpg = 4, tex_u16 = 0, f16 = 0, bilinear = 1;
    int n_groups[kBatchForms] = {0, 0, 0};       // resident groups of each form's persistent sweep
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

ivde_status plan_batch(int32_t n_frames, const ivde_frame *frames, const ivde_options *opt, ivde_batch &b)
{
    if (n_frames < 1 || !frames || !opt) {
        set_error("batch: need at least one frame and options");
        return IVDE_EINVAL;
    }
    if (opt->targets == IVDE_TARGETS_EXPLICIT) {
        set_error("batch: explicit target masks are per call; use IVDE_TARGETS_ALL or IVDE_TARGETS_NEAREST_LR");
        return IVDE_EINVAL;
    }
    b.n_frames = n_frames;
    b.opt = *opt;
    b.frames.assign(frames, frames + n_frames);
    int bit_depth = -1, chroma = -1;
    for (int f = 0; f < n_frames; ++f) {
        const ivde_frame &fr = frames[f];
        ivde_status st = validate_problem(fr.n_views, fr.cams, fr.views, fr.segs, &fr.labels, opt, true);
        if (st != IVDE_OK) {
            set_error("batch frame %d: %s", f, last_error());
            return st;
        }
        if (!fr.cost_out) {
            set_error("batch frame %d: null cost_out", f);
            return IVDE_EINVAL;
        }
        if (bit_depth < 0) {
            bit_depth = fr.views[0].bit_depth;
            chroma = fr.views[0].chroma_shift;
        } else if (fr.views[0].bit_depth != bit_depth || fr.views[0].chroma_shift != chroma) {
            set_error("batch frame %d: all frames must share bit depth and chroma format", f);
            return IVDE_EINVAL;
        }
    }
    // one launch shape for the whole batch: the largest label block any frame needs
    int maxL = 0;
    for (int f = 0; f < n_frames; ++f) maxL = std::max(maxL, frames[f].labels.num_labels);
    ivde_options o = *opt;
    if (!o.labels_per_lane) o.labels_per_lane = default_labels_per_lane(maxL);
    if (!o.waves_per_group) o.waves_per_group = 4;
    b.opt = o;
    b.J = o.labels_per_lane;
    b.wpg = o.waves_per_group;
    b.tex_u16 = bit_depth > 11;
    b.f16 = o.cost_dtype == IVDE_F16;
    b.bilinear = o.sampling == IVDE_BILINEAR;

    size_t off = 0;
    b.layouts.resize(n_frames);
    b.frame_off.resize(n_frames);
    b.task_off.resize(n_frames);
    std::vector<double> work(n_frames);
    for (int f = 0; f < n_frames; ++f) {
        const ivde_frame &fr = frames[f];
        b.layouts[f] = plan_layout(fr.n_views, fr.cams, fr.segs, &fr.labels, &o, bit_depth);
        ivde_status st = check_tex_limits(b.layouts[f]);
        if (st != IVDE_OK) return st;
        b.frame_off[f] = off;
        off = align_up(off + b.layouts[f].workspace_bytes, 256);
        double w = 0;
        for (int v = 0; v < fr.n_views; ++v) w += (double)fr.cams[v].width * fr.cams[v].height;
        work[f] = w * fr.labels.num_labels * (fr.n_views - 1);
    }
    b.order.resize(n_frames);
    std::iota(b.order.begin(), b.order.end(), 0);
    std::stable_sort(b.order.begin(), b.order.end(), [&](int a, int c) {
        const int pa = b.layouts[a].px, pc = b.layouts[c].px;
        return pa != pc ? pa < pc : work[a] > work[c];
    });
    int64_t t = 0;
    for (int f : b.order) {
        b.task_off[f] = t;
        t += b.layouts[f].n_tasks;
        for (int k = form_index(b.layouts[f].px); k < kBatchForms; ++k) b.form_end[k] = t;
    }
    b.n_tasks = t;
    b.off_probs = off;
    off = align_up(off + sizeof(Problem) * n_frames, 256);
    b.off_tasks = off;
    off = align_up(off + sizeof(Task) * (size_t)b.n_tasks, 256);
    b.off_counters = off;
    off = align_up(off + kBatchForms * (kXcds + 1) * sizeof(int32_t), 256);   // per sweep: cursors, then the task count
    // keep host copies of the frame descriptions: the plan outlives the caller's arrays
    b.cams.resize(n_frames);
    b.views.resize(n_frames);
    b.segs.resize(n_frames);
    for (int f = 0; f < n_frames; ++f) {
        const ivde_frame &fr = frames[f];
        b.cams[f].assign(fr.cams, fr.cams + fr.n_views);
        b.views[f].assign(fr.views, fr.views + fr.n_views);
        b.segs[f].assign(fr.segs, fr.segs + fr.n_views);
        b.frames[f].cams = b.cams[f].data();
        b.frames[f].views = b.views[f].data();
        b.frames[f].segs = b.segs[f].data();
    }
    if (b.n_tasks > 0x7fffffff) {
        set_error("batch: too many tasks");
        return IVDE_EINVAL;
    }
    b.total_bytes = off;
    return IVDE_OK;
}

ivde_status enqueue_batch(ivde_batch &b, hipStream_t s)
{
    hipError_t e;
    std::vector<Problem> probs(b.n_frames);
    for (int f = 0; f < b.n_frames; ++f) {
        const ivde_frame &fr = b.frames[f];
        const Layout &ly = b.layouts[f];
        char *fws = b.ws + b.frame_off[f];
        HostConstants hc;
        ivde_status st = compose(fr.n_views, fr.cams, fr.views, fr.segs, &fr.labels, &b.opt, ly, fws, fr.cost_out, hc);
        if (st != IVDE_OK) return st;
        probs[f] = hc.problem;
        if ((e = upload_constants(hc, ly, fws, s)) != hipSuccess) return hip_fail(e, "batch constants");
        if ((e = launch_fill_i32(reinterpret_cast<int32_t *>(fws + ly.off_flag), 0, kFlagWords, s)) != hipSuccess)
            return hip_fail(e, "batch flag");
        const Problem *dp = reinterpret_cast<const Problem *>(fws + ly.off_problem);
        if ((e = launch_prepare(dp, extents_of(ly), ly.tex_u16, s)) != hipSuccess) return hip_fail(e, "batch index");
        Task *tasks = reinterpret_cast<Task *>(b.ws + b.off_tasks) + b.task_off[f];
        if ((e = launch_worklist(dp, extents_of(ly), f, tasks, s)) != hipSuccess) return hip_fail(e, "batch tasks");
    }
    if ((e = launch_upload(b.ws + b.off_probs, probs.data(), sizeof(Problem) * probs.size(), s)) != hipSuccess)
        return hip_fail(e, "batch problem table");
    int32_t *counters = reinterpret_cast<int32_t *>(b.ws + b.off_counters);
    for (int k = 0; k < kBatchForms; ++k) {
        const int64_t n = b.form_end[k] - (k ? b.form_end[k - 1] : 0);
        int32_t *ck = counters + k * (kXcds + 1);
        if ((e = launch_fill_i32(ck, 0, kXcds, s)) != hipSuccess ||
            (e = launch_fill_i32(ck + kXcds, (int32_t)n, 1, s)) != hipSuccess)
            return hip_fail(e, "batch cursors");
    }
    // timing events only in eager runs: a captured graph replays without them
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if ((e = hipStreamIsCapturing(s, &cap)) != hipSuccess) return hip_fail(e, "capture status");
    const bool timed = b.opt.sweep_events[0] && b.opt.sweep_events[1] && cap == hipStreamCaptureStatusNone;
    if (timed && (e = hipEventRecord(static_cast<hipEvent_t>(b.opt.sweep_events[0]), s)) != hipSuccess)
        return hip_fail(e, "event record");
    const Problem *dprobs = reinterpret_cast<const Problem *>(b.ws + b.off_probs);
    const Task *tasks = reinterpret_cast<const Task *>(b.ws + b.off_tasks);
    for (int k = 0; k < kBatchForms; ++k) {
        const int64_t t0 = k ? b.form_end[k - 1] : 0, n = b.form_end[k] - t0;
        int32_t *ck = counters + k * (kXcds + 1);
        if (n > 0 && (e = launch_sweep_persistent(dprobs, tasks + t0, ck + kXcds, ck, n, b.J, kBatchFormPx[k],
                                                  b.bilinear, b.tex_u16, b.f16, b.wpg, b.n_groups[k], s)) != hipSuccess)
            return hip_fail(e, "batch sweep");
    }
    if (timed && (e = hipEventRecord(static_cast<hipEvent_t>(b.opt.sweep_events[1]), s)) != hipSuccess)
        return hip_fail(e, "event record");
    for (int f = 0; f < b.n_frames; ++f) {
        const ivde_frame &fr = b.frames[f];
        if (!fr.label_out) continue;
        if ((e = launch_argmin(fr.cost_out, b.f16, b.layouts[f].total_rows, fr.labels.num_labels, fr.label_out, s)) !=
            hipSuccess)
            return hip_fail(e, "batch argmin");
    }
    return IVDE_OK;
}

int persistent_groups(int J, int px, int bilinear, int tex_u16, int f16, int wpg)
{
    // enough resident groups to fill every CU at the kernel's occupancy
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (sweep_persistent_occupancy(J, px, bilinear, tex_u16, f16, wpg, &per_cu) != hipSuccess) return 0;
    return cus * std::max(1, per_cu);
}

}  // namespace

extern "C" {

ivde_status ivde_batch_size(int32_t n_frames, const ivde_frame *frames, const ivde_options *opt,
                            size_t *workspace_bytes)
{
    ivde_batch b;
    ivde_status st = plan_batch(n_frames, frames, opt, b);
    if (st != IVDE_OK) return st;
    if (workspace_bytes) *workspace_bytes = b.total_bytes;
    return IVDE_OK;
}

ivde_status ivde_batch_create(int32_t n_frames, const ivde_frame *frames, const ivde_options *opt, void *workspace,
                              size_t workspace_bytes, ivde_batch **out)
{
    if (!out) {
        set_error("batch: null output handle");
        return IVDE_EINVAL;
    }
    *out = nullptr;
    ivde_batch *b = new (std::nothrow) ivde_batch;
    if (!b) {
        set_error("batch: out of host memory");
        return IVDE_ENOMEM;
    }
    ivde_status st = plan_batch(n_frames, frames, opt, *b);
    if (st == IVDE_OK) st = check_workspace(workspace, workspace_bytes, b->total_bytes);
    if (st != IVDE_OK) {
        delete b;
        return st;
    }
    b->ws = static_cast<char *>(workspace);
    bool ok = true;
    for (int k = 0; k < kBatchForms; ++k) {
        const bool used = b->form_end[k] > (k ? b->form_end[k - 1] : 0);
        b->n_groups[k] = used ? persistent_groups(b->J, kBatchFormPx[k], b->bilinear, b->tex_u16, b->f16, b->wpg) : 1;
        ok &= b->n_groups[k] > 0;
    }
    if (!ok) {
        delete b;
        set_error("batch: occupancy query failed");
        return IVDE_EHIP;
    }
    *out = b;
    return IVDE_OK;
}

ivde_status ivde_batch_run(ivde_batch *b, ivde_stream stream, int32_t use_graph)
{
    if (!b) {
        set_error("batch: null handle");
        return IVDE_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!use_graph) return enqueue_batch(*b, s);
    if (!b->exec) {
        if (!s) {
            set_error("batch: graph capture needs a non-null stream");
            return IVDE_EINVAL;
        }
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return hip_fail(e, "begin capture");
        ivde_status st = enqueue_batch(*b, s);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (st != IVDE_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "graph instantiate");
        }
        b->graph = g;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return IVDE_OK;
}

void ivde_batch_destroy(ivde_batch *b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
}

}  // extern "C"
