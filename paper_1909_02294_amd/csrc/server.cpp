// Serving runtime: continuous admission of frames from several camera rigs
// under an HBM budget, with each rig's previous cost volume kept resident
// and only the segments the temporal mask marks as changed recomputed (the
// paper's temporal scheme, Sec. III-E, turned into a request loop).
//
// Memory.  The caller hands over one device arena; its size is the budget.
// A rig's registration reserves its resident state (a copy of its segment
// maps and its cost volume).  An admitted request reserves a working set
// (packed images, segment index, task lists) until it completes.  A request
// waits in the queue while no slot or not enough arena is free, and is
// rejected at submission if it could never fit.
//
// Concurrency.  One scheduler thread admits requests in arrival order, gives
// each a slot (its own HIP stream, default priority), enqueues its kernels
// and polls completion events.  Requests of different rigs overlap on the
// device; frames of one rig are ordered by an event dependency on the rig's
// previous frame, because each frame starts from that frame's volume.  Every
// row is computed by the same per-task kernel code as ivde_cost_volume, so a
// frame's result does not depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/ivde.h"
#include "host_common.h"
#include "ivde_internal.h"

using namespace ivde;

namespace {

double now_us()
{
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over the arena, 256-byte granules.
class Arena {
  public:
    void init(size_t bytes) { free_ = {{0, bytes}}; }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(std::max<size_t>(bytes, 1), 256);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (auto &kv : free_) m = std::max(m, kv.second);
        return m;
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Rig {
    int id = -1;
    int n = 0;
    std::vector<ivde_camera> cams;
    std::vector<ivde_segmentation> segs;   // pointing at the arena copies
    ivde_label_range labels{};
    ivde_options opt{};
    Layout ly{};                           // the largest layout (16-bit images): sizes the workspace
    size_t res_off = 0, res_bytes = 0;     // resident: seg maps, workspace, volumes, mean colours
    char *ws = nullptr;                    // the rig's workspace: index, work list, texels, constants
    int index_tex = -1;                    // texel format the index in ws was built for, -1: none
    char *cost = nullptr;                  // resident cost volume (the latest frame)
    char *cost_i = nullptr;                // the latest I frame's volume
    float *mean_prev = nullptr;            // [rows][4] mean colours of the latest frame
    float *mean_i = nullptr;               // [rows][4] mean colours of the latest I frame
    size_t cost_bytes = 0;
    float t_p = 3.f, t_i = 1.f;            // temporal thresholds in 8-bit code values
    bool has_prev = false;                 // resident volume holds a frame
    bool has_i = false;                    // cost_i and mean_i hold an I frame
    hipEvent_t last = nullptr;             // completion of the rig's latest enqueued frame
    bool last_valid = false;
    int pending = 0;                       // requests queued or in flight
};

struct Request {
    uint64_t ticket = 0;
    int rig = -1;
    std::vector<ivde_image> views;
    const uint8_t *mask = nullptr;
    bool rule = false;                     // derive the mask by the temporal rule
    bool iframe = false;                   // rule mode: compute every row and make this the I frame
    void *cost_out = nullptr;
    int32_t *label_out = nullptr;
    ivde_frame_stats st{};
    Layout ly{};                           // depends on the frame's bit depth
    size_t work_bytes = 0;
    int slot = -1;
    size_t work_off = 0;
    bool done = false;
};

// A rig's resident state: its segment maps, its workspace (frames of one
// rig run one after another, so they share it and the segment index built
// by the first), the latest and the I-frame cost volumes, and two
// mean-colour tables.  ly is the largest layout (16-bit images).
size_t resident_bytes(int n_views, const ivde_camera *cams, const Layout &ly, size_t *seg_off, size_t *seg_total)
{
    size_t seg_bytes = 0;
    for (int v = 0; v < n_views; ++v) {
        if (seg_off) seg_off[v] = seg_bytes;
        seg_bytes = align_up(seg_bytes + sizeof(int32_t) * (size_t)cams[v].width * cams[v].height, 256);
    }
    if (seg_total) *seg_total = seg_bytes;
    return seg_bytes + align_up(ly.workspace_bytes, 256) + 2 * align_up(ly.cost_bytes, 256) +
           2 * align_up((size_t)ly.total_rows * 16, 256);
}

// One admitted frame's own memory: counters, the compacted task list, and
// the rule's per-row source and changed flags.
size_t working_set(const Layout &ly)
{
    return 256 + align_up(sizeof(Task) * (size_t)ly.n_tasks, 256) + 2 * align_up((size_t)ly.total_rows, 256);
}

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int32_t *count_host = nullptr;         // pinned [8]: compacted tasks, cursor, rule counts
    uint64_t ticket = 0;
    bool busy = false;
};

}  // namespace

struct ivde_server {
    int device = 0;
    char *arena_base = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    std::vector<Rig> rigs;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::thread thread;
    bool stop = false;

    void run();
    bool try_admit(Request &r);
    ivde_status enqueue(Request &r, Slot &sl, Rig &rig);
    void complete(Slot &sl);
    void fail(Request &r, ivde_status st);
    bool any_busy() const
    {
        for (const Slot &sl : slots)
            if (sl.busy) return true;
        return false;
    }
};

void ivde_server::run()
{
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
        // admit in arrival order; a request that does not fit yet blocks the
        // ones behind it so frames are not reordered
        while (!queue.empty()) {
            Request &r = reqs[queue.front()];
            if (try_admit(r)) {
                queue.pop_front();
                continue;
            }
            // nothing in flight and still no room: it can never fit
            if (!any_busy() && r.work_bytes > arena.largest()) {
                queue.pop_front();
                fail(r, IVDE_EBUDGET);
                continue;
            }
            break;
        }
        // completions
        bool inflight = false;
        for (Slot &sl : slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q != hipErrorNotReady) complete(sl);   // done, or failed (status recorded)
            else inflight = true;
        }
        if (inflight) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else if (queue.empty() && !stop) {
            cv_sched.wait(lk);
        }
    }
}

bool ivde_server::try_admit(Request &r)
{
    Rig &rig = rigs[r.rig];
    int free_slot = -1;
    for (size_t i = 0; i < slots.size(); ++i)
        if (!slots[i].busy) {
            free_slot = (int)i;
            break;
        }
    if (free_slot < 0) return false;
    size_t off = 0;
    if (!arena.alloc(r.work_bytes, &off)) return false;
    r.work_off = off;
    r.slot = free_slot;
    Slot &sl = slots[free_slot];
    sl.busy = true;
    sl.ticket = r.ticket;
    r.st.start_us = now_us();
    ivde_status st = enqueue(r, sl, rig);
    if (st != IVDE_OK) {
        r.st.status = st;
        // nothing may still be running from a failed enqueue: wait it out
        (void)hipStreamSynchronize(sl.stream);
        complete(sl);
    }
    return true;
}

ivde_status ivde_server::enqueue(Request &r, Slot &sl, Rig &rig)
{
    hipStream_t s = sl.stream;
    hipError_t e;
    if (rig.last_valid && (e = hipStreamWaitEvent(s, rig.last, 0)) != hipSuccess) return hip_fail(e, "rig order");
    char *ws = rig.ws;
    const Layout &ly = r.ly;
    Task *tasks = reinterpret_cast<Task *>(ws + ly.off_tasks);
    // the first frame (or one with another texel format) builds the index
    const bool index_ready = rig.index_tex == ly.tex_f32;
    rig.index_tex = -1;
    ivde_status st = enqueue_front(rig.n, rig.cams.data(), r.views.data(), rig.segs.data(), &rig.labels, &rig.opt, ly,
                                   ws, rig.cost, 0, tasks, s, index_ready);
    if (st != IVDE_OK) return st;
    rig.index_tex = ly.tex_f32;
    const Problem *dp = reinterpret_cast<const Problem *>(ws + ly.off_problem);
    const int bil = rig.opt.sampling == IVDE_BILINEAR;
    char *extra = arena_base + r.work_off;
    // [0] tasks kept, [2..4] rule counts, [8, 8 + kXcds) sweep cursors, [8 + kXcds] task count of a full sweep
    int32_t *counters = reinterpret_cast<int32_t *>(extra);
    Task *changed = reinterpret_cast<Task *>(extra + 256);
    uint8_t *source = reinterpret_cast<uint8_t *>(extra + 256 + align_up(sizeof(Task) * (size_t)ly.n_tasks, 256));
    uint8_t *rule_mask = source + align_up((size_t)ly.total_rows, 256);
    float *mean = reinterpret_cast<float *>(ws + ly.off_mean);
    const size_t mean_bytes = (size_t)ly.total_rows * 16;
    const bool full = r.rule ? (r.iframe || !rig.has_prev || !rig.has_i) : (!r.mask || !rig.has_prev);
    const uint8_t *mask = r.mask;
    for (int k = 0; k < 8; ++k) sl.count_host[k] = 0;
    if (r.rule && (e = launch_segment_stats(dp, extents_of(ly), nullptr, s)) != hipSuccess)
        return hip_fail(e, "serve segment statistics");
    if (full) {
        if ((e = launch_sweep(dp, tasks, ly.n_tasks, ly.J, bil, ly.tex_f32, ly.f16, ly.wpg, counters + 8, s)) !=
            hipSuccess)
            return hip_fail(e, "serve sweep");
        sl.count_host[0] = (int32_t)ly.n_tasks;
        if (r.rule) {
            // this frame becomes the I frame of the rule
            if ((e = launch_copy_rows(rig.cost, rig.cost_i, (int64_t)rig.cost_bytes, s)) != hipSuccess ||
                (e = launch_copy_rows(mean, rig.mean_i, (int64_t)mean_bytes, s)) != hipSuccess ||
                (e = launch_copy_rows(mean, rig.mean_prev, (int64_t)mean_bytes, s)) != hipSuccess)
                return hip_fail(e, "serve I frame state");
            rig.has_i = true;
        }
    } else {
        if ((e = launch_fill_i32(counters, 0, 8 + kXcds, s)) != hipSuccess) return hip_fail(e, "serve counters");
        if (r.rule) {
            const float scale = (float)(1 << (r.views[0].bit_depth - 8));
            if ((e = launch_temporal_rule(ly.total_rows, mean, rig.mean_prev, rig.mean_i, rig.t_p * scale,
                                          rig.t_i * scale, source, rule_mask, counters + 2, s)) != hipSuccess)
                return hip_fail(e, "serve temporal rule");
            // rows unchanged since the I frame adopt its result; rows
            // unchanged since the previous frame keep the resident row
            if ((e = launch_copy_rows_where(ly.total_rows, ly.L * (ly.f16 ? 2 : 4), source, 2, rig.cost_i, rig.cost,
                                            s)) != hipSuccess)
                return hip_fail(e, "serve I-frame rows");
            mask = rule_mask;
        }
        if ((e = launch_compact_tasks(dp, tasks, ly.n_tasks, mask, changed, counters, s)) != hipSuccess)
            return hip_fail(e, "serve compaction");
        int per_cu = 0, cus = 0;
        if ((e = sweep_persistent_occupancy(ly.J, bil, ly.tex_f32, ly.f16, ly.wpg, &per_cu)) != hipSuccess)
            return hip_fail(e, "occupancy");
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess)
            return hip_fail(e, "device attribute");
        if ((e = launch_sweep_persistent(dp, changed, counters, counters + 8, ly.n_tasks, ly.J, bil, ly.tex_f32, ly.f16,
                                         ly.wpg, std::max(1, per_cu) * std::max(1, cus), s)) != hipSuccess)
            return hip_fail(e, "serve sweep");
        if ((e = hipMemcpyAsync(sl.count_host, counters, 5 * sizeof(int32_t), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
            return hip_fail(e, "serve count");
        if (r.rule && (e = launch_copy_rows(mean, rig.mean_prev, (int64_t)mean_bytes, s)) != hipSuccess)
            return hip_fail(e, "serve mean colours");
    }
    if (r.label_out &&
        (e = launch_argmin(rig.cost, ly.f16, ly.total_rows, rig.labels.num_labels, r.label_out, s)) != hipSuccess)
        return hip_fail(e, "serve argmin");
    if (r.cost_out && (e = launch_copy_rows(rig.cost, r.cost_out, (int64_t)rig.cost_bytes, s)) != hipSuccess)
        return hip_fail(e, "serve copy");
    if ((e = hipEventRecord(sl.done, s)) != hipSuccess) return hip_fail(e, "serve event");
    if ((e = hipEventRecord(rig.last, s)) != hipSuccess) return hip_fail(e, "serve event");
    rig.last_valid = true;
    rig.has_prev = true;
    r.st.rows_total = ly.total_rows;
    return IVDE_OK;
}

void ivde_server::complete(Slot &sl)
{
    Request &r = reqs[sl.ticket];
    Rig &rig = rigs[r.rig];
    r.st.done_us = now_us();
    if (r.st.status == IVDE_OK) {
        const hipError_t q = hipEventQuery(sl.done);
        if (q != hipSuccess) r.st.status = IVDE_EHIP;
    }
    if (r.st.status == IVDE_OK) {
        r.st.rows_recomputed = (int64_t)sl.count_host[0] / std::max(1, r.ly.n_lblocks);
        r.st.rows_from_iframe = sl.count_host[4];   // rule counts: [2] recompute, [3] keep, [4] I frame
    }
    arena.release(r.work_off, r.work_bytes);
    sl.busy = false;
    r.done = true;
    rig.pending--;
    cv_done.notify_all();
}

void ivde_server::fail(Request &r, ivde_status st)
{
    r.st.status = st;
    r.st.start_us = r.st.done_us = now_us();
    r.done = true;
    rigs[r.rig].pending--;
    cv_done.notify_all();
}

extern "C" {

ivde_status ivde_server_create(const ivde_server_config *cfg, ivde_server **out)
{
    if (!cfg || !out || !cfg->arena || cfg->arena_bytes < 256 || cfg->max_slots < 1 || cfg->max_slots > 16) {
        set_error("server: need an arena, at least 256 bytes, and 1..16 slots");
        return IVDE_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(cfg->arena) % 256) {
        set_error("server: the arena must be 256-byte aligned");
        return IVDE_EINVAL;
    }
    *out = nullptr;
    ivde_server *s = new (std::nothrow) ivde_server;
    if (!s) {
        set_error("server: out of host memory");
        return IVDE_ENOMEM;
    }
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "get device");
    }
    s->arena_base = static_cast<char *>(cfg->arena);
    s->arena.init(cfg->arena_bytes);
    s->slots.resize(cfg->max_slots);
    for (Slot &sl : s->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipHostMalloc(reinterpret_cast<void **>(&sl.count_host), 8 * sizeof(int32_t), hipHostMallocDefault)) !=
                hipSuccess) {
            ivde_server_destroy(s);
            return hip_fail(e, "server resources");
        }
        for (int k = 0; k < 8; ++k) sl.count_host[k] = 0;
    }
    s->thread = std::thread([s] { s->run(); });
    *out = s;
    return IVDE_OK;
}

ivde_status ivde_rig_register(ivde_server *srv, int32_t n_views, const ivde_camera *cams,
                              const ivde_segmentation *segs, const ivde_label_range *labels, const ivde_options *opt,
                              int32_t *rig_id)
{
    if (!srv || !rig_id) {
        set_error("rig_register: null argument");
        return IVDE_EINVAL;
    }
    ivde_status st = validate_problem(n_views, cams, nullptr, segs, labels, opt, false);
    if (st != IVDE_OK) return st;
    if (opt->targets == IVDE_TARGETS_EXPLICIT) {
        set_error("rig_register: use IVDE_TARGETS_ALL or IVDE_TARGETS_NEAREST_LR");
        return IVDE_EINVAL;
    }
    Rig rig;
    rig.n = n_views;
    rig.cams.assign(cams, cams + n_views);
    rig.labels = *labels;
    rig.opt = *opt;
    rig.opt.sweep_events[0] = rig.opt.sweep_events[1] = nullptr;
    rig.ly = plan_layout(n_views, cams, segs, labels, &rig.opt, 16);
    if ((st = check_tex_limits(rig.ly)) != IVDE_OK) return st;
    rig.cost_bytes = rig.ly.cost_bytes;
    std::vector<size_t> seg_off(n_views);
    size_t seg_bytes = 0;
    rig.res_bytes = resident_bytes(n_views, cams, rig.ly, seg_off.data(), &seg_bytes);
    const size_t mean_bytes = align_up((size_t)rig.ly.total_rows * 16, 256);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (!srv->arena.alloc(rig.res_bytes, &rig.res_off)) {
        set_error("rig_register: the rig's resident state (%zu bytes) does not fit the arena", rig.res_bytes);
        return IVDE_EBUDGET;
    }
    char *base = srv->arena_base + rig.res_off;
    rig.ws = base + seg_bytes;
    rig.cost = rig.ws + align_up(rig.ly.workspace_bytes, 256);
    rig.cost_i = rig.cost + align_up(rig.cost_bytes, 256);
    rig.mean_prev = reinterpret_cast<float *>(rig.cost_i + align_up(rig.cost_bytes, 256));
    rig.mean_i = reinterpret_cast<float *>(reinterpret_cast<char *>(rig.mean_prev) + mean_bytes);
    rig.segs.resize(n_views);
    hipError_t e = hipSuccess;
    for (int v = 0; v < n_views && e == hipSuccess; ++v) {
        int32_t *dst = reinterpret_cast<int32_t *>(base + seg_off[v]);
        e = hipMemcpy2D(dst, sizeof(int32_t) * cams[v].width, segs[v].seg_map, sizeof(int32_t) * segs[v].pitch,
                        sizeof(int32_t) * cams[v].width, cams[v].height, hipMemcpyDeviceToDevice);
        rig.segs[v] = segs[v];
        rig.segs[v].seg_map = dst;
        rig.segs[v].pitch = cams[v].width;
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&rig.last, hipEventDisableTiming);
    if (e != hipSuccess) {
        srv->arena.release(rig.res_off, rig.res_bytes);
        return hip_fail(e, "rig_register");
    }
    rig.id = (int)srv->rigs.size();
    *rig_id = rig.id;
    srv->rigs.push_back(std::move(rig));
    return IVDE_OK;
}

static ivde_status submit(ivde_server *srv, int32_t rig_id, const ivde_image *views, const uint8_t *changed_mask,
                          bool rule, bool iframe, void *cost_out, int32_t *label_out, uint64_t *ticket);

ivde_status ivde_server_footprint(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                                  const ivde_label_range *labels, const ivde_options *opt, int32_t bit_depth,
                                  size_t *resident, size_t *per_request)
{
    ivde_status st = validate_problem(n_views, cams, nullptr, segs, labels, opt, false);
    if (st != IVDE_OK) return st;
    if (bit_depth < 8 || bit_depth > 16) {
        set_error("bit_depth must be 8..16");
        return IVDE_EINVAL;
    }
    ivde_options o = *opt;
    o.sweep_events[0] = o.sweep_events[1] = nullptr;
    // the resident workspace is sized for 16-bit images, as at registration
    const Layout big = plan_layout(n_views, cams, segs, labels, &o, 16);
    const Layout ly = plan_layout(n_views, cams, segs, labels, &o, bit_depth);
    if (resident) *resident = align_up(resident_bytes(n_views, cams, big, nullptr, nullptr), 256);
    if (per_request) *per_request = align_up(working_set(ly), 256);
    return IVDE_OK;
}

ivde_status ivde_stream_submit(ivde_server *srv, int32_t rig_id, const ivde_image *views, const uint8_t *changed_mask,
                               void *cost_out, int32_t *label_out, uint64_t *ticket)
{
    return submit(srv, rig_id, views, changed_mask, false, false, cost_out, label_out, ticket);
}

ivde_status ivde_stream_submit_rule(ivde_server *srv, int32_t rig_id, const ivde_image *views, int32_t iframe,
                                    void *cost_out, int32_t *label_out, uint64_t *ticket)
{
    return submit(srv, rig_id, views, nullptr, true, iframe != 0, cost_out, label_out, ticket);
}

ivde_status ivde_rig_set_temporal(ivde_server *srv, int32_t rig_id, float t_p, float t_i)
{
    if (!srv || !(t_p >= 0.f) || !(t_i >= 0.f)) {
        set_error("rig_set_temporal: thresholds must be >= 0");
        return IVDE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (rig_id < 0 || rig_id >= (int)srv->rigs.size()) {
        set_error("rig_set_temporal: unknown rig");
        return IVDE_ENOTFOUND;
    }
    srv->rigs[rig_id].t_p = t_p;
    srv->rigs[rig_id].t_i = t_i;
    return IVDE_OK;
}

}  // extern "C"

static ivde_status submit(ivde_server *srv, int32_t rig_id, const ivde_image *views, const uint8_t *changed_mask,
                          bool rule, bool iframe, void *cost_out, int32_t *label_out, uint64_t *ticket)
{
    if (!srv || !views || !ticket) {
        set_error("stream_submit: null argument");
        return IVDE_EINVAL;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    if (rig_id < 0 || rig_id >= (int)srv->rigs.size()) {
        set_error("stream_submit: unknown rig %d", rig_id);
        return IVDE_ENOTFOUND;
    }
    Rig &rig = srv->rigs[rig_id];
    ivde_status st = validate_problem(rig.n, rig.cams.data(), views, rig.segs.data(), &rig.labels, &rig.opt, true);
    if (st != IVDE_OK) return st;
    Request r;
    r.ly = plan_layout(rig.n, rig.cams.data(), rig.segs.data(), &rig.labels, &rig.opt, views[0].bit_depth);
    r.work_bytes = working_set(r.ly);
    // with nothing queued or in flight the free space cannot grow: refuse now
    if (r.work_bytes > srv->arena.largest() && srv->queue.empty() && !srv->any_busy()) {
        set_error("stream_submit: the request's working set (%zu bytes) can never fit the arena", r.work_bytes);
        return IVDE_EBUDGET;
    }
    r.ticket = srv->next_ticket++;
    r.rig = rig_id;
    r.views.assign(views, views + rig.n);
    r.mask = changed_mask;
    r.rule = rule;
    r.iframe = iframe;
    r.cost_out = cost_out;
    r.label_out = label_out;
    r.st.ticket = r.ticket;
    r.st.rig_id = rig_id;
    r.st.status = IVDE_OK;
    r.st.submit_us = now_us();
    rig.pending++;
    *ticket = r.ticket;
    srv->queue.push_back(r.ticket);
    srv->reqs.emplace(r.ticket, std::move(r));
    srv->cv_sched.notify_one();
    return IVDE_OK;
}

extern "C" {

ivde_status ivde_stream_poll(ivde_server *srv, uint64_t ticket, ivde_frame_stats *st)
{
    if (!srv) {
        set_error("stream_poll: null server");
        return IVDE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) {
        set_error("stream_poll: unknown ticket");
        return IVDE_ENOTFOUND;
    }
    if (!it->second.done) return IVDE_EBUSY;
    if (st) *st = it->second.st;
    const ivde_status s = it->second.st.status;
    srv->reqs.erase(it);
    return s;
}

ivde_status ivde_stream_wait(ivde_server *srv, uint64_t ticket, ivde_frame_stats *st)
{
    if (!srv) {
        set_error("stream_wait: null server");
        return IVDE_EINVAL;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) {
        set_error("stream_wait: unknown ticket");
        return IVDE_ENOTFOUND;
    }
    srv->cv_done.wait(lk, [&] { return it->second.done; });
    if (st) *st = it->second.st;
    const ivde_status s = it->second.st.status;
    srv->reqs.erase(it);
    return s;
}

ivde_status ivde_rig_resident(ivde_server *srv, int32_t rig_id, const void **cost, int64_t *rows)
{
    if (!srv) {
        set_error("rig_resident: null server");
        return IVDE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (rig_id < 0 || rig_id >= (int)srv->rigs.size()) {
        set_error("rig_resident: unknown rig");
        return IVDE_ENOTFOUND;
    }
    if (cost) *cost = srv->rigs[rig_id].cost;
    if (rows) *rows = srv->rigs[rig_id].ly.total_rows;
    return IVDE_OK;
}

ivde_status ivde_rig_reset(ivde_server *srv, int32_t rig_id)
{
    if (!srv) {
        set_error("rig_reset: null server");
        return IVDE_EINVAL;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    if (rig_id < 0 || rig_id >= (int)srv->rigs.size()) {
        set_error("rig_reset: unknown rig");
        return IVDE_ENOTFOUND;
    }
    srv->rigs[rig_id].has_prev = false;   // the next admitted frame sweeps every row
    srv->rigs[rig_id].has_i = false;
    return IVDE_OK;
}

void ivde_server_destroy(ivde_server *srv)
{
    if (!srv) return;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        // let queued and in-flight requests finish
        srv->cv_done.wait(lk, [&] {
            bool busy = !srv->queue.empty();
            for (const Slot &sl : srv->slots) busy |= sl.busy;
            return !busy || !srv->thread.joinable();
        });
        srv->stop = true;
        srv->cv_sched.notify_all();
    }
    if (srv->thread.joinable()) srv->thread.join();
    for (Slot &sl : srv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.count_host) (void)hipHostFree(sl.count_host);
    }
    for (Rig &r : srv->rigs)
        if (r.last) (void)hipEventDestroy(r.last);
    delete srv;
}

}  // extern "C"
