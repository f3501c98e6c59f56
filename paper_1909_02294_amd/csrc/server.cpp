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
// previous frame, because each frame starts from that frame's volume, and a
// frame's kernels are enqueued only once its predecessor's are.  Every row is
// computed by the same per-task kernel code as ivde_cost_volume, so a frame's
// result does not depend on what else is in flight.
//
// Full-frame sweeps (I frames) are cut into launches of about chunk_evals
// evaluations.  The persistent sweep holds every CU until its task list is
// drained, so one launch over a whole I frame would make the short frames of
// other rigs that arrive meanwhile wait for all of it.  The scheduler
// enqueues the next launch of a cut sweep only after the previous one has
// completed and while no uncut request is in flight, so a P frame admitted
// during an I frame waits at most for the launch that is running.  Once the
// I frame's own rig has its next frame admitted, the I frame no longer gives
// way: that frame starts from the I frame's volume and waits for it anyway.
//
// Frames may also be handed over in host memory (ivde_stream_submit_host):
// the planes and the mask are copied into the request's working set on its
// stream right at admission, ahead of everything else, so the upload
// overlaps the rig's previous frame and counts in the frame's latency.
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
    std::vector<ivde_image> views;         // device images the kernels read
    const uint8_t *mask = nullptr;         // device changed mask, NULL: every row
    bool rule = false;                     // derive the mask by the temporal rule
    bool iframe = false;                   // rule mode: compute every row and make this the I frame
    bool host = false;                     // planes and mask were handed over in host memory
    std::vector<ivde_image> host_views;
    const uint8_t *host_mask = nullptr;
    void *cost_out = nullptr;
    int32_t *label_out = nullptr;
    ivde_frame_stats st{};
    Layout ly{};                           // depends on the frame's bit depth
    size_t work_bytes = 0;                 // working set, plus the staged planes of a host frame
    int slot = -1;
    size_t work_off = 0;
    bool started = false;                  // its first kernels are enqueued
    bool enqueued = false;                 // all its work and its completion events are enqueued
    bool full = false;                     // every row is swept
    int64_t chunk_tasks = 0;               // > 0: the full sweep runs in launches of this many tasks
    int64_t chunk_next = 0;                // first task of the next launch
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

// Device bytes of a host frame's staged planes (each plane packed, rows of
// its width) and its mask.
size_t host_staging(int n, const ivde_camera *cams, int bit_depth, int chroma_shift, int64_t rows)
{
    const size_t esz = bit_depth > 8 ? 2 : 1;
    size_t b = 0;
    for (int v = 0; v < n; ++v) {
        const size_t W = (size_t)cams[v].width, H = (size_t)cams[v].height;
        const size_t cw = (W + chroma_shift) >> chroma_shift, ch = (H + chroma_shift) >> chroma_shift;
        b += align_up(W * H * esz, 256) + 2 * align_up(cw * ch * esz, 256);
    }
    return b + align_up((size_t)rows, 256);
}

// Pixel-label-target evaluations of a full sweep of a rig.
int64_t frame_evals(int n, const ivde_camera *cams, const ivde_label_range &labels, const ivde_options &opt)
{
    int64_t e = 0;
    for (int c = 0; c < n; ++c) {
        const int targets = opt.targets == IVDE_TARGETS_NEAREST_LR ? (c > 0) + (c < n - 1) : n - 1;
        e += (int64_t)cams[c].width * cams[c].height * labels.num_labels * targets;
    }
    return e;
}

constexpr int64_t kDefaultChunkEvals = 8000000000LL;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t chunk = nullptr;            // completion of the latest launch of a cut sweep
    int32_t *count_host = nullptr;         // pinned [8]: compacted tasks, cursor, rule counts
    uint64_t ticket = 0;
    bool busy = false;
};

}  // namespace

struct ivde_server {
    int device = 0;
    char *arena_base = nullptr;
    Arena arena;
    int64_t chunk_evals = kDefaultChunkEvals;   // <= 0: full sweeps in one launch
    std::vector<Slot> slots;
    std::vector<Rig> rigs;
    std::deque<uint64_t> queue;
    std::vector<uint64_t> active;          // admitted, not all work enqueued yet; admission order
    std::map<uint64_t, Request> reqs;
    uint64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::thread thread;
    bool stop = false;

    void run();
    bool try_admit(Request &r);
    void progress();
    ivde_status start(Request &r, Slot &sl, Rig &rig);
    ivde_status pump(Request &r, Slot &sl, Rig &rig);
    ivde_status finish(Request &r, Slot &sl, Rig &rig);
    bool uncut_in_flight(uint64_t except) const;
    void abort(Request &r, Slot &sl, ivde_status st);
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
        progress();
        // completions of requests whose work is all enqueued
        bool inflight = false;
        for (Slot &sl : slots) {
            if (!sl.busy) continue;
            if (!reqs[sl.ticket].enqueued) {
                inflight = true;
                continue;
            }
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

// Reserves a slot and the working set; a host frame's planes and mask start
// uploading at once on the slot's stream.
bool ivde_server::try_admit(Request &r)
{
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
    active.push_back(r.ticket);
    if (r.host) {
        const Rig &rig = rigs[r.rig];
        char *stage = arena_base + r.work_off + align_up(working_set(r.ly), 256);
        hipError_t e = hipSuccess;
        for (int v = 0; v < rig.n && e == hipSuccess; ++v) {
            const ivde_image &h = r.host_views[v];
            const size_t esz = h.bit_depth > 8 ? 2 : 1;
            for (int i = 0; i < 3 && e == hipSuccess; ++i) {
                const int k = i ? h.chroma_shift : 0;
                const size_t w = ((size_t)rig.cams[v].width + k) >> k, hh = ((size_t)rig.cams[v].height + k) >> k;
                e = hipMemcpy2DAsync(stage, w * esz, h.plane[i], (size_t)h.pitch[i] * esz, w * esz, hh,
                                     hipMemcpyHostToDevice, sl.stream);
                r.views[v].plane[i] = stage;
                r.views[v].pitch[i] = (int64_t)w;
                stage += align_up(w * hh * esz, 256);
            }
        }
        if (e == hipSuccess && r.host_mask) {
            e = hipMemcpyAsync(stage, r.host_mask, (size_t)r.ly.total_rows, hipMemcpyHostToDevice, sl.stream);
            r.mask = reinterpret_cast<const uint8_t *>(stage);
        }
        if (e != hipSuccess) abort(r, sl, hip_fail(e, "serve upload"));
    }
    return true;
}

// True if a request other than `except` whose work is enqueued in one piece
// (a P frame, or a full frame too small to cut) has not completed.
bool ivde_server::uncut_in_flight(uint64_t except) const
{
    for (const Slot &sl : slots) {
        if (!sl.busy || sl.ticket == except) continue;
        const Request &q = reqs.at(sl.ticket);
        if (q.started && q.chunk_tasks == 0 && !q.done) return true;
    }
    return false;
}

// Starts admitted requests whose rig has no earlier request still being
// enqueued, and enqueues the next launch of cut sweeps whose previous launch
// has completed while no uncut request is in flight.
void ivde_server::progress()
{
    std::vector<int> pending_rigs;   // rigs with an earlier request not all enqueued
    // A cut sweep whose rig already has its next frame admitted stops giving
    // way: that frame waits for it by construction.
    std::vector<int> admitted(rigs.size(), 0);
    for (uint64_t t : active) admitted[reqs[t].rig]++;
    for (size_t i = 0; i < active.size();) {
        Request &r = reqs[active[i]];
        Slot &sl = slots[r.slot];
        Rig &rig = rigs[r.rig];
        const bool after_pending =
            std::find(pending_rigs.begin(), pending_rigs.end(), r.rig) != pending_rigs.end();
        if (!r.enqueued && !r.started && !after_pending) {
            const ivde_status st = start(r, sl, rig);
            if (st != IVDE_OK) abort(r, sl, st);
        } else if (!r.enqueued && r.started && hipEventQuery(sl.chunk) != hipErrorNotReady &&
                   (admitted[r.rig] > 1 || !uncut_in_flight(r.ticket))) {
            const ivde_status st = pump(r, sl, rig);
            if (st != IVDE_OK) abort(r, sl, st);
        }
        if (r.enqueued) {
            active.erase(active.begin() + (std::ptrdiff_t)i);
        } else {
            pending_rigs.push_back(r.rig);
            ++i;
        }
    }
}

// A request whose enqueue failed: nothing of it may still run when its
// memory is released.
void ivde_server::abort(Request &r, Slot &sl, ivde_status st)
{
    r.st.status = st;
    (void)hipStreamSynchronize(sl.stream);
    r.started = r.enqueued = true;
}

ivde_status ivde_server::start(Request &r, Slot &sl, Rig &rig)
{
    hipStream_t s = sl.stream;
    hipError_t e;
    r.started = true;
    if (rig.last_valid && (e = hipStreamWaitEvent(s, rig.last, 0)) != hipSuccess) return hip_fail(e, "rig order");
    char *ws = rig.ws;
    const Layout &ly = r.ly;
    Task *tasks = reinterpret_cast<Task *>(ws + ly.off_tasks);
    // the first frame (or one with another texel format) builds the index
    const bool index_ready = rig.index_tex == ly.tex_u16;
    rig.index_tex = -1;
    ivde_status st = enqueue_front(rig.n, rig.cams.data(), r.views.data(), rig.segs.data(), &rig.labels, &rig.opt, ly,
                                   ws, rig.cost, 0, tasks, s, index_ready);
    if (st != IVDE_OK) return st;
    rig.index_tex = ly.tex_u16;
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
    r.full = r.rule ? (r.iframe || !rig.has_prev || !rig.has_i) : (!r.mask || !rig.has_prev);
    const uint8_t *mask = r.mask;
    for (int k = 0; k < 8; ++k) sl.count_host[k] = 0;
    if (r.rule && (e = launch_segment_stats(dp, extents_of(ly), nullptr, s)) != hipSuccess)
        return hip_fail(e, "serve segment statistics");
    if (r.full) {
        sl.count_host[0] = (int32_t)ly.n_tasks;
        const int64_t evals = frame_evals(rig.n, rig.cams.data(), rig.labels, rig.opt);
        const int64_t pieces = chunk_evals > 0 ? (evals + chunk_evals - 1) / chunk_evals : 1;
        r.chunk_tasks = pieces > 1 && ly.n_tasks > 1 ? (ly.n_tasks + pieces - 1) / pieces : 0;
        if (r.chunk_tasks > 0) return pump(r, sl, rig);
        if ((e = launch_sweep(dp, tasks, ly.n_tasks, ly.J, ly.px, bil, ly.tex_u16, ly.f16, ly.wpg, counters + 8, s)) !=
            hipSuccess)
            return hip_fail(e, "serve sweep");
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
        if ((e = sweep_persistent_occupancy(ly.J, ly.px, bil, ly.tex_u16, ly.f16, ly.wpg, &per_cu)) != hipSuccess)
            return hip_fail(e, "occupancy");
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess)
            return hip_fail(e, "device attribute");
        if ((e = launch_sweep_persistent(dp, changed, counters, counters + 8, ly.n_tasks, ly.J, ly.px, bil, ly.tex_u16, ly.f16,
                                         ly.wpg, std::max(1, per_cu) * std::max(1, cus), s)) != hipSuccess)
            return hip_fail(e, "serve sweep");
        if ((e = hipMemcpyAsync(sl.count_host, counters, 5 * sizeof(int32_t), hipMemcpyDeviceToHost, s)) !=
            hipSuccess)
            return hip_fail(e, "serve count");
        if (r.rule && (e = launch_copy_rows(mean, rig.mean_prev, (int64_t)mean_bytes, s)) != hipSuccess)
            return hip_fail(e, "serve mean colours");
    }
    return finish(r, sl, rig);
}

// The next launch of a cut full sweep; after the last one, the frame's tail.
ivde_status ivde_server::pump(Request &r, Slot &sl, Rig &rig)
{
    const Layout &ly = r.ly;
    const Problem *dp = reinterpret_cast<const Problem *>(rig.ws + ly.off_problem);
    const Task *tasks = reinterpret_cast<const Task *>(rig.ws + ly.off_tasks);
    int32_t *counters = reinterpret_cast<int32_t *>(arena_base + r.work_off);
    const int64_t n = std::min(r.chunk_tasks, ly.n_tasks - r.chunk_next);
    hipError_t e = launch_sweep(dp, tasks + r.chunk_next, n, ly.J, ly.px, rig.opt.sampling == IVDE_BILINEAR, ly.tex_u16,
                                ly.f16, ly.wpg, counters + 8, sl.stream);
    if (e != hipSuccess) return hip_fail(e, "serve sweep");
    r.chunk_next += n;
    if ((e = hipEventRecord(sl.chunk, sl.stream)) != hipSuccess) return hip_fail(e, "serve event");
    return r.chunk_next >= ly.n_tasks ? finish(r, sl, rig) : IVDE_OK;
}

// The frame's work after its sweep: the I-frame state of the rule, argmin,
// the copy out, and the completion events.
ivde_status ivde_server::finish(Request &r, Slot &sl, Rig &rig)
{
    hipStream_t s = sl.stream;
    hipError_t e;
    const Layout &ly = r.ly;
    if (r.full && r.rule) {
        // this frame becomes the I frame of the rule
        float *mean = reinterpret_cast<float *>(rig.ws + ly.off_mean);
        const int64_t mean_bytes = ly.total_rows * 16;
        if ((e = launch_copy_rows(rig.cost, rig.cost_i, (int64_t)rig.cost_bytes, s)) != hipSuccess ||
            (e = launch_copy_rows(mean, rig.mean_i, mean_bytes, s)) != hipSuccess ||
            (e = launch_copy_rows(mean, rig.mean_prev, mean_bytes, s)) != hipSuccess)
            return hip_fail(e, "serve I frame state");
        rig.has_i = true;
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
    r.enqueued = true;
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
    if (cfg->reserved != 0) {
        set_error("server: the reserved field must be 0");
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
    s->chunk_evals = cfg->chunk_evals == 0 ? kDefaultChunkEvals : cfg->chunk_evals;
    s->slots.resize(cfg->max_slots);
    for (Slot &sl : s->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.chunk, hipEventDisableTiming)) != hipSuccess ||
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
                          bool rule, bool iframe, bool host, void *cost_out, int32_t *label_out, uint64_t *ticket);

ivde_status ivde_server_footprint(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                                  const ivde_label_range *labels, const ivde_options *opt, int32_t bit_depth,
                                  int32_t chroma_shift, size_t *resident, size_t *per_request,
                                  size_t *per_host_request)
{
    ivde_status st = validate_problem(n_views, cams, nullptr, segs, labels, opt, false);
    if (st != IVDE_OK) return st;
    if (bit_depth < 8 || bit_depth > 16) {
        set_error("bit_depth must be 8..16");
        return IVDE_EINVAL;
    }
    if (chroma_shift != 0 && chroma_shift != 1) {
        set_error("chroma_shift must be 0 or 1");
        return IVDE_EINVAL;
    }
    ivde_options o = *opt;
    o.sweep_events[0] = o.sweep_events[1] = nullptr;
    // the resident workspace is sized for 16-bit images, as at registration
    const Layout big = plan_layout(n_views, cams, segs, labels, &o, 16);
    const Layout ly = plan_layout(n_views, cams, segs, labels, &o, bit_depth);
    if (resident) *resident = align_up(resident_bytes(n_views, cams, big, nullptr, nullptr), 256);
    if (per_request) *per_request = align_up(working_set(ly), 256);
    if (per_host_request)
        *per_host_request = align_up(working_set(ly), 256) +
                            align_up(host_staging(n_views, cams, bit_depth, chroma_shift, ly.total_rows), 256);
    return IVDE_OK;
}

ivde_status ivde_stream_submit(ivde_server *srv, int32_t rig_id, const ivde_image *views, const uint8_t *changed_mask,
                               void *cost_out, int32_t *label_out, uint64_t *ticket)
{
    return submit(srv, rig_id, views, changed_mask, false, false, false, cost_out, label_out, ticket);
}

ivde_status ivde_stream_submit_rule(ivde_server *srv, int32_t rig_id, const ivde_image *views, int32_t iframe,
                                    void *cost_out, int32_t *label_out, uint64_t *ticket)
{
    return submit(srv, rig_id, views, nullptr, true, iframe != 0, false, cost_out, label_out, ticket);
}

ivde_status ivde_stream_submit_host(ivde_server *srv, int32_t rig_id, const ivde_image *host_views, int32_t mode,
                                    const uint8_t *changed_mask, void *cost_out, int32_t *label_out,
                                    uint64_t *ticket)
{
    if (mode != IVDE_SUBMIT_MASK && mode != IVDE_SUBMIT_RULE && mode != IVDE_SUBMIT_RULE_IFRAME) {
        set_error("stream_submit_host: unknown mode %d", mode);
        return IVDE_EINVAL;
    }
    if (mode != IVDE_SUBMIT_MASK && changed_mask) {
        set_error("stream_submit_host: the rule modes take no mask");
        return IVDE_EINVAL;
    }
    return submit(srv, rig_id, host_views, changed_mask, mode != IVDE_SUBMIT_MASK, mode == IVDE_SUBMIT_RULE_IFRAME,
                  true, cost_out, label_out, ticket);
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
                          bool rule, bool iframe, bool host, void *cost_out, int32_t *label_out, uint64_t *ticket)
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
    if (host)
        r.work_bytes = align_up(r.work_bytes, 256) + host_staging(rig.n, rig.cams.data(), views[0].bit_depth,
                                                                  views[0].chroma_shift, r.ly.total_rows);
    // with nothing queued or in flight the free space cannot grow: refuse now
    if (r.work_bytes > srv->arena.largest() && srv->queue.empty() && !srv->any_busy()) {
        set_error("stream_submit: the request's working set (%zu bytes) can never fit the arena", r.work_bytes);
        return IVDE_EBUDGET;
    }
    r.ticket = srv->next_ticket++;
    r.rig = rig_id;
    r.views.assign(views, views + rig.n);
    r.host = host;
    if (host) {
        r.host_views = r.views;
        r.host_mask = changed_mask;
    } else {
        r.mask = changed_mask;
    }
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
        if (sl.chunk) (void)hipEventDestroy(sl.chunk);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.count_host) (void)hipHostFree(sl.count_host);
    }
    for (Rig &r : srv->rigs)
        if (r.last) (void)hipEventDestroy(r.last);
    delete srv;
}

}  // extern "C"
