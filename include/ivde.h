/*
 * ivde.h -- C ABI of libivde, the MI355X (gfx950) per-segment plane-sweep
 * matching-cost library.
 *
 * The method is the segment-based multiview depth estimator of Mieloch,
 * Stankiewicz and Domanski, "Depth Map Estimation for Free-Viewpoint
 * Television".  Its problem statement (Sec. I and Sec. III-A) takes
 * any number of arbitrarily positioned views with intrinsic and extrinsic
 * camera parameters, a segmentation of every view made independently per
 * view, a range of depth levels, and (for video) the segments that changed
 * since the previous frame (Sec. III-E).  This library computes the data
 * term that the paper's graph-cut optimisation consumes: for every segment s
 * of every view c and every depth level l, the mean YCbCr L1 distance
 * (Sec. III-C, Eq. (4)) between the segment's pixels and their
 * reprojections into the other views, minimum over the target views:
 *
 *     C[c][s][l] = min_{c' in D_c, n > 0}  (1 / n) sum_{p in s valid} e(p, c', l)
 *     e = (|dY| + |dCb| + |dCr|) / (3 (2^b - 1))        in [0, 1]
 *
 * Eq. (4) averages over a small window at the segment centre (Sec. III-C,
 * 3x3 in Sec. V-A); this library averages over every pixel of the segment,
 * each reprojected at its own position.  The graph cut itself (Sec. III-B,
 * IV-B) stays with the caller.
 *
 * Geometry conventions (fixed here because the paper only says the
 * transform comes from intrinsic and extrinsic parameters, Sec. III-C):
 *   - a camera maps a world point X to camera coordinates R X + t; K is
 *     3x3 with third row (0, 0, 1); all three are row-major FP64;
 *   - pixel centres are at integer (x, y), x to the right, y down;
 *   - depth levels are planes parallel to a reference camera plane
 *     (Sec. IV-A) at distances z_l, uniform in 1/z from z_far (label 0) to
 *     z_near (label L-1); the reference plane is the rig centre's (Sec.
 *     III-B: depth from the centre camera's plane): mean camera centre,
 *     normalised mean optical axis.  IVDE_REF_OWN uses each view's own plane
 *     and a camera index uses that camera's plane;
 *   - a pixel is valid for a (target, label) if its 3-D point lies in front
 *     of both cameras and its projection samples inside the target image:
 *     nearest: round-half-up of (u, v) inside [0, W) x [0, H); bilinear:
 *     (u, v) within 1/64 px of [0, W-1] x [0, H-1], clamped onto it.  Chroma
 *     is sampled with the luma weights at taps (x >> k, y >> k), k the
 *     chroma shift;
 *   - a segment with no valid pixel in any target gets the cost 1.0.
 *
 * Memory and threading conventions:
 *   - every image, segment map, cost volume, label output, workspace and
 *     arena pointer is DEVICE memory owned by the caller; cameras, options
 *     and target masks are host memory read during the call only;
 *   - calls are asynchronous on the given stream (a hipStream_t passed as
 *     ivde_stream; NULL is the null stream).  Argument errors are found
 *     synchronously, before anything is enqueued, and set a thread-local
 *     message for ivde_last_error().  Segment ids out of range are found on
 *     the device: the offending pixels are skipped and ivde_workspace_status
 *     reports IVDE_EINVAL after the stream has completed;
 *   - no C++ exception crosses this interface;
 *   - ivde_cost_volume and ivde_argmin are re-entrant as long as concurrent
 *     calls use distinct workspaces; every ivde_server call is thread-safe.
 */
#ifndef IVDE_H
#define IVDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ivde_status;
#define IVDE_OK 0
#define IVDE_EINVAL (-1)      /* invalid argument or segment id out of range */
#define IVDE_ENOMEM (-2)      /* host allocation failed or workspace too small */
#define IVDE_EBUDGET (-3)     /* request does not fit the server's HBM budget */
#define IVDE_EHIP (-4)        /* a HIP runtime call failed */
#define IVDE_EBUSY (-5)       /* result not ready yet */
#define IVDE_ENOTFOUND (-6)   /* unknown rig or ticket */

typedef void *ivde_stream;    /* hipStream_t */

#define IVDE_REF_RIG_CENTER (-1)
#define IVDE_REF_OWN (-2)

#define IVDE_NEAREST 0
#define IVDE_BILINEAR 1

#define IVDE_F32 0
#define IVDE_F16 1

#define IVDE_TARGETS_ALL 0          /* every other view */
#define IVDE_TARGETS_NEAREST_LR 1   /* views c-1 and c+1 (Sec. III-B's D) */
#define IVDE_TARGETS_EXPLICIT 2     /* target_mask[c * n + c'] != 0 */

/* One view's camera: intrinsics K and extrinsics (R, t), row-major FP64,
 * host memory (Sec. III-C: the 3-D transform T[.] is built from them). */
typedef struct {
    double K[9];
    double R[9];
    double t[3];
    int32_t width, height;
} ivde_camera;

/* One view's picture as Y, Cb, Cr planes (Sec. III-C uses YCbCr).
 * plane[i] are device pointers to uint8 (bit_depth 8) or uint16 (9..16)
 * samples; pitch[i] is the row pitch in samples.  chroma_shift 0 is 4:4:4,
 * 1 is 4:2:0 with ceil(W/2) x ceil(H/2) chroma planes. */
typedef struct {
    const void *plane[3];
    int64_t pitch[3];
    int32_t bit_depth;
    int32_t chroma_shift;
} ivde_image;

/* One view's segmentation (Sec. III-A: segmented independently per view):
 * device int32 ids in [0, num_segments), row pitch in elements. */
typedef struct {
    const int32_t *seg_map;
    int64_t pitch;
    int32_t num_segments;
} ivde_segmentation;

/* Depth levels (Sec. IV-A: planes parallel to the reference camera plane;
 * Sec. V-A uses 250).  Uniform in inverse depth, label 0 at z_far. */
typedef struct {
    double z_near, z_far;
    int32_t num_labels;
    int32_t depth_ref;        /* IVDE_REF_RIG_CENTER, IVDE_REF_OWN or a view index */
} ivde_label_range;

/* Options.  labels_per_lane (1, 2, 4 or 8) and waves_per_group (1, 2 or 4)
 * are launch-shape knobs; 0 picks the tuned default.  They never change a
 * result.  pixels_per_step 2 runs the pixel-pair sweep (each wave step two
 * pixels at 32 levels instead of one pixel at 64: half the epipolar span
 * per gather), 4 its four-pixel form (four pixels at 16 levels); they exist
 * for one label per lane, elsewhere the one-pixel sweep runs; 1 asks for
 * the one-pixel sweep, 0 picks the
 * default: four pixels where neighbouring levels land at least 3 px apart
 * (6 px with nearest sampling; FP64 mean over each view's image centre
 * projected into its targets), else two.  The sweeps compute the same quantity but add a segment's
 * pixels in different orders and, towards targets proven in front of every
 * level point, the multi-pixel sweeps form a sample's projection from H p~
 * divided by g . p~: their FP32 results may differ in the last bits, and a
 * sample within FP32 rounding of the bilinear validity band's edge may
 * count in one and not the other.  sweep_events, if both non-NULL, are hipEvent_t handles
 * the call records on its stream immediately before and after the sweep
 * kernel (for timing that kernel alone). */
typedef struct {
    int32_t sampling;         /* IVDE_NEAREST or IVDE_BILINEAR */
    int32_t cost_dtype;       /* IVDE_F32 or IVDE_F16 storage */
    int32_t targets;          /* IVDE_TARGETS_* */
    const uint8_t *target_mask;   /* host n x n, for IVDE_TARGETS_EXPLICIT */
    int32_t labels_per_lane;
    int32_t waves_per_group;
    void *sweep_events[2];
    int32_t pixels_per_step;  /* 0, 1, 2 or 4 */
} ivde_options;

/* ---------------------------------------------------------------- plain form */

/* Sizes of the cost volume and of the workspace ivde_cost_volume needs for
 * images of `bit_depth` bits.  The cost volume is [sum_c S_c][L] of float
 * or half, rows in view order then segment order, labels contiguous.
 * Either output pointer may be NULL.  Only sizes are read from cams and
 * segs (their device pointers are not touched). */
ivde_status ivde_cost_volume_size(int32_t n_views, const ivde_camera *cams,
                                  const ivde_segmentation *segs,
                                  const ivde_label_range *labels,
                                  const ivde_options *opt, int32_t bit_depth,
                                  size_t *cost_bytes, size_t *workspace_bytes);

/* The launch shape ivde_cost_volume takes for these arguments: labels per
 * lane, waves per workgroup and pixels per wave step (1: the one-pixel
 * sweep, 2 or 4: the multi-pixel sweep), from the options where they are set and
 * the defaults where they are 0.  Any output pointer may be NULL; arguments
 * are checked as for ivde_cost_volume_size.  Nothing is enqueued. */
ivde_status ivde_sweep_shape(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                             const ivde_label_range *labels, const ivde_options *opt, int32_t bit_depth,
                             int32_t *labels_per_lane, int32_t *waves_per_group, int32_t *pixels_per_step);

/* The cost volume C[view][segment][label] (Sec. III-C Eq. (4) over every
 * pixel of the segment, minimum over the target views).
 *   n_views     >= 1 views (a single view has no target: every row is 1.0)
 *   cams        host array of n_views cameras
 *   views       host array of n_views device images; all views share
 *               bit_depth and chroma_shift
 *   segs        host array of n_views device segment maps (W x H each)
 *   labels, opt host structs
 *   workspace   device buffer of at least the size ivde_cost_volume_size
 *               returns (256-byte aligned); it holds the packed images, the
 *               segment index and the task list until the stream completes
 *   cost_out    device buffer of cost_bytes
 * Returns IVDE_OK once every kernel is enqueued on `stream`. */
ivde_status ivde_cost_volume(int32_t n_views, const ivde_camera *cams,
                             const ivde_image *views, const ivde_segmentation *segs,
                             const ivde_label_range *labels, const ivde_options *opt,
                             void *workspace, size_t workspace_bytes,
                             void *cost_out, ivde_stream stream);

/* Winner-take-all labels: label_out[r] = the lowest l with
 * cost[r][l] == min_l cost[r][l] (NaN never wins).  cost is device
 * [rows][num_labels] of cost_dtype; label_out is device int32 [rows]. */
ivde_status ivde_argmin(int64_t rows, int32_t num_labels, int32_t cost_dtype,
                        const void *cost, int32_t *label_out, ivde_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): ivde_cost_volume
 * without a workspace argument.  The workspace lives in a fixed array of the
 * library in device memory, IVDE_NOALLOC_SCRATCH_BYTES (64 MiB) on every GPU
 * the library runs on, held until the process ends; the call allocates no
 * device memory.  Problems whose ivde_cost_volume_size workspace exceeds
 * that size are refused with IVDE_ENOMEM before anything is enqueued (for
 * example 3 views of 320 x 240 need about 10 MiB; 8 views of 1920 x 1080 do
 * not fit).  Every call on one GPU shares that GPU's array and leaves its
 * contents behind; each call clears what it needs with kernels on its own
 * stream, so calls on one GPU must not overlap (calls on different streams
 * that overlap in time race on the array).  Segment ids out of range are
 * skipped as in ivde_cost_volume but cannot be queried afterwards (there is
 * no workspace to pass to ivde_workspace_status).  Results are bitwise those
 * of ivde_cost_volume with the same arguments. */
#define IVDE_NOALLOC_SCRATCH_BYTES (64u << 20)
ivde_status ivde_cost_volume_noalloc(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                                     const ivde_segmentation *segs, const ivde_label_range *labels,
                                     const ivde_options *opt, void *cost_out, ivde_stream stream);

/* After the stream that ran ivde_cost_volume with this workspace has
 * completed: IVDE_EINVAL if a segment id was out of range, else IVDE_OK.
 * Synchronises `stream`. */
ivde_status ivde_workspace_status(const void *workspace, ivde_stream stream);

/* After the stream that ran ivde_cost_volume with this workspace has
 * completed: the wave steps its multi-pixel sweep took (one step = two
 * pixels of a segment towards one target at 32 levels, or four at 16), in total, on
 * records whose projection base was staged already divided by g . p~
 * (targets proven in front of every level point), and on chunks of records
 * whose every sample was shown to lie inside the bilinear validity band,
 * which run without per-sample validity tests.  All three are 0 after a
 * one-pixel sweep.  For performance accounting; synchronises `stream`. */
ivde_status ivde_workspace_sweep_steps(const void *workspace, ivde_stream stream, int64_t *steps_total,
                                       int64_t *steps_projected, int64_t *steps_inside);

/* ---------------------------------------------------------------- batched form */

/* One frame of a batch: the same fields as one ivde_cost_volume call. */
typedef struct {
    int32_t n_views;
    const ivde_camera *cams;
    const ivde_image *views;
    const ivde_segmentation *segs;
    ivde_label_range labels;
    void *cost_out;           /* device, ivde_cost_volume_size's cost_bytes */
    int32_t *label_out;       /* device int32 [rows] for argmin labels, or NULL */
} ivde_frame;

typedef struct ivde_batch ivde_batch;

/* Plans a batch of frames with uneven view, segment and label counts: one
 * persistent sweep kernel pulls (frame, view, segment, label-block) tasks,
 * sorted by cost, from a shared queue.  The plan records every device
 * pointer of `frames` and the workspace: they must stay valid while the
 * plan is used.  Frames must share sampling and cost dtype (opt). */
ivde_status ivde_batch_size(int32_t n_frames, const ivde_frame *frames, const ivde_options *opt,
                            size_t *workspace_bytes);
ivde_status ivde_batch_create(int32_t n_frames, const ivde_frame *frames, const ivde_options *opt,
                              void *workspace, size_t workspace_bytes, ivde_batch **out);
/* Runs the whole batch (image packing, segment index, task queue, one
 * persistent sweep, argmin for frames with label_out) on `stream`.
 * use_graph != 0 replays a hipGraph captured on first use (on that first
 * call the work is captured and then launched); the stream must not be the
 * null stream then.  The sweep_events of `opt` given to ivde_batch_create
 * bracket the persistent sweep in eager runs (use_graph == 0) only. */
ivde_status ivde_batch_run(ivde_batch *b, ivde_stream stream, int32_t use_graph);
void ivde_batch_destroy(ivde_batch *b);

/* ---------------------------------------------------------------- serving form */

typedef struct ivde_server ivde_server;

typedef struct {
    void *arena;              /* device memory; its size is the HBM budget */
    size_t arena_bytes;
    int32_t max_slots;        /* requests in flight on the device at once (1..16) */
    int32_t reserved;         /* must be 0 */
    int64_t chunk_evals;      /* a full-frame sweep runs as launches of about this many
                                 pixel-label-target evaluations, and the next launch is
                                 enqueued only while no other rig's uncut frame is in
                                 flight (or once its own rig's next frame is admitted), so
                                 short frames wait at most one launch behind a full one;
                                 0: 8e9 (about 8 ms on MI355X); < 0: one launch */
} ivde_server_config;

typedef struct {
    uint64_t ticket;
    int32_t rig_id;
    int32_t status;           /* IVDE_OK or the failure */
    int64_t rows_recomputed;  /* changed segments swept */
    int64_t rows_from_iframe; /* rule mode: unchanged rows that adopted the I frame's result */
    int64_t rows_total;
    double submit_us;         /* host steady-clock times, microseconds */
    double start_us;          /* admitted and enqueued */
    double done_us;           /* device work observed complete */
} ivde_frame_stats;

/* A serving loop (Sec. III-E temporal scheme as a service): rigs are
 * registered once, each keeps its previous frame's cost volume resident in
 * the arena, and every submitted frame recomputes only the segments its
 * changed mask marks, carrying the other rows over.  Requests are admitted
 * while a slot and arena memory are free, and run concurrently on separate
 * streams; frames of one rig run in submission order. */
ivde_status ivde_server_create(const ivde_server_config *cfg, ivde_server **out);

/* Arena bytes a rig holds while registered (resident: segment maps, the
 * rig's workspace sized for 16-bit images, two cost volumes, two mean-colour
 * tables) and one of its frames holds while admitted, for images of
 * bit_depth bits and the given chroma_shift: per_request for frames in
 * device memory, per_host_request for frames handed over in host memory
 * (plus the staged planes and mask).  An arena of resident + k per_request
 * bytes runs k of its frames at once.  Any output may be NULL. */
ivde_status ivde_server_footprint(int32_t n_views, const ivde_camera *cams,
                                  const ivde_segmentation *segs, const ivde_label_range *labels,
                                  const ivde_options *opt, int32_t bit_depth, int32_t chroma_shift,
                                  size_t *resident, size_t *per_request, size_t *per_host_request);

/* Registers a rig: its cameras, fixed segmentation (device maps, read
 * during this call only), label range and options.  Reserves the rig's
 * resident state in the arena; IVDE_EBUDGET if it does not fit. */
ivde_status ivde_rig_register(ivde_server *srv, int32_t n_views, const ivde_camera *cams,
                              const ivde_segmentation *segs, const ivde_label_range *labels,
                              const ivde_options *opt, int32_t *rig_id);

/* Submits one frame of a rig.
 *   views         host array of n_views device images, valid until done
 *   changed_mask  device uint8 [sum_c S_c] (non-zero = recompute the row)
 *                 or NULL: recompute every row (an I frame, Sec. III-E)
 *   cost_out      device, optional: receives a copy of the frame's cost
 *   label_out     device int32 [sum_c S_c], optional: argmin labels
 * IVDE_EBUDGET if the request can never fit the arena. */
ivde_status ivde_stream_submit(ivde_server *srv, int32_t rig_id, const ivde_image *views,
                               const uint8_t *changed_mask, void *cost_out, int32_t *label_out,
                               uint64_t *ticket);
/* Submits one frame whose changed segments the server decides itself by
 * the paper's temporal rule (Sec. III-E): with the frame's mean Y, Cb, Cr
 * per segment (same segment id under the rig's fixed segmentation), a row
 * adopts the latest I frame's result when every component moved by less
 * than t_i since that frame, else keeps the previous frame's row when every
 * component moved by less than t_p, else it is recomputed.  Thresholds are
 * in 8-bit code values (scaled by 2^(b-8)); defaults t_p = 3, t_i = 1.
 * iframe != 0 (or a rig without an I frame yet) recomputes every row and
 * makes this frame the I frame. */
ivde_status ivde_stream_submit_rule(ivde_server *srv, int32_t rig_id, const ivde_image *views,
                                    int32_t iframe, void *cost_out, int32_t *label_out,
                                    uint64_t *ticket);
ivde_status ivde_rig_set_temporal(ivde_server *srv, int32_t rig_id, float t_p, float t_i);

#define IVDE_SUBMIT_MASK 0          /* changed_mask decides; NULL: every row */
#define IVDE_SUBMIT_RULE 1          /* as ivde_stream_submit_rule, iframe = 0 */
#define IVDE_SUBMIT_RULE_IFRAME 2   /* as ivde_stream_submit_rule, iframe = 1 */

/* Submits one frame whose planes are in HOST memory, as camera frames
 * arrive: host_views[v].plane[i] are host pointers (pinned memory from
 * hipHostMalloc lets the copies run asynchronously; pageable memory is
 * accepted but its copies may block the server's scheduler), and in
 * IVDE_SUBMIT_MASK mode changed_mask is a host uint8 [sum_c S_c] array or
 * NULL (rule modes take NULL).  At admission the server copies the planes
 * and the mask into the request's working set on the request's own stream,
 * ahead of its kernels, so the upload overlaps the rig's previous frame and
 * is part of the frame's latency (submit_us to done_us).  The host buffers
 * must stay unchanged until the request completes.  Every view must have
 * the same bit depth and chroma format.  Otherwise as ivde_stream_submit
 * (cost_out and label_out are device memory). */
ivde_status ivde_stream_submit_host(ivde_server *srv, int32_t rig_id, const ivde_image *host_views,
                                    int32_t mode, const uint8_t *changed_mask, void *cost_out,
                                    int32_t *label_out, uint64_t *ticket);
/* IVDE_EBUSY while pending; otherwise fills `st` and forgets the ticket. */
ivde_status ivde_stream_poll(ivde_server *srv, uint64_t ticket, ivde_frame_stats *st);
ivde_status ivde_stream_wait(ivde_server *srv, uint64_t ticket, ivde_frame_stats *st);
/* Device pointer of a rig's resident cost volume (valid until destroy). */
ivde_status ivde_rig_resident(ivde_server *srv, int32_t rig_id, const void **cost, int64_t *rows);
/* Drops a rig's resident volume: its next frame is computed in full. */
ivde_status ivde_rig_reset(ivde_server *srv, int32_t rig_id);
void ivde_server_destroy(ivde_server *srv);

/* ---------------------------------------------------------------- the paper's window term */

/* Output and workspace sizes of ivde_window_cost (out_bytes is the size of
 * each of m_out and hit_out). */
ivde_status ivde_window_cost_size(int32_t n_views, const ivde_camera *cams,
                                  const ivde_segmentation *segs,
                                  const ivde_label_range *labels, int32_t bit_depth,
                                  size_t *out_bytes, size_t *workspace_bytes);

/* The paper's inter-view matching core as printed (Sec. III-C, Eq. (4)):
 * for every segment s of view c, each neighbouring view c' of Sec. III-B
 * (slot 0: c - 1, slot 1: c + 1; views ordered along the rig) and each
 * label l, the centre mu_s of s (the centroid of its pixels rounded half
 * up) is lifted to level l and transformed into c'; the target window is
 * centred on the nearest pixel of the projection.
 *   m_out    device float [rows][2][L]: mean over the (2 radius + 1)^2 taps
 *            of |dY| + |dCb| + |dCr| in 8-bit code values (taps outside an
 *            image are clamped to its edge); NaN where c' does not exist or
 *            the projection is behind a camera or outside c'
 *   hit_out  device int32 [rows][2][L]: the segment s' of c' under the
 *            projected centre, as its row of the volume (row offset of c'
 *            plus its id), or -1 where m is NaN
 * Rows are ordered as in ivde_cost_volume.  radius 0..8 (the paper uses a
 * 3x3 window, radius 1, Sec. V-A). */
ivde_status ivde_window_cost(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                             const ivde_segmentation *segs, const ivde_label_range *labels,
                             int32_t radius, void *workspace, size_t workspace_bytes,
                             float *m_out, int32_t *hit_out, ivde_stream stream);

/* Eq. (5) summed over the neighbouring views for a fixed labelling d of
 * all rows (device int32 [rows]):
 *   out[r][l] = sum over slots with hit >= 0 of [d[hit] == l] min(0, m - K)
 * m and hit as written by ivde_window_cost; the paper uses K = 30. */
ivde_status ivde_window_energy(int64_t rows, int32_t num_labels, const float *m,
                               const int32_t *hit, const int32_t *labelling, float K,
                               float *out, ivde_stream stream);

/* ---------------------------------------------------------------- segment statistics, temporal rule */

ivde_status ivde_segment_stats_size(int32_t n_views, const ivde_camera *cams,
                                    const ivde_segmentation *segs, int32_t bit_depth,
                                    size_t *workspace_bytes);
/* Per segment, rows ordered as in ivde_cost_volume: pixel count
 * (device int32 [rows]), centre (the centroid rounded half up, Sec. III-C's
 * mu_s; int32 [rows][2], -1 for an empty segment) and mean colour (float
 * [rows][4]: Y, Cb, Cr, 0; Sec. III-D and III-E).  Any output may be NULL. */
ivde_status ivde_segment_stats(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                               const ivde_segmentation *segs, void *workspace,
                               size_t workspace_bytes, int32_t *count_out, int32_t *centre_out,
                               float *mean_out, ivde_stream stream);
/* The temporal rule of Sec. III-E on mean colours ([rows][4] as above):
 * source_out[r] = 2 when every component moved by less than t_i against
 * mean_iframe (skipped if NULL), else 1 when by less than t_p against
 * mean_prev, else 0 (recompute).  Thresholds in 8-bit code values. */
ivde_status ivde_temporal_rule(int64_t rows, const float *mean, const float *mean_prev,
                               const float *mean_iframe, float t_p, float t_i, int32_t bit_depth,
                               uint8_t *source_out, ivde_stream stream);

/* ---------------------------------------------------------------- intra-view term */

/* Workspace bytes for ivde_adjacency (segment index and statistics). */
ivde_status ivde_adjacency_size(int32_t n_views, const ivde_camera *cams,
                                const ivde_segmentation *segs, int32_t bit_depth,
                                size_t *workspace_bytes);
/* T(s) of Sec. III-D with the weights of Eq. (3).  Two segments of one view
 * are adjacent when a pixel of one is a 4-neighbour (left, right, above,
 * below) of a pixel of the other.  Outputs, device memory, rows ordered as in
 * ivde_cost_volume:
 *   offsets  int64 [rows + 1]: CSR offsets; offsets[rows] is the total number
 *            of entries (every adjacent pair appears once in each list)
 *   index    int32 [capacity]: neighbour rows, increasing within each row
 *   beta     float [capacity]: beta0 / (||mean_s - mean_t||_1 + eps), mean
 *            Y, Cb, Cr differences in 8-bit code values (divided by
 *            2^(bit_depth - 8)); eps > 0 keeps equal colours finite (Eq. (3)
 *            alone divides by zero there; 1 is the customary choice)
 * Entries at or beyond `capacity` are not written: call with capacity 0
 * (index and beta may then be NULL) to learn offsets[rows], or pass a bound.
 * Segment ids outside [0, num_segments) are ignored and reported by
 * ivde_workspace_status. */
ivde_status ivde_adjacency(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                           const ivde_segmentation *segs, float beta0, float eps, void *workspace,
                           size_t workspace_bytes, int64_t *offsets, int32_t *index, float *beta,
                           int64_t capacity, ivde_stream stream);
/* Eq. (2) seen from each segment with its neighbours' depths held:
 *   out[r][l] = sum over CSR entries (r, t) of beta * |l - labelling[t]|
 * depths in label units; with a mask (device uint8 [rows], NULL = all),
 * only neighbours t with fixed[t] != 0 count -- segments kept out of the
 * optimisation enter their neighbours' costs this way (Sec. III-E).
 * offsets, index, beta as written by ivde_adjacency; labelling int32 [rows];
 * out float [rows][num_labels].  Entries whose row is outside [0, rows) are
 * skipped. */
ivde_status ivde_intra_cost(int64_t rows, int32_t num_labels, const int64_t *offsets,
                            const int32_t *index, const float *beta, const int32_t *labelling,
                            const uint8_t *fixed, float *out, ivde_stream stream);

/* ---------------------------------------------------------------- depth maps */

/* Per-pixel depth maps from segment levels (Sec. III-B: a segment's depth
 * is painted onto its pixels).  label_of_row: device int32 [rows] (rows
 * ordered as in ivde_cost_volume); depth_out: device float, the views one
 * after another, each W x H in rows of W.  A pixel gets the depth of its
 * segment's level, 1 / (1/z_far + l/(L-1) (1/z_near - 1/z_far)), formed in
 * FP64 on the host and stored as FP32, or NaN for a segment id or level out
 * of range.  workspace: device memory of at least 4 * num_labels bytes,
 * 4-byte aligned, that receives the level-depth table (in use until the
 * stream completes).  Only sizes are read from cams. */
ivde_status ivde_depth_map(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                           const ivde_label_range *labels, const int32_t *label_of_row, void *workspace,
                           size_t workspace_bytes, float *depth_out, ivde_stream stream);

/* ---------------------------------------------------------------- depth optimisation (host) */

/* Eq. (1) over segment nodes, in host memory.  With d the label of every
 * row and q(x) = x * quantum rounded half away from zero:
 *   E(d) = sum_r q(unary_weight * unary[r][d_r])
 *        + sum_r sum_slot [h >= 0 and d_h = d_r] q(min(0, m - K)),
 *              m = window_m[r][slot][d_r], h = window_hit[r][slot][d_r]  (Eq. (5))
 *        + sum over adjacency entries (r, t) of q(beta) |d_r - d_t|       (Eq. (2))
 * Integer terms make every maximum flow exact.  Any term group may be
 * absent (NULL).  window_m / window_hit are ivde_window_cost's outputs,
 * adj_* ivde_adjacency's (both copied to the host).  fixed_labels, if
 * given, holds for each row -1 (a free segment) or the label of a segment
 * that is not a node (Sec. III-E: it keeps that label and enters the
 * costs of the others).  The pointers are read during the call only. */
typedef struct ivde_energy {
    int64_t rows;
    int32_t num_labels;
    const float *unary;            /* [rows][num_labels] or NULL */
    double unary_weight;           /* multiplies unary before rounding */
    const float *window_m;         /* [rows][2][num_labels] or NULL */
    const int32_t *window_hit;     /* [rows][2][num_labels], -1 = no match; with window_m */
    float K;                       /* Eq. (5) truncation; the paper uses 30 */
    const int64_t *adj_offsets;    /* [rows + 1] or NULL */
    const int32_t *adj_index;      /* [adj_offsets[rows]] rows */
    const float *adj_beta;         /* [adj_offsets[rows]], >= 0 */
    const int32_t *fixed_labels;   /* [rows] or NULL */
    double quantum;                /* > 0 */
} ivde_energy;

#define IVDE_PARTITION_BLOCKS 0        /* thread k takes levels [k L / n, (k + 1) L / n) */
#define IVDE_PARTITION_INTERLEAVED 1   /* thread k takes levels l with l mod n = k */

/* E(labels) as defined above. */
ivde_status ivde_energy_value(const ivde_energy *energy, const int32_t *labels, int64_t *energy_out);

/* Alpha-expansion from `labels` (updated in place) over the listed levels,
 * in increasing order, in cycles until one changes nothing or max_cycles
 * have run (graph cuts, Sec. III-B).  Each move takes the minimum cut
 * whose source side (segments keeping their label) is smallest, i.e. the
 * nodes reachable from the source in the residual graph; a move is kept
 * when it lowers E.  Fixed rows must carry their fixed label. */
ivde_status ivde_expansion(const ivde_energy *energy, int32_t *labels, const int32_t *label_list,
                           int32_t n_list, int32_t max_cycles, int64_t *energy_out,
                           int32_t *cycles_out);

/* The label-partitioned estimation of Sec. IV-A: n_threads host threads
 * each run ivde_expansion over their subset of the levels (IVDE_PARTITION_*),
 * starting from each row's lowest-unary level of the subset; then results
 * merge pairwise (k with k + 2^c in cycle c, ceil(log2 n) cycles), each merge
 * an expansion over both subsets in which a row may only take one of its
 * two candidate labels, starting from the lower-energy input.  The result
 * does not depend on thread timing.  labels_out: host int32 [rows]. */
ivde_status ivde_optimize(const ivde_energy *energy, int32_t n_threads, int32_t partition,
                          int32_t max_cycles, int32_t *labels_out, int64_t *energy_out);

/* ---------------------------------------------------------------- tuning */

/* Times every (labels_per_lane, waves_per_group, pixels_per_step) launch
 * shape on the given problem (which must already be valid for
 * ivde_cost_volume) and writes the fastest into *opt_out.  The 18
 * candidates, in order: labels per lane 1, 2, 4, 8 x waves per group 1, 2, 4
 * with one pixel per step, then one label per lane x waves per group 1, 2, 4
 * with two and then four pixels per step (skipped, time -1, where those
 * sweeps do not exist).
 * Each candidate runs `reps` times; times in microseconds go to times_us[i]
 * for candidate i if not NULL (capacity max_times).  Synchronises `stream`. */
ivde_status ivde_autotune(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                          const ivde_segmentation *segs, const ivde_label_range *labels,
                          const ivde_options *opt, void *workspace, size_t workspace_bytes,
                          void *cost_out, ivde_stream stream, int32_t reps,
                          ivde_options *opt_out, float *times_us, int32_t max_times);

/* ---------------------------------------------------------------- misc */

const char *ivde_status_string(ivde_status s);
const char *ivde_last_error(void);     /* thread-local, "" if none */
const char *ivde_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IVDE_H */
