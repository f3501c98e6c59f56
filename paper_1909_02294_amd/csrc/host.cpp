// libivde host side: argument validation, FP64 camera composition, workspace
// layout and the plain cost-volume / argmin entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/ivde.h"
#include "host_common.h"
#include "ivde_internal.h"

namespace ivde {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

const char *last_error() { return g_err; }

ivde_status hip_fail(hipError_t e, const char *what)
{
    set_error("%s: %s", what, hipGetErrorString(e));
    return IVDE_EHIP;
}

// ---------------------------------------------------------------- FP64 helpers
static bool inv3(const double *a, double *o)
{
    const double c00 = a[4] * a[8] - a[5] * a[7];
    const double c01 = a[5] * a[6] - a[3] * a[8];
    const double c02 = a[3] * a[7] - a[4] * a[6];
    const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    if (!(std::fabs(det) > 0.0) || !std::isfinite(det)) return false;
    const double r = 1.0 / det;
    o[0] = c00 * r;
    o[1] = (a[2] * a[7] - a[1] * a[8]) * r;
    o[2] = (a[1] * a[5] - a[2] * a[4]) * r;
    o[3] = c01 * r;
    o[4] = (a[0] * a[8] - a[2] * a[6]) * r;
    o[5] = (a[2] * a[3] - a[0] * a[5]) * r;
    o[6] = c02 * r;
    o[7] = (a[1] * a[6] - a[0] * a[7]) * r;
    o[8] = (a[0] * a[4] - a[1] * a[3]) * r;
    return true;
}

static void mul3(const double *a, const double *b, double *o)   // o = a b
{
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
    memcpy(o, t, sizeof(t));
}

static void transpose3(const double *a, double *o)
{
    double t[9] = {a[0], a[3], a[6], a[1], a[4], a[7], a[2], a[5], a[8]};
    memcpy(o, t, sizeof(t));
}

static void mv3(const double *a, const double *v, double *o)
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = a[3 * i] * v[0] + a[3 * i + 1] * v[1] + a[3 * i + 2] * v[2];
    memcpy(o, t, sizeof(t));
}

// ---------------------------------------------------------------- validation
ivde_status validate_problem(int32_t n, const ivde_camera *cams, const ivde_image *views,
                             const ivde_segmentation *segs, const ivde_label_range *labels,
                             const ivde_options *opt, bool need_images)
{
    if (n < 1 || n > kMaxViews) {
        set_error("n_views must be in [1, %d], got %d", kMaxViews, n);
        return IVDE_EINVAL;
    }
    if (!cams || !segs || !labels || !opt || (need_images && !views)) {
        set_error("null argument");
        return IVDE_EINVAL;
    }
    for (int v = 0; v < n; ++v) {
        const ivde_camera &c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384) {
            set_error("view %d: image size %dx%d outside [1, 16384]", v, c.width, c.height);
            return IVDE_EINVAL;
        }
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(c.K[i]) || !std::isfinite(c.R[i])) {
                set_error("view %d: non-finite camera matrix", v);
                return IVDE_EINVAL;
            }
        for (int i = 0; i < 3; ++i)
            if (!std::isfinite(c.t[i])) {
                set_error("view %d: non-finite translation", v);
                return IVDE_EINVAL;
            }
        if (c.K[6] != 0.0 || c.K[7] != 0.0 || c.K[8] != 1.0) {
            set_error("view %d: K must have third row (0, 0, 1)", v);
            return IVDE_EINVAL;
        }
        double ki[9];
        if (!inv3(c.K, ki)) {
            set_error("view %d: singular K", v);
            return IVDE_EINVAL;
        }
        const ivde_segmentation &s = segs[v];
        if (!s.seg_map || s.num_segments < 1 || s.pitch < c.width) {
            set_error("view %d: segmentation needs a map, num_segments >= 1 and pitch >= width", v);
            return IVDE_EINVAL;
        }
        if ((int64_t)c.width * c.height > (int64_t)1 << 28) {
            set_error("view %d: too many pixels", v);
            return IVDE_EINVAL;
        }
    }
    if (need_images) {
        const int b = views[0].bit_depth, k = views[0].chroma_shift;
        if (b < 8 || b > 16 || k < 0 || k > 1) {
            set_error("bit_depth must be 8..16 and chroma_shift 0 or 1");
            return IVDE_EINVAL;
        }
        for (int v = 0; v < n; ++v) {
            const ivde_image &im = views[v];
            if (im.bit_depth != b || im.chroma_shift != k) {
                set_error("view %d: all views must share bit_depth and chroma_shift", v);
                return IVDE_EINVAL;
            }
            const int64_t cw = (cams[v].width + k) >> k;
            for (int p = 0; p < 3; ++p)
                if (!im.plane[p] || im.pitch[p] < (p ? cw : cams[v].width)) {
                    set_error("view %d: plane %d is null or its pitch is too small", v, p);
                    return IVDE_EINVAL;
                }
        }
    }
    const ivde_label_range &lr = *labels;
    if (!(lr.z_near > 0.0) || !(lr.z_far > 0.0) || !std::isfinite(lr.z_near) || !std::isfinite(lr.z_far)) {
        set_error("z_near and z_far must be finite and positive");
        return IVDE_EINVAL;
    }
    if (lr.num_labels < 1 || lr.num_labels > 8192) {
        set_error("num_labels must be in [1, 8192]");
        return IVDE_EINVAL;
    }
    if (lr.depth_ref < IVDE_REF_OWN || lr.depth_ref >= n) {
        set_error("depth_ref must be IVDE_REF_RIG_CENTER, IVDE_REF_OWN or a view index");
        return IVDE_EINVAL;
    }
    if (opt->sampling != IVDE_NEAREST && opt->sampling != IVDE_BILINEAR) {
        set_error("unknown sampling %d", opt->sampling);
        return IVDE_EINVAL;
    }
    if (opt->cost_dtype != IVDE_F32 && opt->cost_dtype != IVDE_F16) {
        set_error("unknown cost dtype %d", opt->cost_dtype);
        return IVDE_EINVAL;
    }
    if (opt->targets < IVDE_TARGETS_ALL || opt->targets > IVDE_TARGETS_EXPLICIT ||
        (opt->targets == IVDE_TARGETS_EXPLICIT && !opt->target_mask)) {
        set_error("bad target selection");
        return IVDE_EINVAL;
    }
    const int J = opt->labels_per_lane;
    if (J != 0 && J != 1 && J != 2 && J != 4 && J != 8) {
        set_error("labels_per_lane must be 0, 1, 2, 4 or 8");
        return IVDE_EINVAL;
    }
    const int w = opt->waves_per_group;
    if (w != 0 && w != 1 && w != 2 && w != 4) {
        set_error("waves_per_group must be 0, 1, 2 or 4");
        return IVDE_EINVAL;
    }
    if (opt->pixels_per_step < 0 || opt->pixels_per_step > 4 || opt->pixels_per_step == 3) {
        set_error("pixels_per_step must be 0, 1, 2 or 4");
        return IVDE_EINVAL;
    }
    return IVDE_OK;
}

// One label per lane (64-label tasks) measured fastest on the 8-view 1080p
// workload: the sweep waits on gathers, and small tasks keep more waves
// resident to hide that latency.
int default_labels_per_lane(int L)
{
    (void)L;
    return 1;
}

// ---------------------------------------------------------------- layout

// Mean distance in pixels between neighbouring levels, at each view's image
// centre projected into each of its targets (FP64; pairs where either end
// lies behind a camera are left out).
static double level_step_px(int32_t n, const ivde_camera *cams, const ivde_label_range *labels,
                            const ivde_options *opt)
{
    const int L = labels->num_labels;
    if (L < 2 || n < 2) return 0.0;
    std::vector<double> M(9 * n), C(3 * n), axis(3 * n);
    for (int v = 0; v < n; ++v) {
        double Kinv[9], Rt[9], c[3];
        inv3(cams[v].K, Kinv);
        transpose3(cams[v].R, Rt);
        mul3(Rt, Kinv, &M[9 * v]);
        mv3(Rt, cams[v].t, c);
        for (int i = 0; i < 3; ++i) {
            C[3 * v + i] = -c[i];
            axis[3 * v + i] = cams[v].R[6 + i];
        }
    }
    double cm[3] = {0, 0, 0}, am[3] = {0, 0, 0};
    for (int u = 0; u < n; ++u)
        for (int i = 0; i < 3; ++i) {
            cm[i] += C[3 * u + i] / n;
            am[i] += axis[3 * u + i] / n;
        }
    const double alen = std::sqrt(am[0] * am[0] + am[1] * am[1] + am[2] * am[2]);
    double sum = 0.0;
    int cnt = 0;
    for (int v = 0; v < n; ++v) {
        double Cr[3], nr[3];
        const int rv = labels->depth_ref == IVDE_REF_RIG_CENTER ? -1
                       : labels->depth_ref == IVDE_REF_OWN  ? v
                                                             : labels->depth_ref;
        for (int i = 0; i < 3; ++i) {
            Cr[i] = rv < 0 ? cm[i] : C[3 * rv + i];
            nr[i] = rv < 0 ? (alen > 0.0 ? am[i] / alen : 0.0) : axis[3 * rv + i];
        }
        const double p[3] = {0.5 * (cams[v].width - 1), 0.5 * (cams[v].height - 1), 1.0};
        double d[3];
        mv3(&M[9 * v], p, d);
        const double nd = nr[0] * d[0] + nr[1] * d[1] + nr[2] * d[2];
        const double delta = nr[0] * (C[3 * v] - Cr[0]) + nr[1] * (C[3 * v + 1] - Cr[1]) + nr[2] * (C[3 * v + 2] - Cr[2]);
        if (!(std::fabs(nd) > 0.0)) continue;
        double X[2][3];
        const double z[2] = {labels->z_far, labels->z_near};
        for (int k = 0; k < 2; ++k) {
            const double tau = (z[k] - delta) / nd;
            for (int i = 0; i < 3; ++i) X[k][i] = C[3 * v + i] + tau * d[i];
        }
        for (int c2 = 0; c2 < n; ++c2) {
            if (c2 == v) continue;
            if (opt->targets == IVDE_TARGETS_NEAREST_LR && c2 != v - 1 && c2 != v + 1) continue;
            if (opt->targets == IVDE_TARGETS_EXPLICIT && !opt->target_mask[v * n + c2]) continue;
            double uv[2][2];
            bool ok = true;
            for (int k = 0; k < 2; ++k) {
                double xc[3], h[3];
                mv3(cams[c2].R, X[k], xc);
                for (int i = 0; i < 3; ++i) xc[i] += cams[c2].t[i];
                mv3(cams[c2].K, xc, h);
                ok &= h[2] > 0.0;
                uv[k][0] = h[0] / h[2];
                uv[k][1] = h[1] / h[2];
            }
            if (!ok) continue;
            sum += std::hypot(uv[1][0] - uv[0][0], uv[1][1] - uv[0][1]);
            cnt += 1;
        }
    }
    return cnt ? sum / cnt / (L - 1) : 0.0;
}

// Pixels per wave step of the sweep (one label per lane; the one-pixel sweep
// elsewhere).  Two pixels at 32 levels per step (pairs) or
// four at 16 (quads) shorten the epipolar stretch every gather spans; towards
// targets proven in front of every level point each sample's projection is
// three multiply-adds on a staged record.  On the 8-view 1080p arc rig
// (5,000 to 40,000 segments per view) pairs beat the one-pixel sweep at
// every level count (64: 14.7-15.8 against 23.7-30.1 ms; 256: 28.2-28.6
// against 31.1-32.8 ms), and quads beat pairs where neighbouring levels
// land far apart (64 levels, 8 px: 11.7-11.9 against 14.7-15.8 ms; 128
// levels, 4 px: 16.7-17.7 against 17.9-18.7 ms) but lose where they land
// close (256 levels, 2 px: 28.8-31.2 against 28.2-28.6 ms; 512 levels:
// 54.4-59.6 against 53.7-54.4 ms): each pass then has four times the
// groups' ragged tails and a quarter of the levels.  So: quads from 3 px
// between neighbouring levels at the image centres, pairs below.  Nearest
// sampling reads one texel per sample instead of four, so the shorter
// stretch pays only further apart: on the same rig (20,000 segments) pairs
// took 10.5 against 11.3 ms at 128 levels (4 px) and quads 6.6 against 7.4
// ms at 64 (8 px); there quads start at 6 px.
static int choose_px(int32_t n, const ivde_camera *cams, const ivde_label_range *labels, const ivde_options *opt,
                     int J)
{
    if (J != 1) return 1;
    if (opt->pixels_per_step) return opt->pixels_per_step;
    const double quads_from = opt->sampling == IVDE_NEAREST ? 6.0 : 3.0;
    return level_step_px(n, cams, labels, opt) >= quads_from ? 4 : 2;
}

Layout plan_layout(int32_t n, const ivde_camera *cams, const ivde_segmentation *segs, const ivde_label_range *labels,
                   const ivde_options *opt, int bit_depth)
{
    Layout ly{};
    ly.n = n;
    ly.L = labels->num_labels;
    ly.J = opt->labels_per_lane ? opt->labels_per_lane : default_labels_per_lane(ly.L);
    ly.wpg = opt->waves_per_group ? opt->waves_per_group : 4;
    ly.n_lblocks = (ly.L + 64 * ly.J - 1) / (64 * ly.J);
    ly.tex_u16 = bit_depth > 11;
    ly.px = choose_px(n, cams, labels, opt, ly.J);
    ly.f16 = opt->cost_dtype == IVDE_F16;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    ly.off_problem = take(sizeof(Problem));
    ly.off_views = take(sizeof(ViewDesc) * n);
    ly.off_pairs = take(sizeof(PairConst) * n * n);
    ly.off_sigma = take(sizeof(float) * n * ly.L);
    ly.off_flag = take(kFlagWords * sizeof(int32_t));   // error flag, then 3 x 64-bit sweep step counts
    ly.total_rows = 0;
    ly.max_w = ly.max_h = ly.max_s = ly.max_bands = 0;
    for (int v = 0; v < n; ++v) {
        const int W = cams[v].width, H = cams[v].height, S = segs[v].num_segments;
        ViewLayout &vl = ly.views[v];
        vl.row0 = ly.total_rows;
        ly.total_rows += S;
        vl.n_bands = (H + kBand - 1) / kBand;
        vl.tex_bytes = (int64_t)(W + 2) * (H + 2) * 8;
        vl.off_tex = take((size_t)vl.tex_bytes + 16);
        vl.off_counts = take(sizeof(int32_t) * S);
        vl.off_offsets = take(sizeof(int32_t) * (S + 1));
        vl.off_bbox = take(sizeof(int32_t) * 4 * S);
        vl.off_pixrec = take(sizeof(float) * 8 * (size_t)W * H);
        vl.off_bands = take(sizeof(int32_t) * 2 * vl.n_bands);
        ly.max_w = W > ly.max_w ? W : ly.max_w;
        ly.max_h = H > ly.max_h ? H : ly.max_h;
        ly.max_s = S > ly.max_s ? S : ly.max_s;
        ly.max_bands = vl.n_bands > ly.max_bands ? vl.n_bands : ly.max_bands;
    }
    ly.n_tasks = ly.total_rows * ly.n_lblocks;
    ly.off_tasks = take(sizeof(Task) * (size_t)ly.n_tasks);
    ly.off_centre = take(sizeof(int32_t) * 2 * (size_t)ly.total_rows);
    ly.off_mean = take(sizeof(float) * 4 * (size_t)ly.total_rows);
    ly.off_sums = take(sizeof(uint64_t) * 6 * (size_t)ly.total_rows);
    ly.off_cursors = take(sizeof(int32_t) * (kXcds + 1));
    ly.workspace_bytes = off;
    ly.cost_bytes = (size_t)ly.total_rows * ly.L * (ly.f16 ? 2 : 4);
    return ly;
}

// ---------------------------------------------------------------- composition
// Builds the host image of the device constants: per-view descriptors, the
// pair projections (h = H p~ + sigma (g . p~) e) and the sigma table, all
// composed in FP64 and cast to FP32.
ivde_status compose(int32_t n, const ivde_camera *cams, const ivde_image *views, const ivde_segmentation *segs,
                    const ivde_label_range *labels, const ivde_options *opt, const Layout &ly, char *ws_base,
                    void *cost_out, HostConstants &hc)
{
    const int L = ly.L;
    hc.views.assign(n, ViewDesc{});
    hc.pairs.assign((size_t)n * n, PairConst{});
    hc.sigma.assign((size_t)n * L, 0.f);

    std::vector<double> Kinv(9 * n), M(9 * n), C(3 * n), axis(3 * n);
    for (int v = 0; v < n; ++v) {
        inv3(cams[v].K, &Kinv[9 * v]);
        double Rt[9];
        transpose3(cams[v].R, Rt);
        mul3(Rt, &Kinv[9 * v], &M[9 * v]);            // ray direction d = M p~
        double c[3];
        mv3(Rt, cams[v].t, c);
        for (int i = 0; i < 3; ++i) {
            C[3 * v + i] = -c[i];
            axis[3 * v + i] = cams[v].R[6 + i];
        }
    }
    // reference plane(s): normal n_r through C_r
    std::vector<double> Cr(3 * n), nr(3 * n);
    for (int v = 0; v < n; ++v) {
        if (labels->depth_ref == IVDE_REF_RIG_CENTER) {
            double cm[3] = {0, 0, 0}, am[3] = {0, 0, 0};
            for (int u = 0; u < n; ++u)
                for (int i = 0; i < 3; ++i) {
                    cm[i] += C[3 * u + i] / n;
                    am[i] += axis[3 * u + i] / n;
                }
            const double len = std::sqrt(am[0] * am[0] + am[1] * am[1] + am[2] * am[2]);
            if (!(len > 0.0)) {
                set_error("the mean optical axis of the rig vanishes");
                return IVDE_EINVAL;
            }
            for (int i = 0; i < 3; ++i) {
                Cr[3 * v + i] = cm[i];
                nr[3 * v + i] = am[i] / len;
            }
        } else {
            const int rv = labels->depth_ref == IVDE_REF_OWN ? v : labels->depth_ref;
            for (int i = 0; i < 3; ++i) {
                Cr[3 * v + i] = C[3 * rv + i];
                nr[3 * v + i] = axis[3 * rv + i];
            }
        }
    }
    std::vector<double> zl(L);
    for (int l = 0; l < L; ++l) {
        const double f = L > 1 ? (double)l / (double)(L - 1) : 0.0;
        const double rho = 1.0 / labels->z_far + f * (1.0 / labels->z_near - 1.0 / labels->z_far);
        zl[l] = 1.0 / rho;
    }
    // target sets
    std::vector<uint8_t> T((size_t)n * n, 0);
    for (int c = 0; c < n; ++c)
        for (int c2 = 0; c2 < n; ++c2) {
            if (c2 == c) continue;
            if (opt->targets == IVDE_TARGETS_ALL) T[c * n + c2] = 1;
            else if (opt->targets == IVDE_TARGETS_NEAREST_LR) T[c * n + c2] = (c2 == c - 1 || c2 == c + 1);
            else T[c * n + c2] = opt->target_mask[c * n + c2] != 0;
        }

    for (int v = 0; v < n; ++v) {
        ViewDesc &d = hc.views[v];
        const ViewLayout &vl = ly.views[v];
        for (int p = 0; p < 3; ++p) {
            d.plane[p] = views ? views[v].plane[p] : nullptr;
            d.pitch[p] = views ? views[v].pitch[p] : 0;
        }
        d.seg = segs[v].seg_map;
        d.seg_pitch = segs[v].pitch;
        d.tex = ws_base + vl.off_tex;
        d.tex_bytes = vl.tex_bytes;
        d.W = cams[v].width;
        d.H = cams[v].height;
        d.tex_pitch = cams[v].width + 2;
        d.S = segs[v].num_segments;
        d.row0 = vl.row0;
        d.counts = reinterpret_cast<int32_t *>(ws_base + vl.off_counts);
        d.offsets = reinterpret_cast<int32_t *>(ws_base + vl.off_offsets);
        d.bbox = reinterpret_cast<int32_t *>(ws_base + vl.off_bbox);
        d.pixrec = reinterpret_cast<float *>(ws_base + vl.off_pixrec);
        d.band_count = reinterpret_cast<int32_t *>(ws_base + vl.off_bands);
        d.centre = reinterpret_cast<int32_t *>(ws_base + ly.off_centre) + 2 * vl.row0;
        d.mean = reinterpret_cast<float *>(ws_base + ly.off_mean) + 4 * vl.row0;
        d.n_bands = vl.n_bands;
        d.n_targets = 0;
        for (int c2 = 0; c2 < n; ++c2)
            if (T[v * n + c2]) d.targets[d.n_targets++] = c2;
        // g_c = M_c^T n_r, so g . p~ = n_r . (M_c p~) = n_r . d
        const double *Mv = &M[9 * v], *nv = &nr[3 * v];
        for (int i = 0; i < 3; ++i) d.g[i] = (float)(Mv[i] * nv[0] + Mv[3 + i] * nv[1] + Mv[6 + i] * nv[2]);
        d.g[3] = 0.f;
        const double delta = nv[0] * (C[3 * v] - Cr[3 * v]) + nv[1] * (C[3 * v + 1] - Cr[3 * v + 1]) +
                             nv[2] * (C[3 * v + 2] - Cr[3 * v + 2]);
        bool sig_pos = true;
        for (int l = 0; l < L; ++l) {
            const double den = zl[l] - delta;
            const double sg = den != 0.0 ? 1.0 / den : 0.0;
            hc.sigma[(size_t)v * L + l] = std::isfinite(sg) ? (float)sg : 0.f;
            sig_pos &= std::isfinite(sg) && (float)sg > 0.f;
        }
        // g . p~ is affine in the pixel: its minimum over the image is at a
        // corner.  With a margin for the FP32 evaluation, g . p~ > 0 and
        // sigma > 0 everywhere mean every 3-D point is in front of camera v.
        double gmin = INFINITY, gmax = 0.0;
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const double x = cx ? cams[v].width - 1 : 0, y = cy ? cams[v].height - 1 : 0;
                const double gpv = (Mv[0] * nv[0] + Mv[3] * nv[1] + Mv[6] * nv[2]) * x +
                                   (Mv[1] * nv[0] + Mv[4] * nv[1] + Mv[7] * nv[2]) * y +
                                   (Mv[2] * nv[0] + Mv[5] * nv[1] + Mv[8] * nv[2]);
                gmin = std::fmin(gmin, gpv);
                gmax = std::fmax(gmax, std::fabs(gpv));
            }
        d.front_all = sig_pos && gmin > 1e-4 * gmax;
        // With every point in front of camera v, the points of view v at all
        // labels fill the part of its viewing frustum (the rays through the
        // image rectangle) between the nearest and the farthest level plane: a
        // convex solid whose corners are the four corner rays at those two
        // planes.  Depth in a target camera is affine in the point, so when all
        // eight corners lie in front of the target (with a margin for the FP32
        // evaluation), every point does and the sweep needs no depth test for
        // that target.
        d.front_targets = 0;
        if (d.front_all) {
            double zmin = INFINITY, zmax = 0.0;
            for (int l = 0; l < L; ++l) {
                zmin = std::fmin(zmin, zl[l]);
                zmax = std::fmax(zmax, zl[l]);
            }
            double corner[8][3];
            int k = 0;
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    const double p[3] = {cx ? cams[v].width - 1.0 : 0.0, cy ? cams[v].height - 1.0 : 0.0, 1.0};
                    double dir[3];
                    mv3(Mv, p, dir);
                    const double nd = nv[0] * dir[0] + nv[1] * dir[1] + nv[2] * dir[2];
                    for (int zi = 0; zi < 2; ++zi, ++k) {
                        const double tau = ((zi ? zmax : zmin) - delta) / nd;
                        for (int i = 0; i < 3; ++i) corner[k][i] = C[3 * v + i] + tau * dir[i];
                    }
                }
            for (int c2 = 0; c2 < n; ++c2) {
                if (c2 == v) continue;
                double dmin = INFINITY, dmax = 0.0;
                for (int q = 0; q < 8; ++q) {
                    double xc[3];
                    mv3(cams[c2].R, corner[q], xc);
                    const double depth = xc[2] + cams[c2].t[2];
                    dmin = std::fmin(dmin, depth);
                    dmax = std::fmax(dmax, std::fabs(depth));
                }
                if (std::isfinite(dmin) && dmin > 1e-3 * dmax) d.front_targets |= 1u << c2;
            }
        }
        // pairs: H = K2 R2 M_c, e = K2 (R2 C_c + t2), both shifted by one
        // pixel in x and y (rows 0 and 1 gain row 2) to address the target's
        // bordered texel image, whose texel (x + 1, y + 1) is pixel (x, y)
        for (int c2 = 0; c2 < n; ++c2) {
            if (c2 == v) continue;
            double KR[9], Hm[9], e[3], t1[3];
            mul3(cams[c2].K, cams[c2].R, KR);
            mul3(KR, Mv, Hm);
            mv3(cams[c2].R, &C[3 * v], t1);
            for (int i = 0; i < 3; ++i) t1[i] += cams[c2].t[i];
            mv3(cams[c2].K, t1, e);
            for (int i = 0; i < 3; ++i) {
                Hm[i] += Hm[6 + i];
                Hm[3 + i] += Hm[6 + i];
            }
            e[0] += e[2];
            e[1] += e[2];
            PairConst &pc = hc.pairs[(size_t)v * n + c2];
            for (int i = 0; i < 9; ++i) pc.H[i] = (float)Hm[i];
            for (int i = 0; i < 3; ++i) pc.e[i] = (float)e[i];
        }
    }
    Problem &P = hc.problem;
    memset(&P, 0, sizeof(P));
    P.n_views = n;
    P.L = L;
    P.J = ly.J;
    P.n_lblocks = ly.n_lblocks;
    P.bilinear = opt->sampling == IVDE_BILINEAR;
    P.f16out = ly.f16;
    P.bit_depth = views ? views[0].bit_depth : 8;
    P.chroma_shift = views ? views[0].chroma_shift : 0;
    P.norm = (float)(3.0 * (double)((1 << P.bit_depth) - 1));
    P.tex_u16 = ly.tex_u16;
    P.total_rows = ly.total_rows;
    P.views = reinterpret_cast<ViewDesc *>(ws_base + ly.off_views);
    P.pairs = reinterpret_cast<PairConst *>(ws_base + ly.off_pairs);
    P.sigma = reinterpret_cast<float *>(ws_base + ly.off_sigma);
    P.cost = cost_out;
    P.flag = reinterpret_cast<int32_t *>(ws_base + ly.off_flag);
    P.steps = reinterpret_cast<unsigned long long *>(ws_base + ly.off_flag + 8);
    return IVDE_OK;
}

hipError_t upload_constants(const HostConstants &hc, const Layout &ly, char *ws_base, hipStream_t s)
{
    hipError_t e;
    if ((e = launch_upload(ws_base + ly.off_problem, &hc.problem, sizeof(Problem), s)) != hipSuccess) return e;
    if ((e = launch_upload(ws_base + ly.off_views, hc.views.data(), sizeof(ViewDesc) * hc.views.size(), s)) !=
        hipSuccess)
        return e;
    if ((e = launch_upload(ws_base + ly.off_pairs, hc.pairs.data(), sizeof(PairConst) * hc.pairs.size(), s)) !=
        hipSuccess)
        return e;
    return launch_upload(ws_base + ly.off_sigma, hc.sigma.data(), sizeof(float) * hc.sigma.size(), s);
}

Extents extents_of(const Layout &ly)
{
    Extents x;
    x.n_views = ly.n;
    x.max_w = ly.max_w;
    x.max_h = ly.max_h;
    x.max_s = ly.max_s;
    x.max_bands = ly.max_bands;
    return x;
}

// Everything of one plain cost-volume call except the sweep itself.
ivde_status enqueue_front(int32_t n, const ivde_camera *cams, const ivde_image *views,
                          const ivde_segmentation *segs, const ivde_label_range *labels, const ivde_options *opt,
                          const Layout &ly, char *ws, void *cost_out, int problem_index, Task *tasks,
                          hipStream_t s, bool index_ready, bool texels, bool worklist)
{
    HostConstants hc;
    ivde_status st = compose(n, cams, views, segs, labels, opt, ly, ws, cost_out, hc);
    if (st != IVDE_OK) return st;
    hipError_t e = upload_constants(hc, ly, ws, s);
    if (e != hipSuccess) return hip_fail(e, "constant upload");
    const Problem *dp = reinterpret_cast<const Problem *>(ws + ly.off_problem);
    e = launch_fill_i32(reinterpret_cast<int32_t *>(ws + ly.off_flag) + 2, 0, kFlagWords - 2, s);
    if (e != hipSuccess) return hip_fail(e, "step count reset");
    if (index_ready) {
        // the segment-id flag of the index build stays as it was
        e = launch_refresh(dp, extents_of(ly), ly.tex_u16, s);
        if (e != hipSuccess) return hip_fail(e, "frame refresh");
        return IVDE_OK;
    }
    e = launch_fill_i32(reinterpret_cast<int32_t *>(ws + ly.off_flag), 0, 1, s);
    if (e != hipSuccess) return hip_fail(e, "flag reset");
    e = launch_prepare(dp, extents_of(ly), ly.tex_u16, s, texels);
    if (e != hipSuccess) return hip_fail(e, "segment index");
    if (worklist && (e = launch_worklist(dp, extents_of(ly), problem_index, tasks, s)) != hipSuccess)
        return hip_fail(e, "work list");
    return IVDE_OK;
}

ivde_status enqueue_stats(int32_t n, const ivde_camera *cams, const ivde_image *views,
                          const ivde_segmentation *segs, const ivde_label_range *labels, const ivde_options *opt,
                          const Layout &ly, char *ws, Task *tasks, int32_t *count_flat, hipStream_t s, bool texels)
{
    HostConstants hc;
    ivde_status st = compose(n, cams, views, segs, labels, opt, ly, ws, nullptr, hc);
    if (st != IVDE_OK) return st;
    hipError_t e = upload_constants(hc, ly, ws, s);
    if (e != hipSuccess) return hip_fail(e, "constant upload");
    const Problem *dp = reinterpret_cast<const Problem *>(ws + ly.off_problem);
    e = launch_fill_i32(reinterpret_cast<int32_t *>(ws + ly.off_flag), 0, 1, s);
    if (e != hipSuccess) return hip_fail(e, "flag reset");
    if (texels && (e = launch_pack(dp, extents_of(ly), ly.tex_u16, s)) != hipSuccess)
        return hip_fail(e, "texel packing");
    e = launch_segment_sums(dp, extents_of(ly), reinterpret_cast<unsigned long long *>(ws + ly.off_sums),
                            ly.total_rows, count_flat, tasks, s);
    if (e != hipSuccess) return hip_fail(e, "segment statistics");
    return IVDE_OK;
}

ivde_status check_workspace(const void *workspace, size_t have, size_t need)
{
    if (!workspace) {
        set_error("null workspace");
        return IVDE_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(workspace) % 256) {
        set_error("workspace must be 256-byte aligned");
        return IVDE_EINVAL;
    }
    if (have < need) {
        set_error("workspace too small: %zu bytes given, %zu needed", have, need);
        return IVDE_ENOMEM;
    }
    return IVDE_OK;
}

ivde_status check_tex_limits(const Layout &ly)
{
    for (int v = 0; v < ly.n; ++v)
        if (ly.views[v].tex_bytes + 16 >= ((int64_t)1 << 31)) {
            set_error("view %d: packed image exceeds 2 GiB", v);
            return IVDE_EINVAL;
        }
    return IVDE_OK;
}

ivde_status enqueue_cost_volume(int32_t n, const ivde_camera *cams, const ivde_image *views,
                                const ivde_segmentation *segs, const ivde_label_range *labels,
                                const ivde_options *opt, const Layout &ly, char *ws, void *cost_out, hipStream_t s)
{
    Task *tasks = reinterpret_cast<Task *>(ws + ly.off_tasks);
    ivde_status st = enqueue_front(n, cams, views, segs, labels, opt, ly, ws, cost_out, 0, tasks, s);
    if (st != IVDE_OK) return st;
    const Problem *dp = reinterpret_cast<const Problem *>(ws + ly.off_problem);
    hipError_t e;
    if (opt->sweep_events[0] && opt->sweep_events[1] &&
        (e = hipEventRecord(static_cast<hipEvent_t>(opt->sweep_events[0]), s)) != hipSuccess)
        return hip_fail(e, "event record");
    e = launch_sweep(dp, tasks, ly.n_tasks, ly.J, ly.px, opt->sampling == IVDE_BILINEAR, ly.tex_u16, ly.f16, ly.wpg,
                     reinterpret_cast<int32_t *>(ws + ly.off_cursors), s);
    if (e != hipSuccess) return hip_fail(e, "sweep");
    if (opt->sweep_events[0] && opt->sweep_events[1] &&
        (e = hipEventRecord(static_cast<hipEvent_t>(opt->sweep_events[1]), s)) != hipSuccess)
        return hip_fail(e, "event record");
    return IVDE_OK;
}

}  // namespace ivde

using namespace ivde;

extern "C" {

ivde_status ivde_cost_volume_size(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                                  const ivde_label_range *labels, const ivde_options *opt, int32_t bit_depth,
                                  size_t *cost_bytes, size_t *workspace_bytes)
{
    ivde_status st = validate_problem(n_views, cams, nullptr, segs, labels, opt, false);
    if (st != IVDE_OK) return st;
    if (bit_depth < 8 || bit_depth > 16) {
        set_error("bit_depth must be 8..16");
        return IVDE_EINVAL;
    }
    Layout ly = plan_layout(n_views, cams, segs, labels, opt, bit_depth);
    if (cost_bytes) *cost_bytes = ly.cost_bytes;
    if (workspace_bytes) *workspace_bytes = ly.workspace_bytes;
    return IVDE_OK;
}

ivde_status ivde_sweep_shape(int32_t n_views, const ivde_camera *cams, const ivde_segmentation *segs,
                             const ivde_label_range *labels, const ivde_options *opt, int32_t bit_depth,
                             int32_t *labels_per_lane, int32_t *waves_per_group, int32_t *pixels_per_step)
{
    ivde_status st = validate_problem(n_views, cams, nullptr, segs, labels, opt, false);
    if (st != IVDE_OK) return st;
    if (bit_depth < 8 || bit_depth > 16) {
        set_error("bit_depth must be 8..16");
        return IVDE_EINVAL;
    }
    const Layout ly = plan_layout(n_views, cams, segs, labels, opt, bit_depth);
    if (labels_per_lane) *labels_per_lane = ly.J;
    if (waves_per_group) *waves_per_group = ly.wpg;
    if (pixels_per_step) *pixels_per_step = ly.px;
    return IVDE_OK;
}

ivde_status ivde_cost_volume(int32_t n_views, const ivde_camera *cams, const ivde_image *views,
                             const ivde_segmentation *segs, const ivde_label_range *labels, const ivde_options *opt,
                             void *workspace, size_t workspace_bytes, void *cost_out, ivde_stream stream)
{
    ivde_status st = validate_problem(n_views, cams, views, segs, labels, opt, true);
    if (st != IVDE_OK) return st;
    if (!cost_out) {
        set_error("null cost_out");
        return IVDE_EINVAL;
    }
    const Layout ly = plan_layout(n_views, cams, segs, labels, opt, views[0].bit_depth);
    if ((st = check_workspace(workspace, workspace_bytes, ly.workspace_bytes)) != IVDE_OK) return st;
    if ((st = check_tex_limits(ly)) != IVDE_OK) return st;
    return enqueue_cost_volume(n_views, cams, views, segs, labels, opt, ly, static_cast<char *>(workspace), cost_out,
                               static_cast<hipStream_t>(stream));
}

ivde_status ivde_argmin(int64_t rows, int32_t num_labels, int32_t cost_dtype, const void *cost, int32_t *label_out,
                        ivde_stream stream)
{
    if (rows < 0 || num_labels < 1 || (cost_dtype != IVDE_F32 && cost_dtype != IVDE_F16)) {
        set_error("argmin: rows >= 0, num_labels >= 1 and a known dtype are required");
        return IVDE_EINVAL;
    }
    if (rows > 0 && (!cost || !label_out)) {
        set_error("argmin: null pointer");
        return IVDE_EINVAL;
    }
    hipError_t e = launch_argmin(cost, cost_dtype == IVDE_F16, rows, num_labels, label_out,
                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "argmin");
    return IVDE_OK;
}

ivde_status ivde_workspace_status(const void *workspace, ivde_stream stream)
{
    if (!workspace) {
        set_error("null workspace");
        return IVDE_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    // the problem header sits at the start of the workspace; its flag pointer
    // locates the device error flag
    Problem p;
    e = hipMemcpy(&p, workspace, sizeof(p), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read problem header");
    int32_t flag = 0;
    e = hipMemcpy(&flag, p.flag, sizeof(flag), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read error flag");
    if (flag) {
        set_error("a segment id was outside [0, num_segments)");
        return IVDE_EINVAL;
    }
    return IVDE_OK;
}

ivde_status ivde_workspace_sweep_steps(const void *workspace, ivde_stream stream, int64_t *steps_total,
                                       int64_t *steps_projected, int64_t *steps_inside)
{
    if (!workspace) {
        set_error("null workspace");
        return IVDE_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    Problem p;
    e = hipMemcpy(&p, workspace, sizeof(p), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read problem header");
    unsigned long long c[3] = {0, 0, 0};
    e = hipMemcpy(c, p.steps, sizeof(c), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read step counts");
    if (steps_total) *steps_total = (int64_t)c[0];
    if (steps_projected) *steps_projected = (int64_t)c[1];
    if (steps_inside) *steps_inside = (int64_t)c[2];
    return IVDE_OK;
}

const char *ivde_status_string(ivde_status s)
{
    switch (s) {
    case IVDE_OK: return "ok";
    case IVDE_EINVAL: return "invalid argument";
    case IVDE_ENOMEM: return "out of memory";
    case IVDE_EBUDGET: return "over the HBM budget";
    case IVDE_EHIP: return "HIP runtime error";
    case IVDE_EBUSY: return "not ready";
    case IVDE_ENOTFOUND: return "not found";
    default: return "unknown status";
    }
}

const char *ivde_last_error(void) { return ivde::last_error(); }

const char *ivde_version(void) { return "ivde 0.1 gfx950"; }

}  // extern "C"
