/*
 * oracle.c -- plain FP64 CPU oracle of the per-segment plane-sweep matching
 * cost volume.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU
 * library: it does its own ray-plane intersection per pixel and label instead
 * of the GPU path's affine-in-inverse-depth projection.
 *
 * What it computes (the paper's inter-view matching core, Sec. III-C Eq. (4),
 * generalised from a window at the segment centre to every pixel of the
 * segment):
 *
 *   labels      rho_l = 1/z_far + l/(L-1) * (1/z_near - 1/z_far), z_l = 1/rho_l
 *               (depth levels parallel to a reference camera plane, Sec. IV-A;
 *               depth measured from the rig's centre camera plane, Sec. III-B)
 *   3-D point   pixel p = (x, y) of view c, centre C_c = -R_c^T t_c, ray
 *               d = R_c^T K_c^-1 [x y 1]^T, tau = (z_l - n_r.(C_c - C_r)) / (n_r.d);
 *               tau <= 0 leaves the pixel invalid at this label; X = C_c + tau d
 *   projection  X' = R_c' X + t_c' (invalid if X'_z <= 0), (u, v) = K_c' X'
 *               divided by its third component (the transform T[.] of Eq. (4))
 *   sampling    nearest: (floor(u + 1/2), floor(v + 1/2)) inside the image;
 *               bilinear: -1/64 <= u <= W-1 + 1/64 (same for v), u clamped
 *               to [0, W-1], taps x0 = floor(u), x1 = min(x0 + 1, W - 1)
 *               (same for y); chroma uses the same weights at taps
 *               (x_j >> k, y_j >> k).  The 1/64 px margin keeps samples that
 *               land exactly on the outer pixel centres (every border row of
 *               a rectified rig) from depending on the last bit of u.
 *   pixel cost  e = (|dY| + |dCb| + |dCr|) / (3 (2^b - 1))   (L1 of Eq. (4))
 *   segment     m[c][c'][s][l] = mean of e over the valid pixels of s
 *   cost        C[c][s][l] = min over targets c' with a valid pixel of m,
 *               or 1.0 when no target has one
 *
 * Loops run view -> segment -> pixel -> label -> target, with OpenMP over the
 * requested (view, segment) rows.  Every sum is FP64.
 *
 * Also here: per-segment statistics (count, centre, mean colour) and the
 * paper's own window matching core of Eq. (4) towards the neighbouring views
 * (oracle_segment_stats, oracle_window_rows, at the end of the file).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* margin beyond the outer pixel centres inside which bilinear samples are
 * still taken (clamped to the edge), in pixels */
#define EDGE (1.0 / 64.0)

typedef struct {
    int32_t n_views;
    const double *K;              /* n x 9, row-major */
    const double *R;              /* n x 9, row-major, world -> camera */
    const double *t;              /* n x 3 */
    const int32_t *width;         /* n */
    const int32_t *height;        /* n */
    const void *const *planes;    /* n x 3 host pointers: Y, Cb, Cr */
    const int64_t *pitch;         /* n x 3 row pitches in elements */
    int32_t bit_depth;            /* 8 -> uint8 samples, 9..16 -> uint16 */
    int32_t chroma_shift;         /* 0: 4:4:4, 1: 4:2:0 */
    const int32_t *const *seg;    /* n host pointers to H x W segment ids */
    const int32_t *num_segments;  /* n */
    double z_near, z_far;
    int32_t num_labels;
    int32_t depth_ref;            /* -1 rig centre, -2 own camera, >= 0 camera index */
    int32_t bilinear;             /* 0 nearest, 1 bilinear */
    const uint8_t *targets;       /* n x n, targets[c * n + c2] != 0: c2 is a target of c */
} oracle_problem;

typedef struct {
    int64_t *start;   /* S + 1 */
    int32_t *pix;     /* H * W pixel indices, raster order inside each segment */
} seg_lists;

static double sample_at(const oracle_problem *pb, int v, int ch, int64_t x, int64_t y)
{
    const void *p = pb->planes[v * 3 + ch];
    int64_t off = y * pb->pitch[v * 3 + ch] + x;
    if (pb->bit_depth <= 8) return (double)((const uint8_t *)p)[off];
    return (double)((const uint16_t *)p)[off];
}

/* Inverse of a general 3 x 3 matrix by cofactors. */
static int inv3(const double *a, double *o)
{
    double c00 = a[4] * a[8] - a[5] * a[7];
    double c01 = a[5] * a[6] - a[3] * a[8];
    double c02 = a[3] * a[7] - a[4] * a[6];
    double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    if (det == 0.0 || !isfinite(det)) return -1;
    double r = 1.0 / det;
    o[0] = c00 * r;
    o[1] = (a[2] * a[7] - a[1] * a[8]) * r;
    o[2] = (a[1] * a[5] - a[2] * a[4]) * r;
    o[3] = c01 * r;
    o[4] = (a[0] * a[8] - a[2] * a[6]) * r;
    o[5] = (a[2] * a[3] - a[0] * a[5]) * r;
    o[6] = c02 * r;
    o[7] = (a[1] * a[6] - a[0] * a[7]) * r;
    o[8] = (a[0] * a[4] - a[1] * a[3]) * r;
    return 0;
}

static void camera_centre(const oracle_problem *pb, int v, double *C)
{
    const double *R = pb->R + 9 * v, *t = pb->t + 3 * v;
    for (int i = 0; i < 3; ++i) C[i] = -(R[0 + i] * t[0] + R[3 + i] * t[1] + R[6 + i] * t[2]);
}

static int build_lists(const oracle_problem *pb, int v, seg_lists *out)
{
    int64_t W = pb->width[v], H = pb->height[v], S = pb->num_segments[v];
    const int32_t *m = pb->seg[v];
    out->start = (int64_t *)calloc((size_t)S + 1, sizeof(int64_t));
    out->pix = (int32_t *)malloc((size_t)(W * H > 0 ? W * H : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)calloc((size_t)S + 1, sizeof(int64_t));
    if (!out->start || !out->pix || !fill) { free(fill); return -2; }
    for (int64_t i = 0; i < W * H; ++i) {
        if (m[i] < 0 || m[i] >= S) { free(fill); return -1; }
        out->start[m[i] + 1]++;
    }
    for (int64_t s = 0; s < S; ++s) out->start[s + 1] += out->start[s];
    for (int64_t i = 0; i < W * H; ++i) {
        int32_t s = m[i];
        out->pix[out->start[s] + fill[s]++] = (int32_t)i;
    }
    free(fill);
    return 0;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing only; results do not depend on it). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/*
 * Cost rows for the requested (view, segment) pairs.
 *   cost      n_rows x L          C[c][s][l]
 *   m_out     n_rows x n x L      per-target mean (NaN where no pixel is valid), or NULL
 *   nv_out    n_rows x n x L      per-target valid-pixel counts, or NULL
 * Returns 0, -1 for invalid input, -2 when out of memory.
 */
int oracle_cost_rows(const oracle_problem *pb, int64_t n_rows, const int32_t *row_view,
                     const int32_t *row_seg, double *cost, double *m_out, int64_t *nv_out)
{
    const int n = pb->n_views, L = pb->num_labels;
    if (n <= 0 || L <= 0 || !(pb->z_near > 0) || !(pb->z_far > 0)) return -1;
    if (pb->bit_depth < 8 || pb->bit_depth > 16) return -1;
    if (pb->chroma_shift < 0 || pb->chroma_shift > 1) return -1;
    if (pb->depth_ref < -2 || pb->depth_ref >= n) return -1;

    double *Kinv = (double *)malloc(sizeof(double) * 9 * n);
    double *Cc = (double *)malloc(sizeof(double) * 3 * n);
    double *zl = (double *)malloc(sizeof(double) * L);
    seg_lists *lists = (seg_lists *)calloc((size_t)n, sizeof(seg_lists));
    int rc = 0;
    if (!Kinv || !Cc || !zl || !lists) { rc = -2; goto done; }
    for (int v = 0; v < n; ++v) {
        if (inv3(pb->K + 9 * v, Kinv + 9 * v)) { rc = -1; goto done; }
        camera_centre(pb, v, Cc + 3 * v);
    }
    for (int l = 0; l < L; ++l) {
        double frac = L > 1 ? (double)l / (double)(L - 1) : 0.0;
        double rho = 1.0 / pb->z_far + frac * (1.0 / pb->z_near - 1.0 / pb->z_far);
        zl[l] = 1.0 / rho;
    }
    /* requested views need pixel lists */
    for (int64_t r = 0; r < n_rows; ++r) {
        int v = row_view[r];
        if (v < 0 || v >= n || row_seg[r] < 0 || row_seg[r] >= pb->num_segments[v]) { rc = -1; goto done; }
        if (!lists[v].start) {
            int e = build_lists(pb, v, &lists[v]);
            if (e) { rc = e; goto done; }
        }
    }

    const double norm = 3.0 * (double)((1 << pb->bit_depth) - 1);
    const int k = pb->chroma_shift;

#pragma omp parallel
    {
        double *sum = (double *)malloc(sizeof(double) * n * L);
        int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * n * L);
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < n_rows; ++r) {
            const int c = row_view[r], s = row_seg[r];
            const double *Rc = pb->R + 9 * c, *Ki = Kinv + 9 * c, *C = Cc + 3 * c;
            /* reference plane: normal n_r through point C_r */
            double Cr[3], nr[3];
            if (pb->depth_ref == -1) {
                double a[3] = {0, 0, 0};
                Cr[0] = Cr[1] = Cr[2] = 0.0;
                for (int v = 0; v < n; ++v)
                    for (int i = 0; i < 3; ++i) {
                        Cr[i] += Cc[3 * v + i] / n;
                        a[i] += pb->R[9 * v + 6 + i] / n;
                    }
                double len = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
                for (int i = 0; i < 3; ++i) nr[i] = a[i] / len;
            } else {
                int rv = pb->depth_ref == -2 ? c : pb->depth_ref;
                for (int i = 0; i < 3; ++i) {
                    Cr[i] = Cc[3 * rv + i];
                    nr[i] = pb->R[9 * rv + 6 + i];
                }
            }
            const double offs = nr[0] * (C[0] - Cr[0]) + nr[1] * (C[1] - Cr[1]) + nr[2] * (C[2] - Cr[2]);
            memset(sum, 0, sizeof(double) * n * L);
            memset(cnt, 0, sizeof(int64_t) * n * L);
            const int64_t Wc = pb->width[c];
            for (int64_t q = lists[c].start[s]; q < lists[c].start[s + 1]; ++q) {
                const int64_t pi = lists[c].pix[q];
                const int64_t x = pi % Wc, y = pi / Wc;
                const double ref_y = sample_at(pb, c, 0, x, y);
                const double ref_u = sample_at(pb, c, 1, x >> k, y >> k);
                const double ref_v = sample_at(pb, c, 2, x >> k, y >> k);
                /* ray direction d = R^T K^-1 [x y 1]^T */
                double kp[3];
                for (int i = 0; i < 3; ++i) kp[i] = Ki[3 * i] * x + Ki[3 * i + 1] * y + Ki[3 * i + 2];
                double d[3];
                for (int i = 0; i < 3; ++i) d[i] = Rc[i] * kp[0] + Rc[3 + i] * kp[1] + Rc[6 + i] * kp[2];
                const double nd = nr[0] * d[0] + nr[1] * d[1] + nr[2] * d[2];
                for (int l = 0; l < L; ++l) {
                    const double tau = (zl[l] - offs) / nd;
                    if (!(tau > 0.0) || !isfinite(tau)) continue;
                    double X[3] = {C[0] + tau * d[0], C[1] + tau * d[1], C[2] + tau * d[2]};
                    for (int c2 = 0; c2 < n; ++c2) {
                        if (c2 == c || !pb->targets[c * n + c2]) continue;
                        const double *R2 = pb->R + 9 * c2, *t2 = pb->t + 3 * c2, *K2 = pb->K + 9 * c2;
                        double Xc[3];
                        for (int i = 0; i < 3; ++i)
                            Xc[i] = R2[3 * i] * X[0] + R2[3 * i + 1] * X[1] + R2[3 * i + 2] * X[2] + t2[i];
                        if (!(Xc[2] > 0.0)) continue;
                        double h[3];
                        for (int i = 0; i < 3; ++i) h[i] = K2[3 * i] * Xc[0] + K2[3 * i + 1] * Xc[1] + K2[3 * i + 2] * Xc[2];
                        if (!(h[2] > 0.0)) continue;
                        const double u = h[0] / h[2], vv = h[1] / h[2];
                        const int64_t W2 = pb->width[c2], H2 = pb->height[c2];
                        double sy, su, sv;
                        if (!pb->bilinear) {
                            const double fx = floor(u + 0.5), fy = floor(vv + 0.5);
                            if (!(fx >= 0.0 && fx < (double)W2 && fy >= 0.0 && fy < (double)H2)) continue;
                            const int64_t xi = (int64_t)fx, yi = (int64_t)fy;
                            sy = sample_at(pb, c2, 0, xi, yi);
                            su = sample_at(pb, c2, 1, xi >> k, yi >> k);
                            sv = sample_at(pb, c2, 2, xi >> k, yi >> k);
                        } else {
                            if (!(u >= -EDGE && u <= (double)(W2 - 1) + EDGE &&
                                  vv >= -EDGE && vv <= (double)(H2 - 1) + EDGE)) continue;
                            const double uc = fmin(fmax(u, 0.0), (double)(W2 - 1));
                            const double vc = fmin(fmax(vv, 0.0), (double)(H2 - 1));
                            const double fx = floor(uc), fy = floor(vc);
                            const double ax = uc - fx, ay = vc - fy;
                            const int64_t x0 = (int64_t)fx, y0 = (int64_t)fy;
                            const int64_t x1 = x0 + 1 < W2 ? x0 + 1 : W2 - 1;
                            const int64_t y1 = y0 + 1 < H2 ? y0 + 1 : H2 - 1;
                            const double w00 = (1 - ax) * (1 - ay), w01 = ax * (1 - ay);
                            const double w10 = (1 - ax) * ay, w11 = ax * ay;
                            sy = w00 * sample_at(pb, c2, 0, x0, y0) + w01 * sample_at(pb, c2, 0, x1, y0)
                               + w10 * sample_at(pb, c2, 0, x0, y1) + w11 * sample_at(pb, c2, 0, x1, y1);
                            su = w00 * sample_at(pb, c2, 1, x0 >> k, y0 >> k) + w01 * sample_at(pb, c2, 1, x1 >> k, y0 >> k)
                               + w10 * sample_at(pb, c2, 1, x0 >> k, y1 >> k) + w11 * sample_at(pb, c2, 1, x1 >> k, y1 >> k);
                            sv = w00 * sample_at(pb, c2, 2, x0 >> k, y0 >> k) + w01 * sample_at(pb, c2, 2, x1 >> k, y0 >> k)
                               + w10 * sample_at(pb, c2, 2, x0 >> k, y1 >> k) + w11 * sample_at(pb, c2, 2, x1 >> k, y1 >> k);
                        }
                        /* L1 distance in code values; the 3 (2^b - 1) scale is
                         * applied once per mean so integer sums stay exact */
                        sum[c2 * L + l] += fabs(ref_y - sy) + fabs(ref_u - su) + fabs(ref_v - sv);
                        cnt[c2 * L + l] += 1;
                    }
                }
            }
            for (int l = 0; l < L; ++l) {
                double best = INFINITY;
                for (int c2 = 0; c2 < n; ++c2) {
                    const int64_t nv = cnt[c2 * L + l];
                    const double m = nv > 0 ? sum[c2 * L + l] / ((double)nv * norm) : NAN;
                    if (m_out) m_out[(r * n + c2) * L + l] = m;
                    if (nv_out) nv_out[(r * n + c2) * L + l] = nv;
                    if (nv > 0 && m < best) best = m;
                }
                cost[r * L + l] = isfinite(best) ? best : 1.0;
            }
        }
        free(sum);
        free(cnt);
    }

done:
    if (lists) {
        for (int v = 0; v < n; ++v) { free(lists[v].start); free(lists[v].pix); }
        free(lists);
    }
    free(Kinv);
    free(Cc);
    free(zl);
    return rc;
}

/*
 * Per-segment statistics of view v: pixel count, centre (the centroid of the
 * pixel coordinates rounded half up, the segment centre mu_s of Sec. III-C)
 * and mean Y, Cb, Cr (the segment colour of Sec. III-D and III-E).
 *   count  S      centre  2 S (x, y)      mean  3 S
 */
int oracle_segment_stats(const oracle_problem *pb, int v, int64_t *count, int32_t *centre, double *mean)
{
    if (v < 0 || v >= pb->n_views) return -1;
    const int64_t W = pb->width[v], H = pb->height[v], S = pb->num_segments[v];
    const int k = pb->chroma_shift;
    double *sx = (double *)calloc((size_t)S, sizeof(double));
    double *sy = (double *)calloc((size_t)S, sizeof(double));
    if (!sx || !sy) { free(sx); free(sy); return -2; }
    for (int64_t s = 0; s < S; ++s) { count[s] = 0; mean[3 * s] = mean[3 * s + 1] = mean[3 * s + 2] = 0.0; }
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            const int32_t s = pb->seg[v][y * W + x];
            if (s < 0 || s >= S) { free(sx); free(sy); return -1; }
            count[s]++;
            sx[s] += (double)x;
            sy[s] += (double)y;
            mean[3 * s] += sample_at(pb, v, 0, x, y);
            mean[3 * s + 1] += sample_at(pb, v, 1, x >> k, y >> k);
            mean[3 * s + 2] += sample_at(pb, v, 2, x >> k, y >> k);
        }
    for (int64_t s = 0; s < S; ++s) {
        if (count[s] == 0) { centre[2 * s] = centre[2 * s + 1] = -1; continue; }
        const double n = (double)count[s];
        centre[2 * s] = (int32_t)floor(sx[s] / n + 0.5);
        centre[2 * s + 1] = (int32_t)floor(sy[s] / n + 0.5);
        for (int c = 0; c < 3; ++c) mean[3 * s + c] /= n;
    }
    free(sx);
    free(sy);
    return 0;
}

/*
 * The paper's window matching core (Sec. III-C, Eq. (4)) for the requested
 * rows, towards the neighbouring views of Sec. III-B: slot 0 is view c - 1,
 * slot 1 view c + 1 (views ordered along the rig).  For label l the centre
 * mu_s is lifted to the level plane and transformed into c' (the same T[.]
 * as oracle_cost_rows); the target window is centred on the nearest pixel
 * of the projection.  Window taps outside an image are clamped to its edge.
 *   m    n_rows x 2 x L   mean over the (2r+1)^2 taps of |dY| + |dCb| + |dCr|
 *                         in 8-bit code values (divided by 2^(b-8));
 *                         NaN where there is no neighbour or the projection
 *                         is behind a camera or outside c'
 *   hit  n_rows x 2 x L   the segment of c' under the projected centre, as a
 *                         row of the volume (row offset of c' plus its id),
 *                         or -1 where m is NaN
 *   uv   n_rows x 2 x L x 2 (optional) the projected centre in pixels of c'
 */
int oracle_window_rows(const oracle_problem *pb, int64_t n_rows, const int32_t *row_view, const int32_t *row_seg,
                       int32_t radius, double *m, int64_t *hit, double *uv)
{
    const int n = pb->n_views, L = pb->num_labels;
    if (n <= 0 || L <= 0 || radius < 0 || radius > 8) return -1;
    if (pb->depth_ref < -2 || pb->depth_ref >= n) return -1;
    double *Kinv = (double *)malloc(sizeof(double) * 9 * n);
    double *Cc = (double *)malloc(sizeof(double) * 3 * n);
    double *zl = (double *)malloc(sizeof(double) * L);
    int64_t *row0 = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    int32_t **centres = (int32_t **)calloc((size_t)n, sizeof(int32_t *));
    int rc = 0;
    if (!Kinv || !Cc || !zl || !row0 || !centres) { rc = -2; goto done; }
    row0[0] = 0;
    for (int v = 0; v < n; ++v) {
        if (inv3(pb->K + 9 * v, Kinv + 9 * v)) { rc = -1; goto done; }
        camera_centre(pb, v, Cc + 3 * v);
        row0[v + 1] = row0[v] + pb->num_segments[v];
    }
    for (int l = 0; l < L; ++l) {
        const double frac = L > 1 ? (double)l / (double)(L - 1) : 0.0;
        zl[l] = 1.0 / (1.0 / pb->z_far + frac * (1.0 / pb->z_near - 1.0 / pb->z_far));
    }
    for (int64_t r = 0; r < n_rows; ++r) {
        const int v = row_view[r];
        if (v < 0 || v >= n || row_seg[r] < 0 || row_seg[r] >= pb->num_segments[v]) { rc = -1; goto done; }
        if (!centres[v]) {
            const int64_t S = pb->num_segments[v];
            int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * S);
            double *mean = (double *)malloc(sizeof(double) * 3 * S);
            centres[v] = (int32_t *)malloc(sizeof(int32_t) * 2 * S);
            if (!cnt || !mean || !centres[v]) { free(cnt); free(mean); rc = -2; goto done; }
            rc = oracle_segment_stats(pb, v, cnt, centres[v], mean);
            free(cnt);
            free(mean);
            if (rc) goto done;
        }
    }
    {
        const double scale = (double)(1 << (pb->bit_depth - 8));
        const int k = pb->chroma_shift;
        const int taps = (2 * radius + 1) * (2 * radius + 1);
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t r = 0; r < n_rows; ++r) {
            const int c = row_view[r], s = row_seg[r];
            const int64_t Wc = pb->width[c], Hc = pb->height[c];
            const int32_t mx = centres[c][2 * s], my = centres[c][2 * s + 1];
            /* reference plane */
            double Cr[3], nr[3];
            if (pb->depth_ref == -1) {
                double a[3] = {0, 0, 0};
                Cr[0] = Cr[1] = Cr[2] = 0.0;
                for (int v = 0; v < n; ++v)
                    for (int i = 0; i < 3; ++i) {
                        Cr[i] += Cc[3 * v + i] / n;
                        a[i] += pb->R[9 * v + 6 + i] / n;
                    }
                const double len = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
                for (int i = 0; i < 3; ++i) nr[i] = a[i] / len;
            } else {
                const int rv = pb->depth_ref == -2 ? c : pb->depth_ref;
                for (int i = 0; i < 3; ++i) { Cr[i] = Cc[3 * rv + i]; nr[i] = pb->R[9 * rv + 6 + i]; }
            }
            for (int slot = 0; slot < 2; ++slot) {
                const int c2 = slot == 0 ? c - 1 : c + 1;
                for (int l = 0; l < L; ++l) {
                    const int64_t o = (r * 2 + slot) * L + l;
                    m[o] = NAN;
                    hit[o] = -1;
                    if (uv) uv[2 * o] = uv[2 * o + 1] = NAN;
                }
                if (c2 < 0 || c2 >= n || mx < 0) continue;
                const double *Ki = Kinv + 9 * c, *Rc = pb->R + 9 * c, *C = Cc + 3 * c;
                double kp[3], d[3];
                for (int i = 0; i < 3; ++i) kp[i] = Ki[3 * i] * mx + Ki[3 * i + 1] * my + Ki[3 * i + 2];
                for (int i = 0; i < 3; ++i) d[i] = Rc[i] * kp[0] + Rc[3 + i] * kp[1] + Rc[6 + i] * kp[2];
                const double nd = nr[0] * d[0] + nr[1] * d[1] + nr[2] * d[2];
                const double offs = nr[0] * (C[0] - Cr[0]) + nr[1] * (C[1] - Cr[1]) + nr[2] * (C[2] - Cr[2]);
                const int64_t W2 = pb->width[c2], H2 = pb->height[c2];
                for (int l = 0; l < L; ++l) {
                    const int64_t o = (r * 2 + slot) * L + l;
                    const double tau = (zl[l] - offs) / nd;
                    if (!(tau > 0.0) || !isfinite(tau)) continue;
                    const double X[3] = {C[0] + tau * d[0], C[1] + tau * d[1], C[2] + tau * d[2]};
                    const double *R2 = pb->R + 9 * c2, *t2 = pb->t + 3 * c2, *K2 = pb->K + 9 * c2;
                    double Xc[3], h[3];
                    for (int i = 0; i < 3; ++i)
                        Xc[i] = R2[3 * i] * X[0] + R2[3 * i + 1] * X[1] + R2[3 * i + 2] * X[2] + t2[i];
                    if (!(Xc[2] > 0.0)) continue;
                    for (int i = 0; i < 3; ++i) h[i] = K2[3 * i] * Xc[0] + K2[3 * i + 1] * Xc[1] + K2[3 * i + 2] * Xc[2];
                    if (!(h[2] > 0.0)) continue;
                    const double u = h[0] / h[2], vv = h[1] / h[2];
                    if (uv) { uv[2 * o] = u; uv[2 * o + 1] = vv; }
                    const double fx = floor(u + 0.5), fy = floor(vv + 0.5);
                    if (!(fx >= 0.0 && fx < (double)W2 && fy >= 0.0 && fy < (double)H2)) continue;
                    const int64_t tx = (int64_t)fx, ty = (int64_t)fy;
                    double sum = 0.0;
                    for (int dy = -radius; dy <= radius; ++dy)
                        for (int dx = -radius; dx <= radius; ++dx) {
                            int64_t ax = mx + dx, ay = my + dy, bx = tx + dx, by = ty + dy;
                            ax = ax < 0 ? 0 : (ax >= Wc ? Wc - 1 : ax);
                            ay = ay < 0 ? 0 : (ay >= Hc ? Hc - 1 : ay);
                            bx = bx < 0 ? 0 : (bx >= W2 ? W2 - 1 : bx);
                            by = by < 0 ? 0 : (by >= H2 ? H2 - 1 : by);
                            sum += fabs(sample_at(pb, c, 0, ax, ay) - sample_at(pb, c2, 0, bx, by));
                            sum += fabs(sample_at(pb, c, 1, ax >> k, ay >> k) - sample_at(pb, c2, 1, bx >> k, by >> k));
                            sum += fabs(sample_at(pb, c, 2, ax >> k, ay >> k) - sample_at(pb, c2, 2, bx >> k, by >> k));
                        }
                    m[o] = sum / ((double)taps * scale);
                    hit[o] = row0[c2] + pb->seg[c2][ty * W2 + tx];
                }
            }
        }
    }
done:
    if (centres) {
        for (int v = 0; v < n; ++v) free(centres[v]);
        free(centres);
    }
    free(Kinv);
    free(Cc);
    free(zl);
    free(row0);
    return rc;
}
