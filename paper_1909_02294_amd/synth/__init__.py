"""Seeded synthetic multiview workloads for the segment cost volume.

The paper measures on free-viewpoint test sequences (Sec. V-A, Table I:
1024x768 to 1920x1080, 8 views, about 250 depth levels, 1k-150k segments
per view).  Those sequences are not available here, so this module renders
stand-ins with the same shapes: camera rigs (a rectified line and a
converging arc), textured planar scenes ray-cast into YCbCr views, Voronoi
segment label maps, and short sequences with changed-segment masks.

The module only renders inputs.  It computes no matching cost; the GPU path
and the CPU oracle both consume the arrays it returns and nothing else from
it.

Conventions shared by every consumer of these arrays (they are also the
library's documented conventions):
  * a camera maps world points X to camera coordinates R @ X + t, K is the
    upper-triangular zero-skew intrinsic matrix, pixel centres sit at
    integer (x, y) with x to the right and y down, cx = (W - 1) / 2;
  * images are Y, U, V planes of unsigned integers at `bit_depth` bits;
    with chroma_shift = 1 (4:2:0) the chroma planes are ceil(W/2) x ceil(H/2)
    and pixel (x, y) owns chroma sample (x >> 1, y >> 1);
  * a segment map is an int32 H x W array of ids in [0, S).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 1909002294


# base seeds of the synthetic workloads
SEED_RECTIFIED = BASE_SEED
SEED_ARC_1080P = BASE_SEED + 1000
SEED_BATCH = BASE_SEED + 2000
SEED_PRECISION = BASE_SEED + 3000
SEED_SERVING = BASE_SEED + 4000
SEED_PAPER_HD = BASE_SEED + 5000


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
@dataclass
class Camera:
    K: np.ndarray          # 3x3 float64
    R: np.ndarray          # 3x3 float64, world -> camera rotation
    t: np.ndarray          # 3 float64, world -> camera translation
    width: int
    height: int

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t

    @property
    def axis(self) -> np.ndarray:
        """Optical axis (camera +z) in world coordinates."""
        return self.R[2].copy()


def intrinsics(f: float, width: int, height: int) -> np.ndarray:
    return np.array([[f, 0.0, (width - 1) / 2.0],
                     [0.0, f, (height - 1) / 2.0],
                     [0.0, 0.0, 1.0]])


def look_at(center, target, width, height, f) -> Camera:
    """Camera at `center` looking at `target`; world y points down."""
    center = np.asarray(center, float)
    z = np.asarray(target, float) - center
    z /= np.linalg.norm(z)
    x = np.cross(np.array([0.0, 1.0, 0.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return Camera(intrinsics(f, width, height), R, -R @ center, width, height)


def rectified_rig(n=3, baseline=0.05, f=300.0, width=320, height=240):
    """`n` cameras on the x axis, identity rotation, spaced by `baseline`."""
    cams = []
    for i in range(n):
        c = np.array([(i - (n - 1) / 2.0) * baseline, 0.0, 0.0])
        R = np.eye(3)
        cams.append(Camera(intrinsics(f, width, height), R, -R @ c, width, height))
    return cams


def arc_rig(n=8, radius=3.0, arc_deg=30.0, f=1400.0, width=1920, height=1080):
    """`n` cameras on a horizontal arc of `radius` metres spanning `arc_deg`,
    each looking at the arc centre (the world origin)."""
    cams = []
    for i in range(n):
        th = math.radians(-arc_deg / 2.0 + i * arc_deg / max(n - 1, 1))
        c = np.array([radius * math.sin(th), 0.0, -radius * math.cos(th)])
        cams.append(look_at(c, np.zeros(3), width, height, f))
    return cams


def rig_reference(cams):
    """Mean camera centre and normalised mean optical axis of a rig."""
    C = np.mean([c.center for c in cams], axis=0)
    a = np.mean([c.axis for c in cams], axis=0)
    return C, a / np.linalg.norm(a)


# --------------------------------------------------------------------------
# textured planar scenes
# --------------------------------------------------------------------------
@dataclass
class Plane:
    origin: np.ndarray     # a point on the plane (texture centre)
    normal: np.ndarray     # unit normal
    a1: np.ndarray         # unit in-plane axes
    a2: np.ndarray
    half1: float           # half extents along a1, a2 (metres)
    half2: float
    texel: float           # texel edge length (metres)
    tex: np.ndarray = field(repr=False)   # (3, m1, m2) float32 Y, U, V texels


def channel_ranges(bit_depth: int):
    s = float(1 << (bit_depth - 8))
    return (16.0 * s, 235.0 * s), (16.0 * s, 240.0 * s)


def make_texture(rng, m1, m2, bit_depth):
    """i.i.d. uniform texels smoothed by the separable [1, 2, 1] / 4 filter."""
    (ylo, yhi), (clo, chi) = channel_ranges(bit_depth)
    raw = np.empty((3, m1 + 2, m2 + 2), np.float32)
    raw[0] = rng.uniform(ylo, yhi, size=(m1 + 2, m2 + 2))
    raw[1] = rng.uniform(clo, chi, size=(m1 + 2, m2 + 2))
    raw[2] = rng.uniform(clo, chi, size=(m1 + 2, m2 + 2))
    a = 0.25 * raw[:, :-2, :] + 0.5 * raw[:, 1:-1, :] + 0.25 * raw[:, 2:, :]
    return (0.25 * a[:, :, :-2] + 0.5 * a[:, :, 1:-1] + 0.25 * a[:, :, 2:]).astype(np.float32)


def _basis(normal):
    n = normal / np.linalg.norm(normal)
    helper = np.array([0.0, 1.0, 0.0]) if abs(n[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    a1 = np.cross(helper, n)
    a1 /= np.linalg.norm(a1)
    a2 = np.cross(n, a1)
    return n, a1, a2


def make_plane(rng, origin, normal, half1, half2, texel, bit_depth, max_texels=6000):
    n, a1, a2 = _basis(np.asarray(normal, float))
    texel = max(texel, 2.0 * max(half1, half2) / max_texels)
    m1 = int(math.ceil(2 * half1 / texel)) + 1
    m2 = int(math.ceil(2 * half2 / texel)) + 1
    return Plane(np.asarray(origin, float), n, a1, a2, half1, half2, texel,
                 make_texture(rng, m1, m2, bit_depth))


def _pixel_rays(cam: Camera, x0, x1, y0, y1):
    xs = np.arange(x0, x1, dtype=np.float64)
    ys = np.arange(y0, y1, dtype=np.float64)
    X, Y = np.meshgrid(xs, ys)
    Kinv = np.linalg.inv(cam.K)
    d_cam = np.stack([Kinv[0, 0] * X + Kinv[0, 1] * Y + Kinv[0, 2],
                      Kinv[1, 1] * Y + Kinv[1, 2],
                      np.ones_like(X)], axis=-1)
    return d_cam @ cam.R          # rows are R^T d_cam; camera-z component is 1


def _plane_pixel_box(plane: Plane, cam: Camera):
    """Pixel box covering the plane's image, or the full frame if unsure."""
    full = (0, cam.width, 0, cam.height)
    if not (np.isfinite(plane.half1) and np.isfinite(plane.half2)):
        return full
    us, vs = [], []
    for s1 in (-plane.half1, plane.half1):
        for s2 in (-plane.half2, plane.half2):
            X = plane.origin + s1 * plane.a1 + s2 * plane.a2
            Xc = cam.R @ X + cam.t
            if Xc[2] <= 1e-6:
                return full
            p = cam.K @ Xc
            us.append(p[0] / p[2])
            vs.append(p[1] / p[2])
    x0 = max(0, int(math.floor(min(us))) - 2)
    x1 = min(cam.width, int(math.ceil(max(us))) + 3)
    y0 = max(0, int(math.floor(min(vs))) - 2)
    y1 = min(cam.height, int(math.ceil(max(vs))) + 3)
    if x0 >= x1 or y0 >= y1:
        return None
    return x0, x1, y0, y1


def render(planes, cam: Camera, bit_depth=8, chroma_shift=0):
    """Ray-cast the planes into `cam` (nearest hit wins).

    Returns (Y, U, V, plane_id) with Y full resolution, U and V subsampled by
    `chroma_shift`, and plane_id the int16 index of the visible plane (-1 for
    none; such pixels get mid-grey).
    """
    W, H = cam.width, cam.height
    C = cam.center
    zbuf = np.full((H, W), np.inf)
    pid = np.full((H, W), -1, np.int16)
    s1buf = np.zeros((H, W))
    s2buf = np.zeros((H, W))
    for k, pl in enumerate(planes):
        box = _plane_pixel_box(pl, cam)
        if box is None:
            continue
        x0, x1, y0, y1 = box
        d = _pixel_rays(cam, x0, x1, y0, y1)
        denom = d @ pl.normal
        num = float((pl.origin - C) @ pl.normal)
        with np.errstate(divide="ignore", invalid="ignore"):
            tt = num / denom
        ok = np.isfinite(tt) & (tt > 0)
        rel = C - pl.origin
        s1 = rel @ pl.a1 + tt * (d @ pl.a1)
        s2 = rel @ pl.a2 + tt * (d @ pl.a2)
        ok &= (np.abs(s1) <= pl.half1) & (np.abs(s2) <= pl.half2)
        zsub = zbuf[y0:y1, x0:x1]
        win = ok & (tt < zsub)
        zsub[win] = tt[win]
        pid[y0:y1, x0:x1][win] = k
        s1buf[y0:y1, x0:x1][win] = s1[win]
        s2buf[y0:y1, x0:x1][win] = s2[win]
    mid = float(1 << (bit_depth - 1))
    img = np.full((3, H, W), mid, np.float64)
    for k, pl in enumerate(planes):
        m = pid == k
        if not m.any():
            continue
        i1 = np.clip(np.floor((s1buf[m] + pl.half1) / pl.texel).astype(np.int64), 0, pl.tex.shape[1] - 1)
        i2 = np.clip(np.floor((s2buf[m] + pl.half2) / pl.texel).astype(np.int64), 0, pl.tex.shape[2] - 1)
        for ch in range(3):
            img[ch][m] = pl.tex[ch, i1, i2]
    return (*quantize_yuv(img, bit_depth, chroma_shift), pid)


def quantize_yuv(img, bit_depth, chroma_shift):
    """Round a float (3, H, W) YUV 4:4:4 image to integer planes; 4:2:0
    chroma is the rounded mean of each 2x2 block (edge blocks may be partial)."""
    hi = (1 << bit_depth) - 1
    dt = np.uint8 if bit_depth <= 8 else np.uint16
    Y = np.clip(np.rint(img[0]), 0, hi).astype(dt)
    if chroma_shift == 0:
        return Y, np.clip(np.rint(img[1]), 0, hi).astype(dt), np.clip(np.rint(img[2]), 0, hi).astype(dt)
    H, W = img.shape[1:]
    Hc, Wc = (H + 1) // 2, (W + 1) // 2
    out = []
    for ch in (1, 2):
        p = np.pad(img[ch], ((0, 2 * Hc - H), (0, 2 * Wc - W)), mode="edge")
        m = 0.25 * (p[0::2, 0::2] + p[1::2, 0::2] + p[0::2, 1::2] + p[1::2, 1::2])
        out.append(np.clip(np.rint(m), 0, hi).astype(dt))
    return Y, out[0], out[1]


# --------------------------------------------------------------------------
# segmentations
# --------------------------------------------------------------------------
def voronoi(width, height, n_seeds, rng, weight_sigma=0.0, k_candidates=12, jittered=False):
    """Voronoi label map from `n_seeds` seeds.

    Seeds are uniform over the image, or with `jittered` one uniform point in
    each of `n_seeds` distinct cells drawn from the smallest grid of about
    square cells that has at least `n_seeds` of them (more regular cells),
    taken in raster order of the cells, so that segment ids follow the image
    as those of grid-seeded superpixel methods do.
    With weight_sigma > 0 the cells are multiplicatively weighted: pixel p
    joins argmin_i |p - c_i| / w_i with w_i ~ LogNormal(0, weight_sigma),
    searched among the k nearest seeds (exact ties, which need coincident
    float seeds, go to the nearer candidate).
    Empty cells are removed and ids compacted to [0, S) in seed order.
    Returns (int32 map, S).
    """
    from scipy.spatial import cKDTree

    if jittered:
        nx = int(np.ceil(np.sqrt(n_seeds * width / height)))
        ny = int(np.ceil(n_seeds / nx))
        cell = np.sort(rng.choice(nx * ny, n_seeds, replace=False))   # raster order of the grid
        seeds = np.stack([(cell % nx + rng.uniform(0, 1, n_seeds)) * (width / nx),
                          (cell // nx + rng.uniform(0, 1, n_seeds)) * (height / ny)], axis=1)
    else:
        seeds = np.stack([rng.uniform(0, width, n_seeds), rng.uniform(0, height, n_seeds)], axis=1)
    w = rng.lognormal(0.0, weight_sigma, n_seeds) if weight_sigma > 0 else None
    ys, xs = np.mgrid[0:height, 0:width]
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.float64)
    tree = cKDTree(seeds)
    if w is None:
        _, idx = tree.query(pts, k=1, workers=-1)
        lab = idx.astype(np.int64)
    else:
        k = min(k_candidates, n_seeds)
        dist, idx = tree.query(pts, k=k, workers=-1)
        if k == 1:
            dist, idx = dist[:, None], idx[:, None]
        score = dist / w[idx]
        j = np.argmin(score, axis=1)
        lab = idx[np.arange(len(idx)), j].astype(np.int64)
    used = np.zeros(n_seeds, bool)
    used[lab] = True
    remap = np.cumsum(used) - 1
    return remap[lab].reshape(height, width).astype(np.int32), int(used.sum())


def segment_area_sigma(seg):
    """Standard deviation of log segment areas (the realised log-normal sigma)."""
    a = np.bincount(seg.ravel())
    a = a[a > 0]
    return float(np.std(np.log(a)))


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    cams: list
    Y: list
    U: list
    V: list
    seg: list
    S: list
    bit_depth: int
    chroma_shift: int
    z_near: float
    z_far: float
    num_labels: int
    bilinear: bool
    seed: int
    plane_ids: list = field(default_factory=list, repr=False)
    info: dict = field(default_factory=dict)

    @property
    def n_views(self):
        return len(self.cams)

    def evals(self, rows_fraction=1.0):
        """Pixel-label-view evaluations of a full sweep with all other views."""
        n = self.n_views
        px = sum(c.width * c.height for c in self.cams)
        return int(px * self.num_labels * (n - 1) * rows_fraction)


def _fronto_scene(rng, cams, z_lo, z_hi, n_planes, bit_depth, f):
    """Rectified-rig scene: fronto-parallel planes; the deepest is a full-frame
    background, the others random rectangles."""
    depths = np.sort(rng.uniform(z_lo, z_hi, n_planes))[::-1]
    W, H = cams[0].width, cams[0].height
    planes = []
    for k, z in enumerate(depths):
        if k == 0:
            half1 = (W / 2 + 40) * z / f + 1.0
            half2 = (H / 2 + 40) * z / f + 1.0
            cx = cy = 0.0
        else:
            half1 = rng.uniform(0.15, 0.35) * W * z / f
            half2 = rng.uniform(0.15, 0.35) * H * z / f
            cx = rng.uniform(-0.3, 0.3) * W * z / f
            cy = rng.uniform(-0.3, 0.3) * H * z / f
        planes.append(make_plane(rng, [cx, cy, z], [0, 0, -1.0], half1, half2, z / f, bit_depth))
    return planes


def _arc_scene(rng, cams, z_lo, z_hi, n_planes, bit_depth, f, z_bg):
    """Arc-rig scene: rectangles of random orientation (normals within 60
    degrees of the rig axis, facing the rig), sides U[0.5, 3] m, depths
    U[z_lo, z_hi] from the rig's reference plane, plus a fronto-parallel
    background at z_bg."""
    Cr, nr = rig_reference(cams)
    W, H = cams[0].width, cams[0].height
    planes = []
    # background: wide enough for every view's frustum
    half1 = (z_bg + 1.0) * math.tan(math.atan(W / 2 / f) + math.radians(25)) + 2.0
    half2 = (z_bg + 1.0) * (H / 2 / f) + 1.0
    planes.append(make_plane(rng, Cr + z_bg * nr, -nr, half1, half2, z_bg / f, bit_depth))
    for _ in range(n_planes):
        z = rng.uniform(z_lo, z_hi)
        # direction within 60 degrees of -nr
        while True:
            v = rng.normal(size=3)
            v /= np.linalg.norm(v)
            if v @ (-nr) >= math.cos(math.radians(60)):
                break
        side1, side2 = rng.uniform(0.5, 3.0, 2)
        lat = rng.uniform(-0.35, 0.35) * W * z / f
        ver = rng.uniform(-0.35, 0.35) * H * z / f
        origin = Cr + z * nr + lat * np.array([1.0, 0.0, 0.0]) + ver * np.array([0.0, 1.0, 0.0])
        planes.append(make_plane(rng, origin, v, side1 / 2, side2 / 2, max(z, 1.0) / f, bit_depth))
    return planes


def _render_all(planes, cams, bit_depth, chroma_shift):
    Ys, Us, Vs, P = [], [], [], []
    for cam in cams:
        y, u, v, pid = render(planes, cam, bit_depth, chroma_shift)
        Ys.append(y); Us.append(u); Vs.append(v); P.append(pid)
    return Ys, Us, Vs, P


def make_rectified_320x240(seed=None):
    """3 rectified views 320x240, baseline 0.05 m, f = 300, YUV444 u8; 4
    fronto-parallel planes at depths U[1, 5] m; 1200 Voronoi seeds per view;
    64 labels over [1, 5] m; nearest sampling."""
    seed = SEED_RECTIFIED if seed is None else seed
    ss = np.random.SeedSequence(seed)
    s_scene, *s_views = ss.spawn(4)
    cams = rectified_rig(3, 0.05, 300.0, 320, 240)
    planes = _fronto_scene(np.random.default_rng(s_scene), cams, 1.0, 5.0, 4, 8, 300.0)
    Y, U, V, P = _render_all(planes, cams, 8, 0)
    segs, Ss = [], []
    for sv in s_views:
        m, S = voronoi(320, 240, 1200, np.random.default_rng(sv))
        segs.append(m); Ss.append(S)
    return Workload("rectified-3x320x240", cams, Y, U, V, segs, Ss, 8, 0,
                    1.0, 5.0, 64, False, seed, P)


def make_arc_workload(name, seed, n_views=8, width=1920, height=1080, f=1400.0,
                      n_segments=20000, num_labels=256, arc_deg=30.0,
                      z_near=1.5, z_far=10.0, bit_depth=10, chroma_shift=1,
                      n_planes=20, weight_sigma=0.207, bilinear=True, planes=None):
    """Arc rig: views on an arc of radius 3 m looking at its
    centre, a planar scene in [z_near, z_far] plus a background at z_far,
    multiplicatively weighted Voronoi segments from jittered-grid seeds.
    With weight_sigma = 0.207 the log segment areas have a standard
    deviation of 0.50 (measured from 5000 to 100000 seeds per view; the
    realised value is kept in info["area_sigma"])."""
    ss = np.random.SeedSequence(seed)
    s_scene, s_seg = ss.spawn(2)
    cams = arc_rig(n_views, 3.0, arc_deg, f, width, height)
    if planes is None:
        planes = _arc_scene(np.random.default_rng(s_scene), cams, z_near, z_far,
                            n_planes, bit_depth, f, z_far)
    Y, U, V, P = _render_all(planes, cams, bit_depth, chroma_shift)
    segs, Ss = [], []
    for sv in s_seg.spawn(n_views):
        m, S = voronoi(width, height, n_segments, np.random.default_rng(sv), weight_sigma, jittered=True)
        segs.append(m); Ss.append(S)
    wl = Workload(name, cams, Y, U, V, segs, Ss, bit_depth, chroma_shift,
                  z_near, z_far, num_labels, bilinear, seed, P)
    wl.info["planes"] = planes
    wl.info["area_sigma"] = float(np.mean([segment_area_sigma(s) for s in segs]))
    return wl


def make_arc_1080p(seed=None, **kw):
    """8 views 1920x1080 YUV420 10-bit on a 30-degree arc, 20 planes, 20000
    weighted Voronoi segments per view (log-area sigma 0.50), 256 labels over
    [1.5, 10] m, bilinear."""
    seed = SEED_ARC_1080P if seed is None else seed
    return make_arc_workload("arc-8x1920x1080", seed, **kw)


def make_small_arc(seed=12345, n_views=4, width=160, height=96, n_segments=150,
                   num_labels=24, bilinear=True, bit_depth=10, chroma_shift=1, f=None):
    """A reduced arc rig with the structure of the 8-view 1080p arc rig, sized for the oracle."""
    f = 1400.0 * width / 1920.0 if f is None else f
    return make_arc_workload(f"arc-{n_views}x{width}x{height}", seed, n_views=n_views,
                             width=width, height=height, f=f, n_segments=n_segments,
                             num_labels=num_labels, n_planes=8, bilinear=bilinear,
                             bit_depth=bit_depth, chroma_shift=chroma_shift)


def iter_batch_frames(n_frames=16, seed=None, width=1920, height=1080, n_views=8,
                      seg_range=(5000, 40000), label_choices=(128, 256)):
    """Batching workload, one frame at a time: `n_frames` independent
    arc-rig frames with segment counts U{seg_range} and label counts drawn
    from `label_choices`.  Frame i is the same for any n_frames > i."""
    seed = SEED_BATCH if seed is None else seed
    rng = np.random.default_rng(seed)
    for i, s in enumerate(np.random.SeedSequence(seed).spawn(n_frames)):
        S = int(rng.integers(seg_range[0], seg_range[1] + 1))
        L = int(rng.choice(label_choices))
        yield make_arc_workload(f"batch-frame{i}", int(s.generate_state(1)[0]),
                                n_views=n_views, width=width, height=height,
                                n_segments=S, num_labels=L,
                                f=1400.0 * width / 1920.0)


def make_batch_frames(n_frames=16, seed=None, width=1920, height=1080, n_views=8,
                      seg_range=(5000, 40000), label_choices=(128, 256)):
    """Batching workload: `n_frames` independent arc-rig frames with segment
    counts U{seg_range} and label counts drawn from `label_choices`."""
    return list(iter_batch_frames(n_frames, seed, width, height, n_views, seg_range, label_choices))


def true_depth(wl: Workload, view: int):
    """Ground-truth depth of every pixel of a rendered view, measured from
    the rig's reference plane (mean centre, mean axis) like the depth
    levels; NaN where no plane is visible."""
    cam = wl.cams[view]
    pid = wl.plane_ids[view]
    planes = wl.info["planes"]
    Cr, nr = rig_reference(wl.cams)
    d = _pixel_rays(cam, 0, cam.width, 0, cam.height)
    C = cam.center
    out = np.full(pid.shape, np.nan)
    for k, pl in enumerate(planes):
        m = pid == k
        if not m.any():
            continue
        dk = d[m]
        tt = float((pl.origin - C) @ pl.normal) / (dk @ pl.normal)
        out[m] = (C[None, :] + tt[:, None] * dk - Cr[None, :]) @ nr
    return out


def truth_labels(wl: Workload):
    """Reference levels of a rendered workload: each segment's median
    ground-truth depth mapped to the nearest level in inverse depth (levels
    uniform in 1/z, level 0 at z_far), clipped to the range."""
    L = wl.num_labels
    inv_far, inv_near = 1.0 / wl.z_far, 1.0 / wl.z_near
    out = []
    for v in range(wl.n_views):
        z = true_depth(wl, v).ravel()
        seg = wl.seg[v].ravel()
        order = np.argsort(seg, kind="stable")
        bounds = np.searchsorted(seg[order], np.arange(wl.S[v] + 1))
        med = np.full(wl.S[v], np.nan)
        for s in range(wl.S[v]):
            if bounds[s + 1] > bounds[s]:
                med[s] = np.nanmedian(z[order[bounds[s]:bounds[s + 1]]])
        lab = np.rint((1.0 / med - inv_far) / (inv_near - inv_far) * (L - 1))
        out.append(np.clip(np.nan_to_num(lab, nan=0.0), 0, L - 1).astype(np.int32))
    return np.concatenate(out)


# --------------------------------------------------------------------------
# sequences with temporal change (serving)
# --------------------------------------------------------------------------
def changed_mask(seg, pid_prev, pid_cur, moved):
    """Segments whose pixels see a moved plane in either frame (ground truth
    for the temporal mask)."""
    mv = np.zeros(max(int(pid_prev.max()), int(pid_cur.max()), max(moved, default=0)) + 2, bool)
    mv[list(moved)] = True
    hit = mv[pid_prev.astype(np.int64)] | mv[pid_cur.astype(np.int64)]
    S = int(seg.max()) + 1
    return np.bincount(seg.ravel(), weights=hit.ravel(), minlength=S) > 0


def make_sequence(wl: Workload, n_frames, seed, target_rate=0.15, tries=8):
    """Frames 1.. move 2-6 seeded planes of `wl` (translation of up to 5% of
    their depth).  Returns a list of frames, each a dict with Y, U, V and the
    per-view changed masks against the previous frame (None for frame 0)."""
    rng = np.random.default_rng(seed)
    planes = [Plane(p.origin.copy(), p.normal, p.a1, p.a2, p.half1, p.half2, p.texel, p.tex)
              for p in wl.info["planes"]]
    frames = [dict(Y=wl.Y, U=wl.U, V=wl.V, pid=wl.plane_ids, mask=None, rate=1.0)]
    Cr, nr = rig_reference(wl.cams)
    for _ in range(1, n_frames):
        best = None
        for _ in range(tries):
            k = int(rng.integers(2, 7))
            moved = sorted(rng.choice(np.arange(1, len(planes)), size=min(k, len(planes) - 1),
                                      replace=False).tolist())
            cand = [Plane(p.origin.copy(), p.normal, p.a1, p.a2, p.half1, p.half2, p.texel, p.tex)
                    for p in planes]
            for j in moved:
                z = float((cand[j].origin - Cr) @ nr)
                cand[j].origin = cand[j].origin + rng.uniform(-0.05, 0.05, 3) * max(z, 1.0)
            Y, U, V, P = _render_all(cand, wl.cams, wl.bit_depth, wl.chroma_shift)
            masks = [changed_mask(s, pp, pc, moved) for s, pp, pc in zip(wl.seg, frames[-1]["pid"], P)]
            rate = float(np.mean(np.concatenate(masks)))
            if best is None or abs(rate - target_rate) < abs(best[0] - target_rate):
                best = (rate, cand, dict(Y=Y, U=U, V=V, pid=P, mask=masks, rate=rate, moved=moved))
            if abs(rate - target_rate) < 0.03:
                break
        planes = best[1]
        frames.append(best[2])
    return frames
