"""Small seeded problems shared by the oracle pins and the GPU parity tests."""
from __future__ import annotations

import json
import math
import os
from types import SimpleNamespace

import numpy as np

from paper_1909_02294_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def cam(K, R, t, w, h):
    return synth.Camera(np.asarray(K, float), np.asarray(R, float), np.asarray(t, float), w, h)


def rotation(axis, deg):
    a = np.asarray(axis, float)
    a = a / np.linalg.norm(a)
    th = math.radians(deg)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * K @ K


def random_images(rng, cams, bit_depth, chroma_shift):
    hi = (1 << bit_depth) - 1
    dt = np.uint8 if bit_depth <= 8 else np.uint16
    Y, U, V = [], [], []
    for c in cams:
        w, h = c.width, c.height
        wc, hc = (w + chroma_shift) >> chroma_shift, (h + chroma_shift) >> chroma_shift
        Y.append(rng.integers(0, hi + 1, (h, w)).astype(dt))
        U.append(rng.integers(0, hi + 1, (hc, wc)).astype(dt))
        V.append(rng.integers(0, hi + 1, (hc, wc)).astype(dt))
    return Y, U, V


def random_segments(rng, w, h, n):
    m, S = synth.voronoi(w, h, n, rng)
    return m, S


def tiny_problem(seed, n_views=3, width=12, height=8, n_seg=6, L=5, bit_depth=8,
                 chroma_shift=0, bilinear=False, rotated=False, f=10.37):
    """A few views of a tiny random image set with a rectified or a rotated
    (converging) rig, for brute-force checks.  The default focal length keeps
    rectified disparities away from exact half pixels, where nearest
    sampling would depend on the last bit of the projection."""
    rng = np.random.default_rng(seed)
    if rotated:
        cams = synth.arc_rig(n_views, radius=2.0, arc_deg=20.0, f=f, width=width, height=height)
        # perturb every camera a little so no symmetry hides an index mistake
        out = []
        for c in cams:
            Rp = rotation(rng.normal(size=3), rng.uniform(0.5, 2.0)) @ c.R
            C = c.center + rng.normal(scale=0.01, size=3)
            K = c.K.copy()
            K[0, 0] *= rng.uniform(0.95, 1.05)
            K[1, 1] *= rng.uniform(0.95, 1.05)
            K[0, 1] = rng.uniform(-0.05, 0.05)
            out.append(cam(K, Rp, -Rp @ C, width, height))
        cams = out
        z_near, z_far = 1.0, 4.0
    else:
        cams = synth.rectified_rig(n_views, 0.1, f, width, height)
        z_near, z_far = 0.5, 3.0
    Y, U, V = random_images(rng, cams, bit_depth, chroma_shift)
    seg, S = [], []
    for _ in cams:
        m, s = random_segments(rng, width, height, n_seg)
        seg.append(m)
        S.append(s)
    return SimpleNamespace(cams=cams, Y=Y, U=U, V=V, seg=seg, S=S, bit_depth=bit_depth,
                           chroma_shift=chroma_shift, z_near=z_near, z_far=z_far,
                           num_labels=L, bilinear=bilinear)


def hand_case_problem(case_index):
    with open(os.path.join(GOLDEN, "hand_two_view.json")) as fh:
        g = json.load(fh)
    w, h, f = g["width"], g["height"], g["f"]
    K = [[f, 0, (w - 1) / 2], [0, f, (h - 1) / 2], [0, 0, 1]]
    cams = [cam(K, np.eye(3), [-cx, 0, 0], w, h) for cx in g["centres_x"]]
    Y = [np.array([v["Y"]], np.uint8) for v in g["views"]]
    U = [np.array([v["U"]], np.uint8) for v in g["views"]]
    V = [np.array([v["V"]], np.uint8) for v in g["views"]]
    seg = [np.arange(w, dtype=np.int32)[None, :] for _ in cams]
    c = g["cases"][case_index]
    pb = SimpleNamespace(cams=cams, Y=Y, U=U, V=V, seg=seg, S=[w, w], bit_depth=g["bit_depth"],
                         chroma_shift=0, z_near=c["z_near"], z_far=c["z_far"], num_labels=1,
                         bilinear=c["sampling"] == "bilinear")
    return pb, np.array(c["expected"])


def fronto_plane_views(rng, cams, f, baseline_x, shifts, bit_depth=8, width=None, height=None):
    """Views of one full-frame fronto-parallel textured plane whose disparity
    between view c and the texture frame is the integer shifts[c]: view c
    pixel (x, y) shows texture column x + shifts[c]."""
    w = width or cams[0].width
    h = height or cams[0].height
    lo, hi = 16, (235 << (bit_depth - 8))
    pad = int(max(abs(s) for s in shifts)) + 2
    tex = rng.integers(lo, hi, (3, h, w + 2 * pad))
    dt = np.uint8 if bit_depth <= 8 else np.uint16
    Y, U, V = [], [], []
    for s in shifts:
        sl = tex[:, :, pad + s: pad + s + w]
        Y.append(sl[0].astype(dt)); U.append(sl[1].astype(dt)); V.append(sl[2].astype(dt))
    return Y, U, V


def blocky_problem(seed, sizes, n_ids, bit_depth=10, chroma_shift=1):
    """Views whose label maps are random small rectangles with ids drawn
    from n_ids (some ids never drawn, so some segments are empty) plus a few
    single pixels, over random images."""
    rng = np.random.default_rng(seed)
    cams, seg, S = [], [], []
    for (w, h), n in zip(sizes, n_ids):
        K = [[6.0, 0, (w - 1) / 2], [0, 6.0, (h - 1) / 2], [0, 0, 1]]
        cams.append(cam(K, np.eye(3), [-0.05 * len(cams), 0, 0], w, h))
        bw, bh = rng.integers(1, 4), rng.integers(1, 4)
        blocks = rng.integers(0, n, ((h + bh - 1) // bh, (w + bw - 1) // bw))
        m = np.kron(blocks, np.ones((bh, bw), np.int64))[:h, :w]
        for _ in range(3):
            m[rng.integers(0, h), rng.integers(0, w)] = rng.integers(0, n)
        seg.append(m.astype(np.int32))
        S.append(int(n))
    Y, U, V = random_images(rng, cams, bit_depth, chroma_shift)
    return SimpleNamespace(cams=cams, Y=Y, U=U, V=V, seg=seg, S=S, bit_depth=bit_depth, chroma_shift=chroma_shift,
                           z_near=1.0, z_far=3.0, num_labels=6)


def islands_problem(seed, width=160, height=96, n_islands=300):
    """One background segment holding many small islands (single pixels and
    2 x 2 blocks), in two views: a segment with hundreds of pixels and
    hundreds of neighbours."""
    rng = np.random.default_rng(seed)
    cams, seg, S = [], [], []
    for v in range(2):
        K = [[80.0, 0, (width - 1) / 2], [0, 80.0, (height - 1) / 2], [0, 0, 1]]
        cams.append(cam(K, np.eye(3), [-0.05 * v, 0, 0], width, height))
        m = np.zeros((height, width), np.int32)
        ys = rng.choice(np.arange(1, height - 2, 3), n_islands)
        xs = rng.choice(np.arange(1, width - 2, 3), n_islands)
        for i, (y, x) in enumerate(zip(ys, xs)):
            if i % 2:
                m[y:y + 2, x:x + 2] = i + 1
            else:
                m[y, x] = i + 1
        seg.append(m)
        S.append(n_islands + 3)                 # two ids never used
    Y, U, V = random_images(rng, cams, 8, 0)
    return SimpleNamespace(cams=cams, Y=Y, U=U, V=V, seg=seg, S=S, bit_depth=8, chroma_shift=0,
                           z_near=1.0, z_far=3.0, num_labels=6)


def random_energy_terms(seed, rows=9, L=4, p_hit=0.6, adj=True, unary=True, fixed=None, quantum=64.0,
                        m_high=60.0):
    """Terms of a random Eq. (1) instance: two views of rows/2 segments,
    window hits into the other view, random adjacency inside each view,
    weights and values exact in FP32."""
    rng = np.random.default_rng(seed)
    half = rows // 2
    view = np.array([0] * half + [1] * (rows - half))
    hit = np.full((rows, 2, L), -1, np.int32)
    m = rng.uniform(0, m_high, (rows, 2, L)).astype(np.float32)
    for r in range(rows):
        others = np.nonzero(view != view[r])[0]
        slot = 1 if view[r] == 0 else 0
        take = rng.random(L) < p_hit
        hit[r, slot, take] = rng.choice(others, int(take.sum()))
    U = rng.uniform(0, 20, (rows, L)).astype(np.float32) if unary else None
    off = idx = beta = None
    if adj:
        lists = [[] for _ in range(rows)]
        w = {}
        for v in (0, 1):
            ids = np.nonzero(view == v)[0]
            for a in ids:
                for b in ids:
                    if a < b and rng.random() < min(1.0, 4.0 / max(1, len(ids))):
                        lists[a].append(b)
                        lists[b].append(a)
                        w[(a, b)] = w[(b, a)] = np.float32(rng.uniform(0.5, 8))
        off = np.concatenate([[0], np.cumsum([len(x) for x in lists])]).astype(np.int64)
        idx = np.array([t for r in range(rows) for t in sorted(lists[r])], np.int32)
        beta = np.array([w[(r, t)] for r in range(rows) for t in sorted(lists[r])], np.float32)
    return dict(rows=rows, num_labels=L, unary=U, m=m, hit=hit, K=30.0, offsets=off, index=idx, beta=beta,
                fixed=fixed, quantum=quantum)


def facing_problem(seed, width=12, height=8, n_seg=6, L=5, bit_depth=8, chroma_shift=0, bilinear=False):
    """Four cameras placed so that 3-D points fall behind cameras (the paper's
    cameras are arbitrarily positioned, Sec. III-A): views 0 and 1 look along
    +z from near the origin, view 2 looks back at them from z = 3.2 (level
    points beyond it lie behind it), and view 3 looks along +z from z = 3.0,
    among the level planes (levels nearer than its own position give
    tau <= 0 for its pixels).  Random images and Voronoi segments."""
    rng = np.random.default_rng(seed)
    f = 1.1 * width
    cams = [
        synth.look_at([0.0, 0.0, 0.0], [0.0, 0.0, 5.0], width, height, f),
        synth.look_at([0.3, 0.0, 0.1], [0.0, 0.0, 4.0], width, height, f * 1.03),
        synth.look_at([0.15, 0.05, 3.2], [0.1, 0.0, 0.0], width, height, f * 0.97),
        synth.look_at([-0.25, 0.02, 3.0], [0.0, 0.0, 8.0], width, height, f),
    ]
    Y, U, V = random_images(rng, cams, bit_depth, chroma_shift)
    seg, S = [], []
    for _ in cams:
        m, s = random_segments(rng, width, height, n_seg)
        seg.append(m)
        S.append(s)
    return SimpleNamespace(cams=cams, Y=Y, U=U, V=V, seg=seg, S=S, bit_depth=bit_depth,
                           chroma_shift=chroma_shift, z_near=1.0, z_far=4.5, num_labels=L, bilinear=bilinear)


def behind_geometry(ns, depth_ref="rig"):
    """FP64 geometry of every (view, pixel, label, target) sample, computed
    here with numpy and independently of both implementations: per view the
    share of (pixel, label) whose level point has tau <= 0; the share of
    (pixel, label, target) samples with tau > 0 behind the target
    (camera-frame z <= 0); and how many of those behind-target samples would
    land inside the target if the sign of z were ignored (so the test of the
    sign decides their validity)."""
    n = len(ns.cams)
    centres = np.array([c.center for c in ns.cams])
    axes = np.array([c.axis for c in ns.cams])
    if depth_ref == "rig":
        Cr_all = np.repeat(centres.mean(0)[None], n, 0)
        a = axes.mean(0)
        nr_all = np.repeat((a / np.linalg.norm(a))[None], n, 0)
    elif depth_ref == "own":
        Cr_all, nr_all = centres, axes
    else:
        Cr_all = np.repeat(centres[int(depth_ref)][None], n, 0)
        nr_all = np.repeat(axes[int(depth_ref)][None], n, 0)
    rho = 1 / ns.z_far + np.arange(ns.num_labels) / max(ns.num_labels - 1, 1) * (1 / ns.z_near - 1 / ns.z_far)
    z = 1 / rho
    out = dict(tau_nonpos=[], behind=0, behind_flip_inside=0, samples=0)
    for c, cam_c in enumerate(ns.cams):
        h, w = cam_c.height, cam_c.width
        ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
        p = np.stack([xs.ravel(), ys.ravel(), np.ones(h * w)])
        d = (cam_c.R.T @ np.linalg.inv(cam_c.K) @ p).T                  # (P, 3)
        nd = d @ nr_all[c]
        tau = (z[None, :] - (centres[c] - Cr_all[c]) @ nr_all[c]) / nd[:, None]   # (P, L)
        out["tau_nonpos"].append(float((tau <= 0).mean()))
        X = centres[c][None, None, :] + tau[..., None] * d[:, None, :]              # (P, L, 3)
        for c2, cam_t in enumerate(ns.cams):
            if c2 == c:
                continue
            Xc = X @ cam_t.R.T + cam_t.t
            front = tau > 0
            behind = front & (Xc[..., 2] <= 0)
            hh = Xc @ cam_t.K.T
            with np.errstate(divide="ignore", invalid="ignore"):
                u, v = hh[..., 0] / hh[..., 2], hh[..., 1] / hh[..., 2]
            inside = (u >= 0) & (u <= cam_t.width - 1) & (v >= 0) & (v <= cam_t.height - 1)
            out["samples"] += tau.size
            out["behind"] += int(behind.sum())
            out["behind_flip_inside"] += int((behind & inside).sum())
    out["behind_share"] = out["behind"] / max(out["samples"], 1)
    return out
