"""Pure-Python brute force of the segment cost volume for tiny inputs.

TEST INFRASTRUCTURE, written separately from oracle.c to check it.  It uses
Python floats and lists only, and takes the steps in the order the
definition states them:

  1. depth levels uniform in inverse depth between z_far (label 0) and
     z_near (label L-1), on planes parallel to the reference camera plane
     (Sec. IV-A; reference = rig centre camera plane, Sec. III-B);
  2. each pixel of segment s in view c is lifted to the plane of label l;
  3. the 3-D point is transformed into every target view c' (the transform
     T[.] of Sec. III-C) and that view is sampled;
  4. the YCbCr L1 distance (Eq. (4)) is averaged over the valid pixels of s,
     normalised to [0, 1], and the minimum over the target views is kept.
"""
from __future__ import annotations

import math


def _mat(a):
    return [[float(a[i][j]) for j in range(3)] for i in range(3)]


def _vec(a):
    return [float(a[i]) for i in range(3)]


def _mv(M, v):
    return [M[i][0] * v[0] + M[i][1] * v[1] + M[i][2] * v[2] for i in range(3)]


def _mtv(M, v):
    return [M[0][i] * v[0] + M[1][i] * v[1] + M[2][i] * v[2] for i in range(3)]


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _k_inverse_pixel(K, x, y):
    """K^-1 [x, y, 1] for upper-triangular K (back substitution)."""
    z = 1.0
    yy = (y - K[1][2] * z) / K[1][1]
    xx = (x - K[0][1] * yy - K[0][2] * z) / K[0][0]
    return [xx, yy, z]


def cost_volume(cams, Y, U, V, seg, S, bit_depth, chroma_shift, z_near, z_far, L,
                bilinear, targets, depth_ref="rig"):
    """Rows in [view][segment] order, each a list of L floats.

    targets[c][c2] truthy marks c2 as a target view of c.  depth_ref: "rig"
    (mean centre, normalised mean axis), "own", or a camera index."""
    n = len(cams)
    k = chroma_shift
    maxv = float((1 << bit_depth) - 1)
    Ks = [_mat(c.K) for c in cams]
    Rs = [_mat(c.R) for c in cams]
    ts = [_vec(c.t) for c in cams]
    centres = [[-v for v in _mtv(Rs[i], ts[i])] for i in range(n)]
    axes = [list(Rs[i][2]) for i in range(n)]

    def ref_plane(c):
        if depth_ref == "rig":
            Cr = [sum(centres[i][j] for i in range(n)) / n for j in range(3)]
            a = [sum(axes[i][j] for i in range(n)) / n for j in range(3)]
            ln = math.sqrt(_dot(a, a))
            return Cr, [v / ln for v in a]
        i = c if depth_ref == "own" else int(depth_ref)
        return centres[i], axes[i]

    depths = []
    for l in range(L):
        f = l / (L - 1) if L > 1 else 0.0
        depths.append(1.0 / (1.0 / z_far + f * (1.0 / z_near - 1.0 / z_far)))

    def px(plane, x, y):
        return float(plane[y][x])

    def sample(c2, u, v):
        W2, H2 = cams[c2].width, cams[c2].height
        if not bilinear:
            xi, yi = math.floor(u + 0.5), math.floor(v + 0.5)
            if not (0 <= xi < W2 and 0 <= yi < H2):
                return None
            return (px(Y[c2], xi, yi), px(U[c2], xi >> k, yi >> k), px(V[c2], xi >> k, yi >> k))
        edge = 1.0 / 64.0    # samples within 1/64 px outside the image are clamped in
        if not (-edge <= u <= W2 - 1 + edge and -edge <= v <= H2 - 1 + edge):
            return None
        u, v = min(max(u, 0.0), W2 - 1.0), min(max(v, 0.0), H2 - 1.0)
        x0, y0 = math.floor(u), math.floor(v)
        ax, ay = u - x0, v - y0
        x1, y1 = min(x0 + 1, W2 - 1), min(y0 + 1, H2 - 1)
        taps = [(x0, y0, (1 - ax) * (1 - ay)), (x1, y0, ax * (1 - ay)),
                (x0, y1, (1 - ax) * ay), (x1, y1, ax * ay)]
        out = []
        for plane, sh in ((Y[c2], 0), (U[c2], k), (V[c2], k)):
            out.append(sum(w * px(plane, xx >> sh, yy >> sh) for xx, yy, w in taps))
        return tuple(out)

    rows = []
    for c in range(n):
        Cr, nr = ref_plane(c)
        Cc = centres[c]
        H, W = len(seg[c]), len(seg[c][0])
        members = [[] for _ in range(S[c])]
        for y in range(H):
            for x in range(W):
                members[int(seg[c][y][x])].append((x, y))
        for s in range(S[c]):
            row = []
            for l in range(L):
                best = None
                for c2 in range(n):
                    if c2 == c or not targets[c][c2]:
                        continue
                    total, count = 0.0, 0
                    for (x, y) in members[s]:
                        d = _mtv(Rs[c], _k_inverse_pixel(Ks[c], x, y))
                        tau = (depths[l] - _dot(nr, [Cc[j] - Cr[j] for j in range(3)])) / _dot(nr, d)
                        if not tau > 0:
                            continue
                        X = [Cc[j] + tau * d[j] for j in range(3)]
                        Xc = [a + b for a, b in zip(_mv(Rs[c2], X), ts[c2])]
                        if not Xc[2] > 0:
                            continue
                        h = _mv(Ks[c2], Xc)
                        got = sample(c2, h[0] / h[2], h[1] / h[2])
                        if got is None:
                            continue
                        ref = (px(Y[c], x, y), px(U[c], x >> k, y >> k), px(V[c], x >> k, y >> k))
                        total += sum(abs(a - b) for a, b in zip(ref, got)) / (3.0 * maxv)
                        count += 1
                    if count:
                        m = total / count
                        best = m if best is None or m < best else best
                row.append(1.0 if best is None else best)
            rows.append(row)
    return rows


def segment_centres(seg, S):
    """Centroid of each segment's pixel coordinates, rounded half up."""
    sx, sy, n = [0] * S, [0] * S, [0] * S
    for y, row in enumerate(seg):
        for x, s in enumerate(row):
            s = int(s)
            sx[s] += x
            sy[s] += y
            n[s] += 1
    return [(math.floor(sx[s] / n[s] + 0.5), math.floor(sy[s] / n[s] + 0.5)) if n[s] else None for s in range(S)]


def window_cost(cams, Y, U, V, seg, S, bit_depth, chroma_shift, z_near, z_far, L, radius, depth_ref="rig"):
    """Eq. (4) at each segment centre towards the views c - 1 and c + 1:
    returns (m, hit) as nested lists [row][slot][label]; m in 8-bit code
    values or None, hit the matched segment's volume row or -1."""
    n = len(cams)
    k = chroma_shift
    scale = float(1 << (bit_depth - 8))
    Ks = [_mat(c.K) for c in cams]
    Rs = [_mat(c.R) for c in cams]
    ts = [_vec(c.t) for c in cams]
    centres = [[-v for v in _mtv(Rs[i], ts[i])] for i in range(n)]
    axes = [list(Rs[i][2]) for i in range(n)]
    row0 = [sum(S[:i]) for i in range(n)]
    if depth_ref == "rig":
        Cr = [sum(centres[i][j] for i in range(n)) / n for j in range(3)]
        a = [sum(axes[i][j] for i in range(n)) / n for j in range(3)]
        ln = math.sqrt(_dot(a, a))
        nr = [v / ln for v in a]
    depths = [1.0 / (1.0 / z_far + (l / (L - 1) if L > 1 else 0.0) * (1.0 / z_near - 1.0 / z_far)) for l in range(L)]

    def pix(luma, plane, sh, x, y):
        # clamp to the image (luma size), then read the plane at its resolution
        h, w = len(luma), len(luma[0])
        x = min(max(x, 0), w - 1)
        y = min(max(y, 0), h - 1)
        return float(plane[y >> sh][x >> sh])

    ms, hits = [], []
    for c in range(n):
        if depth_ref != "rig":
            i = c if depth_ref == "own" else int(depth_ref)
            Cr, nr = centres[i], axes[i]
        mus = segment_centres(seg[c], S[c])
        for s in range(S[c]):
            mrow, hrow = [], []
            for c2 in (c - 1, c + 1):
                mm, hh = [None] * L, [-1] * L
                if 0 <= c2 < n and mus[s] is not None:
                    mx, my = mus[s]
                    d = _mtv(Rs[c], _k_inverse_pixel(Ks[c], mx, my))
                    for l in range(L):
                        tau = (depths[l] - _dot(nr, [centres[c][j] - Cr[j] for j in range(3)])) / _dot(nr, d)
                        if not tau > 0:
                            continue
                        X = [centres[c][j] + tau * d[j] for j in range(3)]
                        Xc = [a + b for a, b in zip(_mv(Rs[c2], X), ts[c2])]
                        if not Xc[2] > 0:
                            continue
                        h = _mv(Ks[c2], Xc)
                        tx, ty = math.floor(h[0] / h[2] + 0.5), math.floor(h[1] / h[2] + 0.5)
                        if not (0 <= tx < cams[c2].width and 0 <= ty < cams[c2].height):
                            continue
                        tot = 0.0
                        for dy in range(-radius, radius + 1):
                            for dx in range(-radius, radius + 1):
                                for plane, sh in ((0, 0), (1, k), (2, k)):
                                    src = (Y, U, V)[plane]
                                    a_ = pix(Y[c], src[c], sh, mx + dx, my + dy)
                                    b_ = pix(Y[c2], src[c2], sh, tx + dx, ty + dy)
                                    tot += abs(a_ - b_)
                        mm[l] = tot / ((2 * radius + 1) ** 2 * scale)
                        hh[l] = row0[c2] + int(seg[c2][ty][tx])
                mrow.append(mm)
                hrow.append(hh)
            ms.append(mrow)
            hits.append(hrow)
    return ms, hits


def adjacency_sets(seg_maps, S):
    """T(s) as Python sets of (view, segment): 4-neighbour pixel contact."""
    adj = {}
    for v, seg in enumerate(seg_maps):
        h, w = len(seg), len(seg[0])
        for s in range(S[v]):
            adj[(v, s)] = set()
        for y in range(h):
            for x in range(w):
                a = int(seg[y][x])
                for dx, dy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    xx, yy = x + dx, y + dy
                    if 0 <= xx < w and 0 <= yy < h and int(seg[yy][xx]) != a:
                        adj[(v, a)].add((v, int(seg[yy][xx])))
    return adj


def intra_terms(seg_maps, S, means, beta0, bit_depth, labelling, num_labels, eps=1.0):
    """Eq. (3) weights and Eq. (2) costs by loops: returns
    (beta {(row_s, row_t): value}, U [rows][L] list, energy)."""
    off = [0]
    for s in S:
        off.append(off[-1] + s)
    adj = adjacency_sets(seg_maps, S)
    scale = float(2 ** (bit_depth - 8))
    beta = {}
    for (v, s), nb in adj.items():
        for (_, t) in nb:
            rs, rt = off[v] + s, off[v] + t
            d = sum(abs(means[rs][k] - means[rt][k]) for k in range(3)) / scale
            beta[(rs, rt)] = beta0 / (d + eps)
    rows = off[-1]
    U = [[0.0] * num_labels for _ in range(rows)]
    energy = 0.0
    for (rs, rt), b in beta.items():
        for l in range(num_labels):
            U[rs][l] += b * abs(l - labelling[rt])
        energy += b * abs(labelling[rs] - labelling[rt])
    return beta, U, energy
