"""CPU oracle of the per-segment plane-sweep matching cost volume.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The GPU library never loads it,
and it shares no code, header or table with the GPU library.

Two independent implementations live here:
  * oracle.c  -- FP64 C with OpenMP, ray-plane intersection per pixel and
    label (the paper's inter-view matching core, Sec. III-C Eq. (4), taken
    over every pixel of a segment, minimum over target views);
  * brute.py  -- pure-Python loops for tiny inputs, used to check oracle.c.

Every function here is pinned by tests against closed forms, exact
zero-cost scenes, invariants and hand-derived values (tests/test_oracle_*.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

# depth reference selectors (match the C convention)
REF_RIG_CENTER = -1
REF_OWN = -2


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                        "-shared", "-fPIC", "-std=c11", "-Wall", "-Wextra",
                        "-o", tmp, SRC, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_views", ctypes.c_int32),
        ("K", ctypes.POINTER(ctypes.c_double)),
        ("R", ctypes.POINTER(ctypes.c_double)),
        ("t", ctypes.POINTER(ctypes.c_double)),
        ("width", ctypes.POINTER(ctypes.c_int32)),
        ("height", ctypes.POINTER(ctypes.c_int32)),
        ("planes", ctypes.POINTER(ctypes.c_void_p)),
        ("pitch", ctypes.POINTER(ctypes.c_int64)),
        ("bit_depth", ctypes.c_int32),
        ("chroma_shift", ctypes.c_int32),
        ("seg", ctypes.POINTER(ctypes.c_void_p)),
        ("num_segments", ctypes.POINTER(ctypes.c_int32)),
        ("z_near", ctypes.c_double),
        ("z_far", ctypes.c_double),
        ("num_labels", ctypes.c_int32),
        ("depth_ref", ctypes.c_int32),
        ("bilinear", ctypes.c_int32),
        ("targets", ctypes.POINTER(ctypes.c_uint8)),
    ]


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB)
        lib.oracle_cost_rows.restype = ctypes.c_int
        lib.oracle_cost_rows.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        lib.oracle_segment_stats.restype = ctypes.c_int
        lib.oracle_segment_stats.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_window_rows.restype = ctypes.c_int
        lib.oracle_window_rows.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads for the following calls (for timing; no result depends on it)."""
    load().oracle_set_num_threads(int(n))


def target_matrix(n_views: int, targets="all", explicit=None) -> np.ndarray:
    """n x n uint8 matrix; row c marks the target views of view c.

    "all": every other view.  "nearest_lr": the nearest left and right views
    by index (Sec. III-B: the two neighbouring views; the end views get one).
    "explicit": the given matrix (the diagonal is ignored)."""
    T = np.zeros((n_views, n_views), np.uint8)
    if targets == "all":
        T[:] = 1
    elif targets == "nearest_lr":
        for c in range(n_views):
            if c > 0:
                T[c, c - 1] = 1
            if c + 1 < n_views:
                T[c, c + 1] = 1
    elif targets == "explicit":
        T[:] = np.asarray(explicit, np.uint8) != 0
    else:
        raise ValueError(targets)
    np.fill_diagonal(T, 0)
    return T


class Problem:
    """Host-side description of one cost-volume problem for the oracle.

    cams: objects with K, R, t (float64 arrays), width, height.
    Y, U, V: per-view 2-D unsigned integer arrays (chroma subsampled by
    chroma_shift).  seg: per-view int32 H x W maps; S: segment counts."""

    def __init__(self, cams, Y, U, V, seg, S, bit_depth, chroma_shift, z_near, z_far,
                 num_labels, bilinear, depth_ref=REF_RIG_CENTER, targets="all", target_explicit=None):
        self.cams, self.Y, self.U, self.V = list(cams), list(Y), list(U), list(V)
        self.seg, self.S = [np.ascontiguousarray(s, np.int32) for s in seg], [int(x) for x in S]
        self.bit_depth, self.chroma_shift = int(bit_depth), int(chroma_shift)
        self.z_near, self.z_far, self.num_labels = float(z_near), float(z_far), int(num_labels)
        self.bilinear, self.depth_ref = bool(bilinear), int(depth_ref)
        n = len(self.cams)
        self.T = target_matrix(n, targets, target_explicit)

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.cams, wl.Y, wl.U, wl.V, wl.seg, wl.S, wl.bit_depth, wl.chroma_shift,
                   wl.z_near, wl.z_far, wl.num_labels, wl.bilinear, **kw)

    @property
    def n_views(self):
        return len(self.cams)

    def row_offsets(self):
        return np.concatenate([[0], np.cumsum(self.S)]).astype(np.int64)


def _c_problem(pb: Problem):
    """The C view of a Problem; returns (struct, keep-alive list)."""
    n, L = pb.n_views, pb.num_labels
    dt = np.uint8 if pb.bit_depth <= 8 else np.uint16
    keep = []

    def arr(a, dtype):
        a = np.ascontiguousarray(a, dtype)
        keep.append(a)
        return a

    K = arr(np.stack([c.K for c in pb.cams]), np.float64)
    R = arr(np.stack([c.R for c in pb.cams]), np.float64)
    t = arr(np.stack([c.t for c in pb.cams]), np.float64)
    W = arr([c.width for c in pb.cams], np.int32)
    H = arr([c.height for c in pb.cams], np.int32)
    planes = (ctypes.c_void_p * (3 * n))()
    pitch = arr(np.zeros(3 * n), np.int64)
    for v in range(n):
        for ch, P in enumerate((pb.Y[v], pb.U[v], pb.V[v])):
            P = arr(P, dt)
            planes[3 * v + ch] = P.ctypes.data
            pitch[3 * v + ch] = P.shape[1]
    segp = (ctypes.c_void_p * n)()
    for v in range(n):
        m = arr(pb.seg[v], np.int32)
        if m.shape != (pb.cams[v].height, pb.cams[v].width):
            raise ValueError("segment map shape does not match the camera")
        segp[v] = m.ctypes.data
    S = arr(pb.S, np.int32)
    T = arr(pb.T, np.uint8)
    prob = _Problem(n, K.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    R.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                    W.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    H.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    ctypes.cast(planes, ctypes.POINTER(ctypes.c_void_p)),
                    pitch.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                    pb.bit_depth, pb.chroma_shift,
                    ctypes.cast(segp, ctypes.POINTER(ctypes.c_void_p)),
                    S.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                    pb.z_near, pb.z_far, L, pb.depth_ref, int(pb.bilinear),
                    T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    keep.extend([planes, segp])
    return prob, keep


def cost_rows(pb: Problem, views, segs, with_terms=False):
    """C rows (float64, len(views) x L) for the (view, segment) pairs; with
    with_terms also the per-target means m (NaN where nothing is valid) and
    valid counts, both len(views) x n x L."""
    lib = load()
    n, L = pb.n_views, pb.num_labels
    prob, keep = _c_problem(pb)

    def arr(a, dtype):
        a = np.ascontiguousarray(a, dtype)
        keep.append(a)
        return a

    rv = arr(views, np.int32)
    rs = arr(segs, np.int32)
    nr = len(rv)
    cost = np.empty((nr, L), np.float64)
    m = np.empty((nr, n, L), np.float64) if with_terms else None
    nv = np.empty((nr, n, L), np.int64) if with_terms else None
    rc = lib.oracle_cost_rows(ctypes.byref(prob), nr, rv.ctypes.data, rs.ctypes.data, cost.ctypes.data,
                              m.ctypes.data if with_terms else None,
                              nv.ctypes.data if with_terms else None)
    if rc != 0:
        raise ValueError(f"oracle_cost_rows failed with status {rc}")
    return (cost, m, nv) if with_terms else cost


def all_rows(pb: Problem):
    views = np.concatenate([np.full(s, v, np.int32) for v, s in enumerate(pb.S)])
    segs = np.concatenate([np.arange(s, dtype=np.int32) for s in pb.S])
    return views, segs


def cost_volume(pb: Problem, with_terms=False):
    """The whole volume, rows in [view][segment] order, labels contiguous."""
    return cost_rows(pb, *all_rows(pb), with_terms=with_terms)


def argmin(C) -> np.ndarray:
    """Lowest label attaining each row's minimum."""
    return np.argmin(np.asarray(C), axis=-1).astype(np.int32)


def served(prev, pb: Problem, changed):
    """Frame cost after a temporal update: rows marked changed are
    recomputed, the others keep the previous frame's cost (Sec. III-E:
    unchanged segments adopt the earlier result).  prev None: every row."""
    if prev is None:
        return cost_volume(pb)
    out = np.array(prev, np.float64, copy=True)
    changed = np.asarray(changed, bool)
    idx = np.nonzero(changed)[0]
    if len(idx):
        off = pb.row_offsets()
        views = (np.searchsorted(off, idx, side="right") - 1).astype(np.int32)
        segs = (idx - off[views]).astype(np.int32)
        out[idx] = cost_rows(pb, views, segs)
    return out


def segment_stats(pb: Problem, view: int):
    """(count [S], centre [S, 2] int, mean YCbCr [S, 3]) of one view: the
    segment centre mu_s of Sec. III-C is the centroid rounded half up."""
    lib = load()
    prob, keep = _c_problem(pb)
    S = pb.S[view]
    cnt = np.empty(S, np.int64)
    cen = np.empty((S, 2), np.int32)
    mean = np.empty((S, 3), np.float64)
    rc = lib.oracle_segment_stats(ctypes.byref(prob), int(view), cnt.ctypes.data, cen.ctypes.data, mean.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_segment_stats failed with status {rc}")
    return cnt, cen, mean


def window_rows(pb: Problem, views, segs, radius=1, with_uv=False):
    """Eq. (4) of Sec. III-C at the segment centre towards views c - 1 (slot 0)
    and c + 1 (slot 1): m [n, 2, L] in 8-bit code values (NaN where there is
    no match), hit [n, 2, L] the matched segment's volume row (-1), and with
    with_uv the projected centre [n, 2, L, 2]."""
    lib = load()
    prob, keep = _c_problem(pb)
    rv = np.ascontiguousarray(views, np.int32)
    rs = np.ascontiguousarray(segs, np.int32)
    nr, L = len(rv), pb.num_labels
    m = np.empty((nr, 2, L), np.float64)
    hit = np.empty((nr, 2, L), np.int64)
    uv = np.empty((nr, 2, L, 2), np.float64) if with_uv else None
    rc = lib.oracle_window_rows(ctypes.byref(prob), nr, rv.ctypes.data, rs.ctypes.data, int(radius), m.ctypes.data,
                                hit.ctypes.data, uv.ctypes.data if with_uv else None)
    if rc != 0:
        raise ValueError(f"oracle_window_rows failed with status {rc}")
    return (m, hit, uv) if with_uv else (m, hit)


def window_energy(m, hit, labelling, K=30.0):
    """Eq. (5) summed over the neighbouring views for a fixed labelling of all
    segments: E[r, l] = sum over slots with a match of
    [labelling[hit] == l] * min(0, m - K)."""
    m = np.asarray(m, np.float64)
    hit = np.asarray(hit)
    lab = np.asarray(labelling)
    L = m.shape[2]
    E = np.zeros((m.shape[0], L))
    ok = hit >= 0
    d_hit = np.where(ok, lab[np.where(ok, hit, 0)], -1)
    same = d_hit == np.arange(L)[None, None, :]
    E += np.where(ok & same, np.minimum(0.0, m - K), 0.0).sum(axis=1)
    return E


def temporal_rule(mean, mean_prev, mean_iframe=None, t_p=3.0, t_i=1.0, bit_depth=8):
    """Sec. III-E: a segment is unchanged when every component of its mean
    Y, Cb, Cr moved by less than T_I against the I frame (source 2: adopt the
    I frame's result) or by less than T_P against the previous frame (source
    1: keep the previous result); else it is recomputed (0).  Thresholds are
    in 8-bit code values, scaled by 2^(b - 8).  The stricter I-frame test is
    taken first."""
    s = float(1 << (bit_depth - 8))
    mean = np.asarray(mean, np.float64)[:, :3]
    dp = np.abs(mean - np.asarray(mean_prev, np.float64)[:, :3]).max(axis=1)
    src = np.where(dp < t_p * s, 1, 0)
    if mean_iframe is not None:
        di = np.abs(mean - np.asarray(mean_iframe, np.float64)[:, :3]).max(axis=1)
        src = np.where(di < t_i * s, 2, src)
    return src.astype(np.uint8)


def served_rule(prev, iframe_cost, pb: Problem, source):
    """One temporally updated frame: rows with source 0 are recomputed, 1
    keep prev, 2 take the I frame's row (Sec. III-E: unchanged segments adopt
    the earlier depth)."""
    out = np.array(prev, np.float64, copy=True)
    source = np.asarray(source)
    out[source == 2] = np.asarray(iframe_cost, np.float64)[source == 2]
    idx = np.nonzero(source == 0)[0]
    if len(idx):
        off = pb.row_offsets()
        views = (np.searchsorted(off, idx, side="right") - 1).astype(np.int32)
        out[idx] = cost_rows(pb, views, (idx - off[views]).astype(np.int32))
    return out


def all_segment_stats(pb: Problem):
    """Counts, centres and mean colours of every row, in volume order."""
    parts = [segment_stats(pb, v) for v in range(pb.n_views)]
    return (np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
            np.concatenate([p[2] for p in parts]))


# ---------------------------------------------------------------- intra-view term (Sec. III-D)

def adjacency(pb: Problem):
    """T(s) of Eq. (1) and Sec. III-D: the segments of the same view adjacent
    to s.  Two segments are adjacent when a pixel of one is a 4-neighbour
    (left, right, above, below) of a pixel of the other.  Returned as CSR over
    volume rows: offsets [rows + 1] and index [edges] (volume rows), each
    list increasing; every adjacent pair appears in both lists."""
    off = pb.row_offsets()
    total = int(off[-1])
    src, dst = [np.zeros(0, np.int64)], [np.zeros(0, np.int64)]
    for v in range(pb.n_views):
        seg = pb.seg[v].astype(np.int64)
        if seg.size and (seg.min() < 0 or seg.max() >= pb.S[v]):
            raise ValueError(f"view {v}: segment id out of range")
        for a, b in ((seg[:, :-1], seg[:, 1:]), (seg[:-1, :], seg[1:, :])):
            a, b = a.ravel(), b.ravel()
            k = a != b
            src += [a[k] + off[v], b[k] + off[v]]
            dst += [b[k] + off[v], a[k] + off[v]]
    key = np.unique(np.concatenate(src) * max(total, 1) + np.concatenate(dst))
    s, t = key // max(total, 1), key % max(total, 1)
    offsets = np.zeros(total + 1, np.int64)
    offsets[1:] = np.cumsum(np.bincount(s, minlength=total))
    return offsets, t.astype(np.int64)


def edge_rows(offsets):
    """The segment (volume row) owning each CSR entry."""
    offsets = np.asarray(offsets, np.int64)
    return np.repeat(np.arange(len(offsets) - 1, dtype=np.int64), np.diff(offsets))


def smoothing_beta(mean, offsets, index, beta0, bit_depth, eps=1.0):
    """Eq. (3) per CSR entry (s, t): beta0 / (||mean_s - mean_t||_1 + eps),
    the L1 distance of the segments' mean Y, Cb, Cr in 8-bit code values
    (differences divided by 2^(b - 8)).  eps = 1 code value keeps segments of
    identical colour finite, where Eq. (3) itself would divide by zero."""
    mean = np.asarray(mean, np.float64)[:, :3]
    s = edge_rows(offsets)
    t = np.asarray(index, np.int64)
    d = np.abs(mean[s] - mean[t]).sum(axis=1) / float(1 << (bit_depth - 8))
    return float(beta0) / (d + float(eps))


def intra_cost(offsets, index, beta, labelling, num_labels, fixed=None):
    """Eq. (2) seen from segment s at label l with its neighbours' labels
    held: U[s, l] = sum over t in T(s) of beta_st * |l - d_t|, depths in
    label units.  With a mask `fixed`, only neighbours t with fixed[t] count
    (segments left out of the optimisation still enter the costs of their
    neighbours, Sec. III-E)."""
    s = edge_rows(offsets)
    t = np.asarray(index, np.int64)
    w = np.asarray(beta, np.float64)
    if fixed is not None:
        keep = np.asarray(fixed, bool)[t]
        s, t, w = s[keep], t[keep], w[keep]
    d_t = np.asarray(labelling, np.int64)[t]
    L = int(num_labels)
    U = np.zeros((len(offsets) - 1, L))
    np.add.at(U, s, w[:, None] * np.abs(np.arange(L)[None, :] - d_t[:, None]))
    return U


def intra_energy(offsets, index, beta, labelling):
    """The intra-view part of Eq. (1) for a labelling: the sum over s and
    t in T(s) of beta_st |d_s - d_t| (each adjacent pair counted from both
    sides, as the double sum is written)."""
    d = np.asarray(labelling, np.int64)
    s = edge_rows(offsets)
    t = np.asarray(index, np.int64)
    return float(np.sum(np.asarray(beta, np.float64) * np.abs(d[s] - d[t])))


# ---------------------------------------------------------------- depth maps

def level_depths(z_near, z_far, num_labels):
    """The depth of each level: uniform in inverse depth, level 0 at z_far
    and level L - 1 at z_near (a single level sits at z_far)."""
    L = int(num_labels)
    out = np.empty(L)
    for l in range(L):
        frac = l / (L - 1) if L > 1 else 0.0
        out[l] = 1.0 / (1.0 / z_far + frac * (1.0 / z_near - 1.0 / z_far))
    return out


def depth_map(pb: Problem, labels):
    """Per-pixel depth maps of all views (Sec. III-B: segment depths are
    painted onto their pixels): view v's pixel (x, y) gets the depth of the
    level of its segment's row; concatenated view after view, rows of W."""
    z = level_depths(pb.z_near, pb.z_far, pb.num_labels)
    off = pb.row_offsets()
    lab = np.asarray(labels, np.int64)
    return np.concatenate([z[lab[off[v] + pb.seg[v].astype(np.int64)]].ravel() for v in range(pb.n_views)])
