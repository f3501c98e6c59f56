"""Pins of the oracle's window matching core (Sec. III-C, Eqs. (4), (5)):
a hand-derived case, the pure-Python brute force, segment centres, an exact
zero-cost plane, and the link to the full-segment cost on one-pixel
segments."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1909_02294_amd import synth
from tests import _problems as P


def _pb(ns, **kw):
    return oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift,
                          ns.z_near, ns.z_far, ns.num_labels, False, **kw)


def _hand():
    g = json.load(open(os.path.join(P.GOLDEN, "hand_window.json")))
    w, h, f = g["width"], g["height"], g["f"]
    K = [[f, 0, (w - 1) / 2], [0, f, (h - 1) / 2], [0, 0, 1]]
    cams = [P.cam(K, np.eye(3), [-cx, 0, 0], w, h) for cx in g["centres_x"]]
    Y = [np.full((h, w), v["Y"], np.uint8) for v in g["views"]]
    U = [np.full((h, w), v["U"], np.uint8) for v in g["views"]]
    V = [np.full((h, w), v["V"], np.uint8) for v in g["views"]]
    seg = [np.array(v["seg"], np.int32) for v in g["views"]]
    S = [int(s.max()) + 1 for s in seg]
    pb = oracle.Problem(cams, Y, U, V, seg, S, 8, 0, g["z_near"], g["z_far"], g["labels"], False)
    return g, pb


def test_hand_derived_window():
    g, pb = _hand()
    m, hit = oracle.window_rows(pb, *oracle.all_rows(pb), radius=1)
    want_m = np.array([[[np.nan if v is None else v for v in sl] for sl in row] for row in g["expected_m"]])
    np.testing.assert_array_equal(np.isnan(m), np.isnan(want_m))
    np.testing.assert_allclose(m[~np.isnan(m)], want_m[~np.isnan(want_m)], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(hit, np.array(g["expected_hit"]))
    E = oracle.window_energy(m, hit, g["labelling"], K=30.0)
    np.testing.assert_allclose(E, np.array(g["expected_energy"]), rtol=0, atol=1e-12)
    bm, bh = brute.window_cost(pb.cams, pb.Y, pb.U, pb.V, pb.seg, pb.S, 8, 0, pb.z_near, pb.z_far, 2, 1)
    np.testing.assert_array_equal(np.array(bh), hit)


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("chroma_shift", [0, 1])
def test_window_matches_brute_force(seed, chroma_shift):
    ns = P.tiny_problem(200 + seed, n_views=3, width=14, height=10, n_seg=7, L=6, rotated=seed % 2 == 1,
                        chroma_shift=chroma_shift, bit_depth=8 if seed < 3 else 10)
    for radius, ref, bref in ((1, oracle.REF_RIG_CENTER, "rig"), (2, oracle.REF_OWN, "own"), (0, 0, 0)):
        pb = _pb(ns, depth_ref=ref)
        m, hit = oracle.window_rows(pb, *oracle.all_rows(pb), radius=radius)
        bm, bh = brute.window_cost(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift,
                                   ns.z_near, ns.z_far, ns.num_labels, radius, depth_ref=bref)
        bm = np.array([[[np.nan if v is None else v for v in sl] for sl in row] for row in bm])
        np.testing.assert_array_equal(np.array(bh), hit)
        np.testing.assert_array_equal(np.isnan(bm), np.isnan(m))
        np.testing.assert_allclose(m[~np.isnan(m)], bm[~np.isnan(bm)], rtol=0, atol=1e-12)
        assert (hit >= 0).mean() > 0.3


def test_segment_centres_and_means():
    ns = P.tiny_problem(7, n_views=2, width=23, height=17, n_seg=9, L=2, chroma_shift=1, bit_depth=10)
    pb = _pb(ns)
    for v in range(2):
        cnt, cen, mean = oracle.segment_stats(pb, v)
        bc = brute.segment_centres(ns.seg[v].tolist(), ns.S[v])
        assert [tuple(c) for c in cen] == bc
        np.testing.assert_array_equal(cnt, np.bincount(ns.seg[v].ravel(), minlength=ns.S[v]))
        ys, xs = np.mgrid[0:17, 0:23]
        Ufull = ns.U[v][ys >> 1, xs >> 1].astype(float)
        for s in range(ns.S[v]):
            sel = ns.seg[v] == s
            np.testing.assert_allclose(mean[s], [ns.Y[v][sel].mean(), Ufull[sel].mean(),
                                                 ns.V[v][ys >> 1, xs >> 1][sel].mean()], rtol=1e-12)


@pytest.mark.parametrize("lstar", [0, 21, 42])
def test_zero_cost_plane_window(lstar):
    """Rectified rig, one plane at an integer-disparity level: the window
    cost at l* is 0 wherever both windows lie inside the images."""
    rng = np.random.default_rng(300 + lstar)
    cams = synth.rectified_rig(3, 0.05, 300.0, 320, 240)
    disp = 3 + 4 * lstar // 21
    Y, U, V = P.fronto_plane_views(rng, cams, 300.0, 0.05, [-disp, 0, disp])
    seg, S = zip(*[P.random_segments(rng, 320, 240, 600) for _ in cams])
    pb = oracle.Problem(cams, Y, U, V, seg, S, 8, 0, 1.0, 5.0, 64, False)
    m, hit = oracle.window_rows(pb, *oracle.all_rows(pb), radius=1)
    ok = ~np.isnan(m[:, :, lstar])
    assert ok.mean() > 0.45
    # matched windows at l* compare identical texture columns unless a window is clamped at an edge
    vals = m[:, :, lstar][ok]
    assert (vals == 0).mean() > 0.97
    # every other level a pixel or more away costs more on random texture
    near = np.abs(np.arange(64) - lstar) <= 2
    far = m[:, :, ~near]
    assert (far[~np.isnan(far)] > 0).mean() > 0.99


def test_radius_zero_one_pixel_segments_equal_full_cost():
    """With one-pixel segments the centre is the pixel and a radius-0 window
    is that pixel: the minimum over the two neighbours of m / (3 * 255) is
    the full-segment nearest cost towards the nearest left and right views."""
    ns = P.tiny_problem(9, n_views=3, width=12, height=8, n_seg=4, L=5, rotated=True)
    ns.seg = [np.arange(96, dtype=np.int32).reshape(8, 12) for _ in range(3)]
    ns.S = [96, 96, 96]
    pb = _pb(ns, targets="nearest_lr")
    C = oracle.cost_volume(pb)
    m, hit = oracle.window_rows(pb, *oracle.all_rows(pb), radius=0)
    win = np.nanmin(np.where(np.isnan(m), np.inf, m), axis=1) / 765.0
    win = np.where(np.isinf(win), 1.0, win)
    np.testing.assert_allclose(win, C, rtol=0, atol=1e-12)
