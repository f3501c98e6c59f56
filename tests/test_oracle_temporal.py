"""Pins of the oracle's temporal rule (Sec. III-E): thresholds T_P = 3 and
T_I = 1 in 8-bit code values on every mean-colour component, strict
inequality, the I-frame test first, scaling with bit depth, and the
temporally updated frame."""
import numpy as np

import oracle
from tests import _problems as P


def _m(*rows):
    return np.array([list(r) + [0.0] for r in rows], np.float64)


def test_rule_hand_cases():
    prev = _m((100, 128, 128), (100, 128, 128), (100, 128, 128), (100, 128, 128), (50, 50, 50), (10, 10, 10))
    cur = _m((102.9, 126, 130), (103, 128, 128), (100, 131, 128), (100, 128, 125.5), (50.5, 50, 50), (30, 10, 10))
    ifr = _m((90, 128, 128), (90, 128, 128), (90, 128, 128), (100, 128, 126), (50, 50, 50.99), (29.5, 10, 10))
    got = oracle.temporal_rule(cur, prev, ifr, 3.0, 1.0, 8)
    # row 0: all |d| < 3 against prev, far from the I frame -> 1
    # row 1: |dY| = 3 is not < 3 -> recompute
    # row 2: |dCb| = 3 -> recompute
    # row 3: |dCr| = 2.5 < 3 against prev, but 0.5 < 1 against the I frame -> 2
    # row 4: every |d| < 1 against the I frame -> 2
    # row 5: 20 against prev, 0.5 against the I frame -> 2
    np.testing.assert_array_equal(got, [1, 0, 0, 2, 2, 2])
    np.testing.assert_array_equal(oracle.temporal_rule(cur, prev, None, 3.0, 1.0, 8), [1, 0, 0, 1, 1, 0])


def test_rule_scales_with_bit_depth():
    prev = _m((400, 512, 512))
    cur = _m((411, 512, 512))
    assert oracle.temporal_rule(cur, prev, None, 3.0, 1.0, 10)[0] == 1     # 11 < 12
    cur = _m((412, 512, 512))
    assert oracle.temporal_rule(cur, prev, None, 3.0, 1.0, 10)[0] == 0     # 12 is not < 12


def test_unchanged_frame_keeps_every_row():
    ns = P.tiny_problem(31, n_views=3, width=24, height=16, n_seg=10, L=4, chroma_shift=1, bit_depth=10)
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, 10, 1, ns.z_near, ns.z_far, 4, True)
    _, _, mean = oracle.all_segment_stats(pb)
    src = oracle.temporal_rule(mean, mean, mean, 3.0, 1.0, 10)
    assert np.all(src == 2)
    C = oracle.cost_volume(pb)
    np.testing.assert_array_equal(oracle.served_rule(C * 0 + 7, C, pb, src), C)


def test_served_rule_recomputes_only_source_zero():
    ns = P.tiny_problem(32, n_views=3, width=24, height=16, n_seg=10, L=4, bilinear=True, rotated=True)
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, 8, 0, ns.z_near, ns.z_far, 4, True)
    C = oracle.cost_volume(pb)
    rows = C.shape[0]
    src = np.arange(rows) % 3
    prev = np.full_like(C, 0.25)
    ifr = np.full_like(C, 0.75)
    out = oracle.served_rule(prev, ifr, pb, src)
    np.testing.assert_array_equal(out[src == 1], prev[src == 1])
    np.testing.assert_array_equal(out[src == 2], ifr[src == 2])
    np.testing.assert_array_equal(out[src == 0], C[src == 0])
