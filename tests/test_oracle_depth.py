"""Pins of the oracle's depth painting (Sec. III-B; levels uniform in
inverse depth between the depth range's ends)."""
import numpy as np

import oracle
from tests import _problems as P


def test_level_depths_closed_form():
    z = oracle.level_depths(1.5, 10.0, 5)
    assert z[0] == 10.0 and z[-1] == 1.5
    # inverse depths are equally spaced
    inv = 1.0 / z
    np.testing.assert_allclose(np.diff(inv), (1 / 1.5 - 1 / 10.0) / 4, rtol=1e-14)
    assert oracle.level_depths(2.0, 7.0, 1)[0] == 7.0


def test_depth_map_paints_segments():
    ns = P.tiny_problem(3, n_views=2, width=9, height=5, n_seg=4, L=6)
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, 8, 0, ns.z_near, ns.z_far, 6, False)
    rows = sum(ns.S)
    lab = np.arange(rows) % 6
    D = oracle.depth_map(pb, lab)
    z = oracle.level_depths(ns.z_near, ns.z_far, 6)
    assert D.shape == (2 * 9 * 5,)
    v1 = D[45:].reshape(5, 9)
    for y in range(5):
        for x in range(9):
            assert v1[y, x] == z[(ns.S[0] + ns.seg[1][y, x]) % 6]
    # a labelling with every segment at the last level paints z_near everywhere
    assert np.all(oracle.depth_map(pb, np.full(rows, 5)) == ns.z_near)
