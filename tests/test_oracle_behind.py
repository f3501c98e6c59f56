"""Pins of the oracle where 3-D points fall behind a camera.

The paper's cameras are arbitrarily positioned (Sec. III-A), so a level
point can lie behind the source camera (tau <= 0: the level plane is on the
far side of the camera along the pixel's ray) or behind a target camera
(camera-frame z <= 0).  Both leave the sample invalid.  Pinned here by

* a hand-derived case of two cameras facing each other
  (tests/golden/hand_behind.json), where each branch decides a row and a
  dropped or sign-flipped test would land on a pixel and change the cost;
* the pure-Python brute force on a four-view rig with a camera looking back
  at the others and one standing among the level planes, for three depth
  references, both samplings and both chroma formats, with the share of
  samples that reach each branch computed from FP64 geometry in the test.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from tests import _problems as P


def hand_behind_problem(sampling):
    with open(os.path.join(P.GOLDEN, "hand_behind.json")) as fh:
        g = json.load(fh)
    w, h = g["width"], g["height"]
    cams = [P.cam(g["K"], R, t, w, h) for R, t in zip(g["R"], g["t"])]
    Y = [np.array([v["Y"]], np.uint8) for v in g["views"]]
    U = [np.array([v["U"]], np.uint8) for v in g["views"]]
    V = [np.array([v["V"]], np.uint8) for v in g["views"]]
    seg = [np.arange(w, dtype=np.int32)[None, :] for _ in cams]
    from types import SimpleNamespace
    ns = SimpleNamespace(cams=cams, Y=Y, U=U, V=V, seg=seg, S=[w, w], bit_depth=g["bit_depth"], chroma_shift=0,
                         z_near=g["z_near"], z_far=g["z_far"], num_labels=g["num_labels"],
                         bilinear=sampling == "bilinear")
    return ns, g["depth_ref"], np.array(g["expected"][sampling])


@pytest.mark.parametrize("sampling", ["nearest", "bilinear"])
def test_hand_derived_facing_cameras(sampling):
    ns, ref, expected = hand_behind_problem(sampling)
    # the geometry of the derivation: view 1's far level lies behind view 1
    # (tau < 0) and view 0's far level lies behind view 1 as a target
    geo = P.behind_geometry(ns, ref)
    assert geo["tau_nonpos"][1] > 0 and geo["behind_flip_inside"] > 0
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, 0, ns.z_near, ns.z_far,
                        ns.num_labels, ns.bilinear, depth_ref=ref)
    C = oracle.cost_volume(pb)
    np.testing.assert_allclose(C, expected, rtol=0, atol=1e-14)
    B = np.array(brute.cost_volume(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, 0, ns.z_near, ns.z_far,
                                   ns.num_labels, ns.bilinear, oracle.target_matrix(2), depth_ref=ref))
    np.testing.assert_allclose(B, expected, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("bilinear", [False, True])
@pytest.mark.parametrize("chroma_shift", [0, 1])
def test_oracle_matches_brute_force_behind_cameras(seed, bilinear, chroma_shift):
    ns = P.facing_problem(40 + seed, bilinear=bilinear, chroma_shift=chroma_shift, bit_depth=8 if seed < 2 else 10)
    for ref, bref in ((oracle.REF_RIG_CENTER, "rig"), (oracle.REF_OWN, "own"), (0, 0)):
        geo = P.behind_geometry(ns, bref)
        # every reference puts samples behind a target, and some of them
        # would land inside it if the sign of their depth were ignored
        assert geo["behind_share"] > 0.1 and geo["behind_flip_inside"] > 0
        if bref != "own":
            # the rig-centre and camera-0 planes lie partly behind views 2, 3
            assert max(geo["tau_nonpos"]) > 0.1
        pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift, ns.z_near,
                            ns.z_far, ns.num_labels, ns.bilinear, depth_ref=ref)
        C = oracle.cost_volume(pb)
        B = np.array(brute.cost_volume(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift,
                                       ns.z_near, ns.z_far, ns.num_labels, ns.bilinear, pb.T, depth_ref=bref))
        np.testing.assert_allclose(C, B, rtol=0, atol=1e-12)
        # real matches as well as sentinels
        assert 0.2 < (C < 1.0).mean() < 1.0


def test_behind_samples_never_count():
    """Per-target valid counts of the oracle never exceed the samples that
    the FP64 geometry finds in front of both cameras, and the levels that
    lie behind view 2 along all of its rays give it only sentinels."""
    ns = P.facing_problem(47, width=16, height=10, n_seg=5, L=6)
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, 0, ns.z_near, ns.z_far,
                        ns.num_labels, False, depth_ref=oracle.REF_RIG_CENTER)
    C, m, nv = oracle.cost_volume(pb, with_terms=True)
    centres = np.array([c.center for c in ns.cams])
    a = np.array([c.axis for c in ns.cams]).mean(0)
    nr, Cr = a / np.linalg.norm(a), centres.mean(0)
    rho = 1 / ns.z_far + np.arange(ns.num_labels) / (ns.num_labels - 1) * (1 / ns.z_near - 1 / ns.z_far)
    off = pb.row_offsets()
    for c in range(4):
        cam = ns.cams[c]
        ys, xs = np.mgrid[0:cam.height, 0:cam.width].astype(float)
        p = np.stack([xs.ravel(), ys.ravel(), np.ones(xs.size)])
        d = (cam.R.T @ np.linalg.inv(cam.K) @ p).T
        tau = (1 / rho[None, :] - (centres[c] - Cr) @ nr) / (d @ nr)[:, None]
        segs = ns.seg[c].ravel()
        for c2 in range(4):
            if c2 == c:
                continue
            X = centres[c] + tau[..., None] * d[:, None, :]
            zc = (X @ ns.cams[c2].R.T + ns.cams[c2].t)[..., 2]
            ok = (tau > 0) & (zc > 0)
            for s in range(ns.S[c]):
                bound = ok[segs == s].sum(0)
                assert np.all(nv[off[c] + s, c2] <= bound)
    # view 2 looks back at the rig from beyond the reference plane: its
    # levels deeper than its own offset (z = 4.5, 2.65, 1.875 here) lie
    # behind it along every ray (tau <= 0), so those columns are sentinels
    far = 1 / rho > (centres[2] - Cr) @ nr
    assert far.sum() == 3
    assert np.all(C[off[2]:off[3]][:, far] == 1.0)
    assert np.all(C[off[2]:off[3]][:, ~far] < 1.0)
