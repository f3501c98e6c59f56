"""GPU test of the LDS-staged sweep (libivde_stage.so, a measurement build):
when a task's target footprint fits the wave's LDS stage, the wave copies
the footprint's texels into LDS and gathers from there.  The staged build
must give bitwise the cost volume of the default build, and the test shows
from the geometry (FP64, independent of both builds) that a good share of
(task, target) footprints takes the staged path."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1909_02294_amd import build, ivde, synth  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EDGE = 1.0 / 64.0

# (seed, views, width, height, segments, levels)
CASES = [(301, 4, 160, 96, 150, 64), (302, 6, 480, 270, 2500, 128)]


def _workload(case):
    seed, n, w, h, S, L = case
    return synth.make_small_arc(seed=seed, n_views=n, width=w, height=h, n_segments=S, num_labels=L)


def _cost(wl):
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    C, _ = ivde.cost_volume(dv, lr, ivde.options(ivde.BILINEAR, ivde.F32, labels_per_lane=1, pixels_per_step=1))
    torch.cuda.synchronize()
    return C.cpu().numpy()


def _fit_fraction(wl, budget):
    """Share of (view, segment, 64-level block, target) footprints that fit
    `budget` texels: the box spanned by the segment's pixel box corners at the
    block's first and last level, projected into the target (bordered texel
    frame, clamped to the bilinear validity band), one texel of margin before
    and two after, as the staged sweep builds it."""
    cams = wl.cams
    Cr, nr = synth.rig_reference(cams)
    L = wl.num_labels
    rho = 1.0 / wl.z_far + np.arange(L) / (L - 1) * (1.0 / wl.z_near - 1.0 / wl.z_far)
    z = 1.0 / rho
    fit = total = 0
    for c, cam in enumerate(cams):
        seg = wl.seg[c]
        ys, xs = np.nonzero(np.ones_like(seg, bool))
        ids = seg.ravel()
        S = wl.S[c]
        x0 = np.full(S, np.inf); x1 = np.full(S, -np.inf); y0 = np.full(S, np.inf); y1 = np.full(S, -np.inf)
        np.minimum.at(x0, ids, xs); np.maximum.at(x1, ids, xs)
        np.minimum.at(y0, ids, ys); np.maximum.at(y1, ids, ys)
        ok = np.isfinite(x0)
        corners = np.stack([np.stack([x0, y0]), np.stack([x1, y0]), np.stack([x0, y1]), np.stack([x1, y1])], 0)
        Kinv = np.linalg.inv(cam.K)
        C = cam.center
        for b in range((L + 63) // 64):
            lo, hi = 64 * b, min(64 * b + 63, L - 1)
            pts = []
            for l in (lo, hi):
                for k in range(4):
                    px = np.stack([corners[k, 0], corners[k, 1], np.ones(S)], 0)
                    d = cam.R.T @ (Kinv @ px)
                    tau = (z[l] - nr @ (C - Cr)) / (nr @ d)
                    pts.append(C[:, None] + tau * d)
            for c2, cam2 in enumerate(cams):
                if c2 == c:
                    continue
                ix, iy = [], []
                for X in pts:
                    h = cam2.K @ (cam2.R @ X + cam2.t[:, None])
                    u = h[0] / h[2] + 1.0
                    v = h[1] / h[2] + 1.0
                    ix.append(np.floor(np.clip(u, 1 - EDGE, cam2.width + EDGE)))
                    iy.append(np.floor(np.clip(v, 1 - EDGE, cam2.height + EDGE)))
                ix, iy = np.array(ix), np.array(iy)
                X0 = np.maximum(ix.min(0) - 1, 0); X1 = np.minimum(ix.max(0) + 2, cam2.width + 1)
                Y0 = np.maximum(iy.min(0) - 1, 0); Y1 = np.minimum(iy.max(0) + 2, cam2.height + 1)
                area = (X1 - X0 + 1) * (Y1 - Y0 + 1)
                fit += int(np.sum(ok & (area <= budget)))
                total += int(np.sum(ok))
    return fit / total


_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from paper_1909_02294_amd import ivde, synth
import torch
for i, case in enumerate(json.loads(sys.argv[2])):
    seed, n, w, h, S, L = case
    wl = synth.make_small_arc(seed=seed, n_views=n, width=w, height=h, n_segments=S, num_labels=L)
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    C, _ = ivde.cost_volume(dv, lr, ivde.options(ivde.BILINEAR, ivde.F32, labels_per_lane=1, pixels_per_step=1))
    torch.cuda.synchronize()
    np.save(f"{sys.argv[3]}/staged{i}.npy", C.cpu().numpy())
print("loaded", ivde.LIB_PATH)
"""


@pytest.mark.skipif(not os.path.exists(build.STAGE_LIB), reason="libivde_stage.so not built")
def test_staged_build_equals_default_build(tmp_path):
    print(f"[case] staged build, cases {CASES}", flush=True)
    env = dict(os.environ, IVDE_LIB=build.STAGE_LIB)
    r = subprocess.run([sys.executable, "-c", _CHILD, ROOT, json.dumps(CASES), str(tmp_path)], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert build.STAGE_LIB in r.stdout
    for i, case in enumerate(CASES):
        wl = _workload(case)
        frac = _fit_fraction(wl, build.STAGE_TEXELS)
        print(f"case {case}: {100 * frac:.1f}% of footprints fit {build.STAGE_TEXELS} texels", flush=True)
        assert frac >= 0.15, "the case must exercise the staged path"
        got = np.load(tmp_path / f"staged{i}.npy")
        want = _cost(wl)
        assert got.shape == want.shape
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), \
            f"case {case}: {int(np.sum(got != want))} entries differ"
