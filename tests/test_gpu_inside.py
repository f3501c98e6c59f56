"""GPU test of the pixel-pair sweep's untested loop, with FP16 and with
16-bit code-value texels: chunks of projected records whose every sample
was shown to lie inside the validity band run without the per-sample clamp
and tests.  The measurement build
libivde_tested.so runs the tested loop on those chunks as well; both builds
must give bitwise the same cost volume, on rigs where many chunks take the
untested loop (its step count shows it) and many do not."""
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

# (generator, arguments), each run bilinear FP32, nearest FP32 and bilinear FP16
CASES = [("small_arc", dict(seed=41, n_views=4, width=160, height=96, n_segments=150, num_labels=70)),
         ("small_arc", dict(seed=42, n_views=6, width=480, height=270, n_segments=2500, num_labels=128)),
         ("small_arc", dict(seed=43, n_views=3, width=200, height=120, n_segments=9, num_labels=33)),
         ("arc_1080p", {}),
         # texels of 16-bit code values: the same loops in the kernels for that encoding
         ("small_arc", dict(seed=44, n_views=4, width=320, height=180, n_segments=600, num_labels=100,
                            bit_depth=16)),
         ("arc_1080p", dict(bit_depth=12))]
FORMS = [("bil", "F32"), ("nn", "F32"), ("bil", "F16")]

_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from tests.test_gpu_inside import CASES, FORMS, run
for i, case in enumerate(CASES):
    for j, form in enumerate(FORMS):
        C, steps = run(case, form)
        np.save(f"{sys.argv[2]}/c{i}_{j}.npy", C)
        np.save(f"{sys.argv[2]}/s{i}_{j}.npy", np.array(steps))
from paper_1909_02294_amd import ivde
print("loaded", ivde.LIB_PATH)
"""

_WL = {}


def workload(case):
    key = json.dumps(case)
    if key not in _WL:
        gen, kw = case
        _WL[key] = synth.make_small_arc(**kw) if gen == "small_arc" else synth.make_arc_1080p(**kw)
    return _WL[key]


def run(case, form):
    wl = workload(case)
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    samp = ivde.BILINEAR if form[0] == "bil" else ivde.NEAREST
    C, ws = ivde.cost_volume(dv, lr, ivde.options(samp, getattr(ivde, form[1])))
    steps = ivde.sweep_steps(ws)
    return C.cpu().numpy(), steps


@pytest.mark.skipif(not os.path.exists(build.TESTED_LIB), reason="libivde_tested.so not built")
def test_untested_loop_equals_tested_build(tmp_path):
    print(f"[case] tested build, {len(CASES)} rigs x {FORMS}", flush=True)
    env = dict(os.environ, IVDE_LIB=build.TESTED_LIB)
    r = subprocess.run([sys.executable, "-c", _CHILD, ROOT, str(tmp_path)], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert build.TESTED_LIB in r.stdout
    for i, case in enumerate(CASES):
        for j, form in enumerate(FORMS):
            got = np.load(tmp_path / f"c{i}_{j}.npy")
            t_steps = tuple(np.load(tmp_path / f"s{i}_{j}.npy"))
            want, steps = run(case, form)
            total, projected, inside = steps
            print(f"{case[0]} {case[1]} {form}: steps {steps}, inside {inside / max(total, 1):.3f}", flush=True)
            # the same work; only the tested build keeps every chunk on the tested loop
            assert t_steps[:2] == (total, projected) and t_steps[2] == 0
            assert 0 < inside < projected, "both loops must run"
            assert got.dtype == want.dtype and got.shape == want.shape
            bits = np.uint16 if got.dtype == np.float16 else np.uint32
            assert np.array_equal(got.view(bits), want.view(bits)), \
                f"{case} {form}: {int(np.sum(got != want))} entries differ"
