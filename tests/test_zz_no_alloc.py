"""GPU test of ivde_cost_volume_noalloc, the plain cost volume with the
library's fixed device scratch array as workspace: through the C ABI, two
calls in a row (the second on a smaller problem, so it runs over what the
first left in the array) must each give bitwise the cost volume of
ivde_cost_volume with a caller workspace, and both must match the oracle at
the stated tolerances."""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import compare, run_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1909_02294_amd import ivde, synth  # noqa: E402


def _noalloc(dv, lr, opt, out, stream):
    return ivde.load().ivde_cost_volume_noalloc(dv.n, dv.c_cams, dv.c_images, dv.c_segs, ctypes.byref(lr),
                                                ctypes.byref(opt), ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_void_p(stream.cuda_stream))


@pytest.mark.parametrize("cost_dtype", [ivde.F32, ivde.F16])
def test_noalloc_equals_workspace_call_twice(cost_dtype):
    print(f"[case] noalloc dtype {cost_dtype}", flush=True)
    big = synth.make_rectified_320x240()
    big.bilinear = True
    small = synth.make_small_arc(seed=77, n_views=3, width=97, height=61, n_segments=60, num_labels=70)
    tdt = torch.float16 if cost_dtype == ivde.F16 else torch.float32
    stream = torch.cuda.Stream()
    results = []
    for wl in (big, small):
        dv = ivde.DeviceViews.from_workload(wl)
        lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
        opt = ivde.options(ivde.BILINEAR if wl.bilinear else ivde.NEAREST, cost_dtype)
        _, wb = ivde.sizes(dv, lr, opt)
        assert wb <= ivde.NOALLOC_SCRATCH_BYTES
        ref, _ = ivde.cost_volume(dv, lr, opt)
        torch.cuda.synchronize()
        out = torch.full((dv.rows, wl.num_labels), -3.0, dtype=tdt, device="cuda")
        torch.cuda.synchronize()
        assert _noalloc(dv, lr, opt, out, stream) == ivde.IVDE_OK
        stream.synchronize()
        assert torch.equal(out, ref), wl.name
        results.append((wl, out.double().cpu().numpy()))
    for wl, G in results:
        compare(G, run_oracle(wl), f16=cost_dtype == ivde.F16, label=wl.name)
