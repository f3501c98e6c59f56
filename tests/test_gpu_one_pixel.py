"""The parity, edge-case and behind-camera tests again with the one-pixel
sweep (pixels_per_step = 1: one pixel at 64 levels per wave step, pixel
records through the scalar unit).  The pixel-pair sweep is the default
wherever it exists, so without this module the one-pixel form would only
run with more labels per lane; both
forms compute the same quantity and are held to the same bars against the
FP64 oracle."""
import pytest

from tests import gpu_common

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from tests.test_gpu_behind import (  # noqa: E402,F401
    test_facing_rig_parity, test_hand_facing_cameras, test_rectified_bilinear_border_rows,
    test_rectified_workload_bilinear)
from tests.test_gpu_parity import (  # noqa: E402,F401
    test_depth_references, test_empty_segments_are_sentinel, test_fp16_storage, test_rectified_full_volume_nearest,
    test_repeat_is_bitwise_identical, test_small_arc_bilinear_420, test_target_sets, test_tiny_cases)


@pytest.fixture(autouse=True)
def _one_pixel_sweep(monkeypatch):
    monkeypatch.setattr(gpu_common, "SWEEP_PX", 1)
