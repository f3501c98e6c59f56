"""The launch-shape cache per shape class (host logic, no GPU): the class key
follows the quantities the sweep's speed depends on, a cached class is
answered without timing anything, and a new class is tuned once and
stored."""
import json
from types import SimpleNamespace

import pytest

from paper_1909_02294_amd import ivde


def _dv(n=8, w=1920, h=1080, S=20000, bits=10):
    cams = [SimpleNamespace(width=w, height=h) for _ in range(n)]
    return SimpleNamespace(cams=cams, S=[S] * n, n=n, bit_depth=bits)


def test_shape_class_keys():
    lr = ivde.label_range(1.5, 10.0, 256)
    o = ivde.options(ivde.BILINEAR, ivde.F32)
    # 103.7 pixels per segment rounds to 128; 7 targets per view
    assert ivde.shape_class(_dv(), lr, o) == "bil-f32-texf16-L256-px128-t7"
    # 40000 segments: 51.8 pixels -> 64; 5000: 414.7 -> 512
    assert ivde.shape_class(_dv(S=40000), lr, o).endswith("-px64-t7")
    assert ivde.shape_class(_dv(S=5000), lr, o).endswith("-px512-t7")
    # levels round up to 64-level blocks; 250 and 256 share a class, 130 does not
    assert ivde.shape_class(_dv(), ivde.label_range(1.5, 10.0, 250), o) == ivde.shape_class(_dv(), lr, o)
    assert "-L192-" in ivde.shape_class(_dv(), ivde.label_range(1.5, 10.0, 130), o)
    # texel encoding (FP16 channels up to 11 bits, 16-bit code values above), storage, sampling and
    # targets split classes
    assert "-texu16-" in ivde.shape_class(_dv(bits=12), lr, o)
    assert "-texf16-" in ivde.shape_class(_dv(bits=11), lr, o)
    assert ivde.shape_class(_dv(), lr, ivde.options(ivde.NEAREST, ivde.F16)).startswith("nn-f16-")
    assert ivde.shape_class(_dv(), lr, ivde.options(targets=ivde.TARGETS_NEAREST_LR)).endswith("-t2")


def test_cached_class_is_not_timed_again(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    lr = ivde.label_range(1.5, 10.0, 256)
    o = ivde.options(ivde.BILINEAR, ivde.F32)
    calls = []

    def fake_autotune(dv, lr_, opt, reps=2, stream=None):
        calls.append(ivde.shape_class(dv, lr_, opt))
        best = ivde.options(opt.sampling, opt.cost_dtype, labels_per_lane=2, waves_per_group=4, pixels_per_step=1)
        return best, {s: 100.0 + i for i, s in enumerate(ivde.AUTOTUNE_SHAPES)}

    monkeypatch.setattr(ivde, "autotune", fake_autotune)
    best, table = ivde.autotune_cached(_dv(), lr, o, str(path))
    assert (best.labels_per_lane, best.waves_per_group) == (2, 4) and table is not None
    stored = json.loads(path.read_text())
    assert stored["bil-f32-texf16-L256-px128-t7"]["labels_per_lane"] == 2
    assert stored["bil-f32-texf16-L256-px128-t7"]["pixels_per_step"] == 1
    assert "1x4x2" in stored["bil-f32-texf16-L256-px128-t7"]["us"]
    # same class (another segment count that rounds alike, 250 levels): from the file
    best2, table2 = ivde.autotune_cached(_dv(S=21000), ivde.label_range(1.5, 10.0, 250), o, str(path))
    assert table2 is None and (best2.labels_per_lane, best2.waves_per_group) == (2, 4)
    assert len(calls) == 1
    # another class is tuned and added beside the first
    ivde.autotune_cached(_dv(S=5000), lr, o, str(path))
    assert len(calls) == 2 and len(json.loads(path.read_text())) == 2


def test_memory_cache_without_a_file(monkeypatch):
    monkeypatch.setattr(ivde, "_TUNE_MEMO", {})
    n = []

    def fake_autotune(dv, lr_, opt, reps=2, stream=None):
        n.append(1)
        return ivde.options(labels_per_lane=1, waves_per_group=4), {}

    monkeypatch.setattr(ivde, "autotune", fake_autotune)
    lr = ivde.label_range(1.5, 10.0, 64)
    for _ in range(3):
        best, _ = ivde.autotune_cached(_dv(n=3, w=320, h=240, S=1200), lr, ivde.options(ivde.NEAREST))
        assert best.waves_per_group == 4
    assert len(n) == 1


if __name__ == "__main__":
    pytest.main([__file__, "-q"])
