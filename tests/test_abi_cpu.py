"""CPU checks of the C ABI: the library loads, exports every function the
header declares, its struct layouts match the Python binding, and argument
errors come back synchronously without touching a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1909_02294_amd import ivde

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ivde.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ivde_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ivde.LIB_PATH):
        from paper_1909_02294_amd import build
        build.build()
    return ivde.load()


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", ivde.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(ivde_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(ivde.SIGNATURES), set(names) ^ set(ivde.SIGNATURES)


def test_struct_layouts_match_the_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "ivde.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(ivde_camera), sizeof(ivde_image),
         sizeof(ivde_segmentation), sizeof(ivde_label_range), sizeof(ivde_options), sizeof(ivde_frame),
         sizeof(ivde_server_config), sizeof(ivde_frame_stats));
  printf("%zu %zu %zu %zu\\n", offsetof(ivde_options, target_mask), offsetof(ivde_options, sweep_events),
         offsetof(ivde_frame, labels), offsetof(ivde_frame_stats, submit_us));
  printf("%zu %zu %zu\\n", sizeof(ivde_energy), offsetof(ivde_energy, K), offsetof(ivde_energy, quantum));
  return 0;
}
""")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [ctypes.sizeof(t) for t in (ivde.Camera, ivde.Image, ivde.Segmentation, ivde.LabelRange,
                                       ivde.Options, ivde.Frame, ivde.ServerConfig, ivde.FrameStats)]
    want += [ivde.Options.target_mask.offset, ivde.Options.sweep_events.offset, ivde.Frame.labels.offset,
             ivde.FrameStats.submit_us.offset]
    want += [ctypes.sizeof(ivde.EnergyDesc), ivde.EnergyDesc.K.offset, ivde.EnergyDesc.quantum.offset]
    assert [int(x) for x in got] == want


def _segs(n, S, w, h):
    arr = (ivde.Segmentation * n)()
    for i in range(n):
        arr[i].seg_map = 0x1000     # sizes only: the pointer is never dereferenced
        arr[i].pitch = w
        arr[i].num_segments = S
    return arr


def _cams(n, w, h):
    from paper_1909_02294_amd import synth
    return ivde.make_cameras(synth.arc_rig(n, 3.0, 30.0, 100.0, w, h))


def test_size_query(lib):
    n, w, h, S, L = 3, 40, 30, 17, 100
    cb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    lr = ivde.label_range(1.0, 5.0, L)
    st = lib.ivde_cost_volume_size(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr),
                                   ctypes.byref(ivde.options(ivde.BILINEAR, ivde.F32)), 10, ctypes.byref(cb),
                                   ctypes.byref(wb))
    assert st == ivde.IVDE_OK
    assert cb.value == n * S * L * 4
    assert wb.value > (w + 1) * (h + 1) * 8 * n
    lib.ivde_cost_volume_size(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr),
                              ctypes.byref(ivde.options(ivde.BILINEAR, ivde.F16)), 10, ctypes.byref(cb), None)
    assert cb.value == n * S * L * 2
    # texels are 8 bytes at every bit depth (FP16 channels up to 11 bits, 16-bit code values above)
    for bits in (8, 11, 12, 16):
        wb2 = ctypes.c_size_t()
        assert lib.ivde_cost_volume_size(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr),
                                         ctypes.byref(ivde.options(ivde.BILINEAR, ivde.F32)), bits, None,
                                         ctypes.byref(wb2)) == ivde.IVDE_OK
        assert wb2.value == wb.value, bits


def test_sweep_steps_needs_a_workspace(lib):
    a = ctypes.c_int64(-1)
    assert lib.ivde_workspace_sweep_steps(None, None, ctypes.byref(a), None, None) == ivde.IVDE_EINVAL
    assert a.value == -1


def test_sweep_shape_query(lib):
    """The launch shape the plain call takes: the pixel-pair sweep by default
    (one label per lane, at any bit depth: FP16 texel channels up to 11 bits,
    16-bit code values above), the one-pixel sweep where asked for or with
    more labels per lane."""
    n, w, h, S = 3, 40, 30, 17
    lr = ivde.label_range(1.0, 5.0, 256)

    def shape(opt, bits=10):
        j, wpg, px = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        st = lib.ivde_sweep_shape(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr), ctypes.byref(opt), bits,
                                  ctypes.byref(j), ctypes.byref(wpg), ctypes.byref(px))
        assert st == ivde.IVDE_OK, st
        return j.value, wpg.value, px.value

    assert shape(ivde.options(ivde.BILINEAR, ivde.F32)) == (1, 4, 2)
    assert shape(ivde.options(ivde.NEAREST, ivde.F16)) == (1, 4, 2)
    assert shape(ivde.options(ivde.BILINEAR, ivde.F32), bits=8) == (1, 4, 2)
    assert shape(ivde.options(ivde.BILINEAR, ivde.F32), bits=12) == (1, 4, 2)
    assert shape(ivde.options(ivde.NEAREST, ivde.F32), bits=16) == (1, 4, 2)
    assert shape(ivde.options(pixels_per_step=1)) == (1, 4, 1)
    assert shape(ivde.options(pixels_per_step=4)) == (1, 4, 4)
    assert shape(ivde.options(labels_per_lane=2, waves_per_group=2)) == (2, 2, 1)
    assert shape(ivde.options(labels_per_lane=2, pixels_per_step=2)) == (2, 4, 1)
    assert shape(ivde.options(pixels_per_step=4), bits=12) == (1, 4, 4)
    assert shape(ivde.options(pixels_per_step=1), bits=16) == (1, 4, 1)
    # few levels over the same depth range land far apart: four pixels per step
    lr_far = ivde.label_range(1.0, 5.0, 16)
    j, wpg, px = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.ivde_sweep_shape(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr_far),
                                ctypes.byref(ivde.options()), 10, ctypes.byref(j), ctypes.byref(wpg),
                                ctypes.byref(px)) == ivde.IVDE_OK
    assert px.value == 4

    # over level counts, four pixels where levels land far apart and two where close; nearest
    # sampling (one texel per sample) needs twice the spacing (6 px against 3 px)
    def px_for(L, samp):
        lr_l = ivde.label_range(1.0, 5.0, L)
        p = ctypes.c_int32()
        assert lib.ivde_sweep_shape(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr_l),
                                    ctypes.byref(ivde.options(samp, ivde.F32)), 10, None, None,
                                    ctypes.byref(p)) == ivde.IVDE_OK
        return p.value

    Ls = [2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 128, 256]
    bil = [px_for(L, ivde.BILINEAR) for L in Ls]
    nn = [px_for(L, ivde.NEAREST) for L in Ls]
    for seq in (bil, nn):
        assert seq[0] == 4 and seq[-1] == 2 and seq == sorted(seq, reverse=True), seq
    assert all(b >= a for a, b in zip(nn, bil)) and nn != bil, (bil, nn)
    # outputs may be NULL; argument errors as for the size query
    assert lib.ivde_sweep_shape(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr),
                                ctypes.byref(ivde.options()), 10, None, None, None) == ivde.IVDE_OK
    assert lib.ivde_sweep_shape(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr),
                                ctypes.byref(ivde.options()), 7, None, None, None) == ivde.IVDE_EINVAL
    assert lib.ivde_sweep_shape(n, _cams(n, w, h), _segs(n, S, w, h), ctypes.byref(lr),
                                ctypes.byref(ivde.options(pixels_per_step=3)), 10, None, None, None) == ivde.IVDE_EINVAL


@pytest.mark.parametrize("field,value", [
    ("n_views", 0), ("n_views", 33), ("z_near", -1.0), ("z_far", float("nan")), ("num_labels", 0),
    ("depth_ref", 7), ("sampling", 5), ("cost_dtype", 9), ("labels_per_lane", 3), ("waves_per_group", 8),
    ("pixels_per_step", 3), ("pixels_per_step", 5), ("pixels_per_step", -1),
    ("bit_depth", 7), ("bit_depth", 17), ("width", 0), ("segments", 0),
])
def test_invalid_arguments_are_rejected(lib, field, value):
    n, w, h, S, L = 3, 40, 30, 17, 64
    cams, segs = _cams(n, w, h), _segs(n, S, w, h)
    lr = ivde.label_range(1.0, 5.0, L)
    opt = ivde.options(ivde.BILINEAR, ivde.F32)
    bd = 10
    if field == "n_views":
        n = value
    elif field in ("z_near", "z_far", "num_labels", "depth_ref"):
        setattr(lr, field, value)
    elif field in ("sampling", "cost_dtype", "labels_per_lane", "waves_per_group", "pixels_per_step"):
        setattr(opt, field, value)
    elif field == "bit_depth":
        bd = value
    elif field == "width":
        cams[1].width = value
    elif field == "segments":
        segs[2].num_segments = value
    cb = ctypes.c_size_t()
    st = lib.ivde_cost_volume_size(n, cams, segs, ctypes.byref(lr), ctypes.byref(opt), bd, ctypes.byref(cb), None)
    assert st == ivde.IVDE_EINVAL
    assert lib.ivde_last_error().decode()


def test_singular_or_projective_k_rejected(lib):
    cams = _cams(2, 20, 10)
    cams[0].K[6] = 0.1
    cb = ctypes.c_size_t()
    lr = ivde.label_range(1.0, 5.0, 8)
    assert lib.ivde_cost_volume_size(2, cams, _segs(2, 4, 20, 10), ctypes.byref(lr),
                                     ctypes.byref(ivde.options()), 8, ctypes.byref(cb), None) == ivde.IVDE_EINVAL
    cams = _cams(2, 20, 10)
    cams[1].K[0] = 0.0
    cams[1].K[1] = 0.0
    assert lib.ivde_cost_volume_size(2, cams, _segs(2, 4, 20, 10), ctypes.byref(lr),
                                     ctypes.byref(ivde.options()), 8, ctypes.byref(cb), None) == ivde.IVDE_EINVAL


def test_argmin_argument_checks(lib):
    assert lib.ivde_argmin(-1, 4, ivde.F32, None, None, None) == ivde.IVDE_EINVAL
    assert lib.ivde_argmin(5, 0, ivde.F32, None, None, None) == ivde.IVDE_EINVAL
    assert lib.ivde_argmin(5, 4, 7, None, None, None) == ivde.IVDE_EINVAL
    assert lib.ivde_argmin(5, 4, ivde.F32, None, None, None) == ivde.IVDE_EINVAL
    assert lib.ivde_argmin(0, 4, ivde.F32, None, None, None) == ivde.IVDE_OK   # nothing to do


def test_cost_volume_rejects_bad_workspace(lib):
    n, w, h, S, L = 2, 16, 8, 3, 8
    cams, segs = _cams(n, w, h), _segs(n, S, w, h)
    imgs = (ivde.Image * n)()
    for i in range(n):
        for p in range(3):
            imgs[i].plane[p] = 0x2000
            imgs[i].pitch[p] = w
        imgs[i].bit_depth, imgs[i].chroma_shift = 8, 0
    lr = ivde.label_range(1.0, 5.0, L)
    opt = ivde.options(ivde.NEAREST)
    # null workspace, misaligned workspace, too small: all before any device work
    assert lib.ivde_cost_volume(n, cams, imgs, segs, ctypes.byref(lr), ctypes.byref(opt), None, 0,
                                ctypes.c_void_p(0x4000), None) == ivde.IVDE_EINVAL
    assert lib.ivde_cost_volume(n, cams, imgs, segs, ctypes.byref(lr), ctypes.byref(opt), ctypes.c_void_p(0x1010),
                                1 << 30, ctypes.c_void_p(0x4000), None) == ivde.IVDE_EINVAL
    assert lib.ivde_cost_volume(n, cams, imgs, segs, ctypes.byref(lr), ctypes.byref(opt), ctypes.c_void_p(0x10000),
                                16, ctypes.c_void_p(0x4000), None) == ivde.IVDE_ENOMEM
    # mixed bit depths
    imgs[1].bit_depth = 10
    assert lib.ivde_cost_volume(n, cams, imgs, segs, ctypes.byref(lr), ctypes.byref(opt), ctypes.c_void_p(0x10000),
                                1 << 30, ctypes.c_void_p(0x4000), None) == ivde.IVDE_EINVAL


def test_batch_and_server_argument_checks(lib):
    wb = ctypes.c_size_t()
    assert lib.ivde_batch_size(0, None, ctypes.byref(ivde.options()), ctypes.byref(wb)) == ivde.IVDE_EINVAL
    frames = (ivde.Frame * 1)()
    opt = ivde.options(targets=ivde.TARGETS_EXPLICIT, target_mask=np.zeros((2, 2), np.uint8))
    assert lib.ivde_batch_size(1, frames, ctypes.byref(opt), ctypes.byref(wb)) == ivde.IVDE_EINVAL
    h = ctypes.c_void_p()
    cfg = ivde.ServerConfig(None, 0, 4)
    assert lib.ivde_server_create(ctypes.byref(cfg), ctypes.byref(h)) == ivde.IVDE_EINVAL
    cfg = ivde.ServerConfig(0x10000, 1 << 20, 99)
    assert lib.ivde_server_create(ctypes.byref(cfg), ctypes.byref(h)) == ivde.IVDE_EINVAL
    cfg = ivde.ServerConfig(0x10000, 1 << 20, 2, 1, 0)     # reserved must be 0
    assert lib.ivde_server_create(ctypes.byref(cfg), ctypes.byref(h)) == ivde.IVDE_EINVAL
    st = ivde.FrameStats()
    assert lib.ivde_stream_poll(None, 1, ctypes.byref(st)) == ivde.IVDE_EINVAL
    t = ctypes.c_uint64()
    imgs = _imgs(2, 16)
    for mode in (ivde.SUBMIT_MASK, ivde.SUBMIT_RULE, ivde.SUBMIT_RULE_IFRAME):
        assert lib.ivde_stream_submit_host(None, 0, imgs, mode, None, None, None, ctypes.byref(t)) == ivde.IVDE_EINVAL
    # unknown mode, and a mask with a rule mode, are refused before the server is looked at
    assert lib.ivde_stream_submit_host(None, 0, imgs, 7, None, None, None, ctypes.byref(t)) == ivde.IVDE_EINVAL
    mask = (ctypes.c_uint8 * 8)()
    assert lib.ivde_stream_submit_host(None, 0, imgs, ivde.SUBMIT_RULE, mask, None, None,
                                       ctypes.byref(t)) == ivde.IVDE_EINVAL
    assert b"mask" in lib.ivde_last_error()
    assert lib.ivde_batch_run(None, None, 0) == ivde.IVDE_EINVAL


def test_status_strings(lib):
    for s in range(-6, 1):
        assert lib.ivde_status_string(s)
    assert b"gfx950" in lib.ivde_version()


def _imgs(n, w, bits=8):
    imgs = (ivde.Image * n)()
    for i in range(n):
        for p in range(3):
            imgs[i].plane[p] = 0x2000
            imgs[i].pitch[p] = w
        imgs[i].bit_depth, imgs[i].chroma_shift = bits, 0
    return imgs


def test_term_entry_points_reject_bad_arguments(lib):
    """Window, statistics, rule, adjacency and intra-cost calls refuse bad
    arguments before any device work."""
    n, w, h, S, L = 2, 16, 8, 3, 8
    cams, segs, imgs = _cams(n, w, h), _segs(n, S, w, h), _imgs(n, w)
    lr = ivde.label_range(1.0, 5.0, L)
    ob, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.ivde_window_cost_size(n, cams, segs, ctypes.byref(lr), 8, ctypes.byref(ob), ctypes.byref(wb)) == 0
    assert ob.value == n * S * 2 * L * 4
    big = ctypes.c_void_p(0x100000)
    # radius out of range, missing outputs
    assert lib.ivde_window_cost(n, cams, imgs, segs, ctypes.byref(lr), 9, big, 1 << 30, big, big, None) == \
        ivde.IVDE_EINVAL
    assert lib.ivde_window_cost(n, cams, imgs, segs, ctypes.byref(lr), 1, big, 1 << 30, None, big, None) == \
        ivde.IVDE_EINVAL
    assert lib.ivde_window_energy(-1, L, None, None, None, ctypes.c_float(30.0), None, None) == ivde.IVDE_EINVAL
    assert lib.ivde_segment_stats_size(n, cams, segs, 20, ctypes.byref(wb)) == ivde.IVDE_EINVAL
    assert lib.ivde_temporal_rule(4, None, None, None, ctypes.c_float(3.0), ctypes.c_float(1.0), 10, None,
                                  None) == ivde.IVDE_EINVAL
    assert lib.ivde_temporal_rule(0, None, None, None, ctypes.c_float(3.0), ctypes.c_float(1.0), 10, None,
                                  None) == ivde.IVDE_OK
    # adjacency: offsets required; index/beta required with a capacity; beta0 and eps positive
    assert lib.ivde_adjacency_size(n, cams, segs, 8, ctypes.byref(wb)) == ivde.IVDE_OK
    f = ctypes.c_float
    assert lib.ivde_adjacency(n, cams, imgs, segs, f(1.0), f(1.0), big, 1 << 30, None, None, None, 0, None) == \
        ivde.IVDE_EINVAL
    assert lib.ivde_adjacency(n, cams, imgs, segs, f(1.0), f(1.0), big, 1 << 30, big, None, None, 5, None) == \
        ivde.IVDE_EINVAL
    assert lib.ivde_adjacency(n, cams, imgs, segs, f(1.0), f(0.0), big, 1 << 30, big, None, None, 0, None) == \
        ivde.IVDE_EINVAL
    assert lib.ivde_adjacency(n, cams, imgs, segs, f(float("nan")), f(1.0), big, 1 << 30, big, None, None, 0,
                              None) == ivde.IVDE_EINVAL
    assert lib.ivde_adjacency(n, cams, imgs, segs, f(1.0), f(1.0), None, 0, big, None, None, 0, None) == \
        ivde.IVDE_EINVAL
    assert lib.ivde_intra_cost(3, 0, None, None, None, None, None, None, None) == ivde.IVDE_EINVAL
    assert lib.ivde_intra_cost(3, 4, None, big, big, big, None, big, None) == ivde.IVDE_EINVAL
    assert lib.ivde_intra_cost(0, 4, None, None, None, None, None, None, None) == ivde.IVDE_OK


def test_depth_map_and_footprint_argument_checks(lib):
    n, w, h, S, L = 2, 16, 8, 3, 8
    cams, segs = _cams(n, w, h), _segs(n, S, w, h)
    big = ctypes.c_void_p(0x100000)
    bad = ivde.label_range(2.0, 2.0, L)
    assert lib.ivde_depth_map(n, cams, segs, ctypes.byref(bad), big, big, 4 * L, big, None) == ivde.IVDE_EINVAL
    lr = ivde.label_range(1.0, 5.0, L)
    assert lib.ivde_depth_map(n, cams, segs, ctypes.byref(lr), None, big, 4 * L, big, None) == ivde.IVDE_EINVAL
    assert lib.ivde_depth_map(0, cams, segs, ctypes.byref(lr), big, big, 4 * L, big, None) == ivde.IVDE_EINVAL
    # the level-depth table needs 4 L bytes of 4-byte aligned workspace
    assert lib.ivde_depth_map(n, cams, segs, ctypes.byref(lr), big, None, 4 * L, big, None) == ivde.IVDE_EINVAL
    assert lib.ivde_depth_map(n, cams, segs, ctypes.byref(lr), big, ctypes.c_void_p(0x100002), 4 * L, big,
                              None) == ivde.IVDE_EINVAL
    assert lib.ivde_depth_map(n, cams, segs, ctypes.byref(lr), big, big, 4 * L - 4, big, None) == ivde.IVDE_ENOMEM
    r, q, qh = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    opt = ivde.options(ivde.BILINEAR, ivde.F16)
    assert lib.ivde_server_footprint(n, cams, segs, ctypes.byref(lr), ctypes.byref(opt), 10, 1, ctypes.byref(r),
                                     ctypes.byref(q), ctypes.byref(qh)) == ivde.IVDE_OK
    # resident holds two FP16 volumes, the maps and a workspace; a frame holds at least its counters
    assert r.value > 2 * n * S * L * 2 + n * w * h * 4 and q.value >= 256
    # a host frame also holds its staged planes (2-byte Y and two 4:2:0 chroma planes per view) and mask
    assert qh.value >= q.value + n * (w * h * 2 + 2 * (w // 2) * (h // 2) * 2) + n * S
    assert lib.ivde_server_footprint(n, cams, segs, ctypes.byref(lr), ctypes.byref(opt), 10, 0, None, None,
                                     None) == ivde.IVDE_OK
    assert lib.ivde_server_footprint(n, cams, segs, ctypes.byref(lr), ctypes.byref(opt), 20, 1, ctypes.byref(r),
                                     ctypes.byref(q), None) == ivde.IVDE_EINVAL
    assert lib.ivde_server_footprint(n, cams, segs, ctypes.byref(lr), ctypes.byref(opt), 10, 2, ctypes.byref(r),
                                     ctypes.byref(q), None) == ivde.IVDE_EINVAL


def test_binding_rejects_tensors_the_library_would_misread():
    """The Python binding passes raw pointers, so it checks dtype,
    contiguity and shape first (checked here on CPU tensors)."""
    torch = pytest.importorskip("torch")
    ok = torch.zeros((5, 8), dtype=torch.float32)
    assert ivde._check(ok, "cost", (torch.float32, torch.float16), (None, 8), cuda=False) is ok
    with pytest.raises(ValueError, match="dtype"):
        ivde._check(ok.to(torch.float64), "cost", (torch.float32, torch.float16), cuda=False)
    with pytest.raises(ValueError, match="contiguous"):
        ivde._check(ok.t(), "cost", torch.float32, cuda=False)
    with pytest.raises(ValueError, match="shape"):
        ivde._check(ok, "cost", torch.float32, (5, 9), cuda=False)
    with pytest.raises(ValueError, match="shape"):
        ivde._check(ok, "cost", torch.float32, (5,), cuda=False)
    with pytest.raises(ValueError, match="GPU"):
        ivde._check(ok, "cost", torch.float32)


def test_noalloc_refuses_problems_beyond_its_scratch_array(lib):
    """ivde_cost_volume_noalloc checks the workspace a problem needs against
    its fixed scratch array before touching any device memory."""
    n, w, h, S, L = 8, 1920, 1080, 100, 64
    cams, segs = _cams(n, w, h), _segs(n, S, w, h)
    imgs = (ivde.Image * n)()
    for i in range(n):
        for p in range(3):
            imgs[i].plane[p] = 0x2000          # never dereferenced: the call is refused first
            imgs[i].pitch[p] = w
        imgs[i].bit_depth, imgs[i].chroma_shift = 10, 1
    lr = ivde.label_range(1.5, 10.0, L)
    opt = ivde.options(ivde.BILINEAR, ivde.F32)
    wb = ctypes.c_size_t()
    assert lib.ivde_cost_volume_size(n, cams, segs, ctypes.byref(lr), ctypes.byref(opt), 10, None,
                                     ctypes.byref(wb)) == ivde.IVDE_OK
    assert wb.value > ivde.NOALLOC_SCRATCH_BYTES
    m = re.search(r"#define IVDE_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == ivde.NOALLOC_SCRATCH_BYTES
    st = lib.ivde_cost_volume_noalloc(n, cams, imgs, segs, ctypes.byref(lr), ctypes.byref(opt),
                                      ctypes.c_void_p(0x3000), None)
    assert st == ivde.IVDE_ENOMEM
    assert b"scratch" in lib.ivde_last_error()
    # a null output is an argument error, found first
    assert lib.ivde_cost_volume_noalloc(n, cams, imgs, segs, ctypes.byref(lr), ctypes.byref(opt), None,
                                        None) == ivde.IVDE_EINVAL
