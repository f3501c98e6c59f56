"""GPU parity of the segment statistics, the temporal rule (Sec. III-E) and
the server's rule-driven frames."""
import numpy as np
import pytest

import oracle
from tests import _problems as P
from tests.gpu_common import compare

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1909_02294_amd import ivde, synth  # noqa: E402


def _case(name):
    print(f"[case] {name}", flush=True)


@pytest.mark.parametrize("chroma,bits", [(0, 8), (1, 10), (1, 12), (0, 16)])
def test_segment_stats(chroma, bits):
    _case(f"stats {chroma} {bits}")
    ns = P.tiny_problem(50 + bits, n_views=3, width=57, height=31, n_seg=25, L=2, chroma_shift=chroma, bit_depth=bits)
    ns.S = [s + 2 for s in ns.S]                       # two empty segments per view
    dv = ivde.DeviceViews(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift)
    cnt, cen, mean, _ = ivde.segment_stats(dv)
    torch.cuda.synchronize()
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, bits, chroma, 1.0, 2.0, 1, False)
    oc, ocen, omean = oracle.all_segment_stats(pb)
    np.testing.assert_array_equal(cnt.cpu().numpy(), oc)
    np.testing.assert_array_equal(cen.cpu().numpy(), ocen)
    g = mean.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(g[:, :3], omean, rtol=1e-6, atol=1e-6)
    assert np.all(g[:, 3] == 0)


def test_segment_stats_one_pixel_segments_and_several_tiles():
    """Every pixel its own segment on a 150 x 40 image (1024 distinct ids per
    64 x 16 tile, more than the per-tile table holds, so most sums take the
    direct global path), in a shuffled order, beside a view of large random
    segments: counts, centres and means exact against the oracle."""
    _case("stats one-pixel segments")
    ns = P.tiny_problem(77, n_views=2, width=150, height=40, n_seg=30, L=2, chroma_shift=1, bit_depth=10)
    rng = np.random.default_rng(3)
    ns.seg[0] = rng.permutation(150 * 40).reshape(40, 150).astype(np.int32)
    ns.S[0] = 150 * 40
    dv = ivde.DeviceViews(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift)
    cnt, cen, mean, ws = ivde.segment_stats(dv)
    torch.cuda.synchronize()
    assert ivde.workspace_status(ws) == ivde.IVDE_OK
    pb = oracle.Problem(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, 10, 1, 1.0, 2.0, 1, False)
    oc, ocen, omean = oracle.all_segment_stats(pb)
    np.testing.assert_array_equal(cnt.cpu().numpy(), oc)
    np.testing.assert_array_equal(cen.cpu().numpy(), ocen)
    np.testing.assert_allclose(mean.cpu().numpy()[:, :3].astype(np.float64), omean, rtol=1e-6, atol=1e-6)


def test_segment_stats_reports_out_of_range_ids():
    _case("stats bad id")
    ns = P.tiny_problem(78, n_views=2, width=40, height=20, n_seg=8, L=2)
    ns.seg[1] = ns.seg[1].copy()
    ns.seg[1][5, 7] = ns.S[1] + 3
    dv = ivde.DeviceViews(ns.cams, ns.Y, ns.U, ns.V, ns.seg, ns.S, ns.bit_depth, ns.chroma_shift)
    *_, ws = ivde.segment_stats(dv)
    torch.cuda.synchronize()
    assert ivde.workspace_status(ws) == ivde.IVDE_EINVAL


def test_temporal_rule_kernel():
    _case("rule kernel")
    rng = np.random.default_rng(5)
    R = 5000
    # eighths are exact in FP32 and FP64, so both sides decide alike
    prev = np.round(rng.uniform(0, 1023, (R, 4)) * 8) / 8
    prev[:, 3] = 0
    cur = prev + np.round(rng.normal(0, 8, (R, 4)) * 8) / 8
    ifr = prev + np.round(rng.normal(0, 3, (R, 4)) * 8) / 8
    cur[:, 3] = ifr[:, 3] = 0
    for bits in (8, 10):
        for use_i in (True, False):
            got = ivde.temporal_rule(torch.tensor(cur, dtype=torch.float32).cuda(),
                                     torch.tensor(prev, dtype=torch.float32).cuda(),
                                     torch.tensor(ifr, dtype=torch.float32).cuda() if use_i else None,
                                     3.0, 1.0, bits).cpu().numpy()
            want = oracle.temporal_rule(cur, prev, ifr if use_i else None, 3.0, 1.0, bits)
            np.testing.assert_array_equal(got, want)
            assert len(np.unique(want)) >= 2


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_server_rule_frames_match_oracle(dtype):
    """Frame 0 is the I frame; frames 1..4 take the rule.  Rows whose mean
    colour change lies within 0.05 code values of a threshold may be decided
    differently by FP32 and FP64 means and are left out of the comparison."""
    _case(f"served rule {dtype}")
    f16 = dtype == "f16"
    wl = synth.make_small_arc(seed=61, n_views=4, width=160, height=96, n_segments=140, num_labels=48)
    frames = synth.make_sequence(wl, 5, seed=62)
    srv = ivde.Server(1 << 30, max_slots=2)
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    rid = srv.register(dv, lr, ivde.options(ivde.BILINEAR, ivde.F16 if f16 else ivde.F32))
    outs, stats = [], []
    for i, fr in enumerate(frames):
        img = ivde.DeviceViews(wl.cams, fr["Y"], fr["U"], fr["V"], wl.seg, wl.S, wl.bit_depth, wl.chroma_shift)
        out = torch.empty((dv.rows, wl.num_labels), dtype=torch.float16 if f16 else torch.float32, device="cuda")
        stats.append(srv.wait(srv.submit_rule(rid, img.c_images, iframe=(i == 0), cost_out=out)))
        outs.append(out.double().cpu().numpy())
    srv.close()
    scale = float(1 << (wl.bit_depth - 8))
    prev = ifr_cost = None
    mean_prev = mean_i = None
    total_checked = 0
    for i, fr in enumerate(frames):
        pb = oracle.Problem(wl.cams, fr["Y"], fr["U"], fr["V"], wl.seg, wl.S, wl.bit_depth, wl.chroma_shift,
                            wl.z_near, wl.z_far, wl.num_labels, True)
        _, _, mean = oracle.all_segment_stats(pb)
        if i == 0:
            want = oracle.cost_volume(pb)
            keep = np.ones(len(want), bool)
            ifr_cost, mean_i = want, mean
            assert stats[i]["rows_recomputed"] == stats[i]["rows_total"]
        else:
            src = oracle.temporal_rule(mean, mean_prev, mean_i, 3.0, 1.0, wl.bit_depth)
            want = oracle.served_rule(prev, ifr_cost, pb, src)
            dp = np.abs(mean - mean_prev).max(1)
            di = np.abs(mean - mean_i).max(1)
            keep = (np.abs(dp - 3.0 * scale) > 0.05) & (np.abs(di - 1.0 * scale) > 0.05)
            if keep.all():
                assert stats[i]["rows_recomputed"] == int((src == 0).sum())
                assert stats[i]["rows_from_iframe"] == int((src == 2).sum())
            assert (src == 0).any() and (src != 0).any()
        compare(outs[i][keep], want[keep], f16=f16, label=f"frame {i}")
        total_checked += keep.sum()
        prev, mean_prev = want, mean
    assert total_checked >= 0.99 * len(frames) * outs[0].shape[0]


def test_server_fp16_odd_label_and_row_counts():
    """FP16 storage with an odd number of levels and of rows: every row of
    the resident volume, every I-frame copy and every cost_out copy is a
    whole number of 2-byte entries but not of 4-byte words.  Rule frames and
    masked frames must equal the same frames served with FP32 storage after
    rounding (the FP16 store rounds the FP32 result)."""
    _case("served fp16 odd L and rows")
    wl = synth.make_small_arc(seed=63, n_views=3, width=128, height=80, n_segments=139, num_labels=47)
    assert sum(wl.S) % 2 == 1 and wl.num_labels % 2 == 1
    frames = synth.make_sequence(wl, 4, seed=64)
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    outs = {}
    for dtype, tdt in ((ivde.F16, torch.float16), (ivde.F32, torch.float32)):
        srv = ivde.Server(1 << 30, max_slots=2)
        rid_rule = srv.register(dv, lr, ivde.options(ivde.BILINEAR, dtype))
        rid_mask = srv.register(dv, lr, ivde.options(ivde.BILINEAR, dtype))
        got = []
        for i, fr in enumerate(frames):
            img = ivde.DeviceViews(wl.cams, fr["Y"], fr["U"], fr["V"], wl.seg, wl.S, wl.bit_depth, wl.chroma_shift)
            a = torch.empty((dv.rows, wl.num_labels), dtype=tdt, device="cuda")
            b = torch.empty((dv.rows, wl.num_labels), dtype=tdt, device="cuda")
            la = torch.empty(dv.rows, dtype=torch.int32, device="cuda")
            st = srv.wait(srv.submit_rule(rid_rule, img.c_images, iframe=(i == 0), cost_out=a, label_out=la))
            assert st["status"] == 0
            m = None if fr["mask"] is None else torch.from_numpy(np.concatenate(fr["mask"]).astype(np.uint8)).cuda()
            st = srv.wait(srv.submit(rid_mask, img.c_images, m, b))
            assert st["status"] == 0
            assert torch.equal(la, ivde.argmin(a))
            got.append((a.clone(), b.clone()))
        srv.close()
        outs[dtype] = got
    for (a16, b16), (a32, b32) in zip(outs[ivde.F16], outs[ivde.F32]):
        assert torch.equal(a16, a32.half()) and torch.equal(b16, b32.half())
