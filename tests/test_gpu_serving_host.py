"""GPU tests of two serving features: frames handed over in host memory
(the server uploads them on the request's stream, so the upload is part of
the frame's latency) and full-frame sweeps cut into several launches (so
that short frames of other rigs do not wait for a whole I frame).  Neither
may change a result: every served volume and label must be bitwise the one
the unchunked device-memory path gives, alone and in a mix of rigs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1909_02294_amd import ivde, synth  # noqa: E402


def _case(name):
    print(f"[case] {name}", flush=True)


def _sequence(seed, n_views, width, height, n_seg, L, n_frames):
    wl = synth.make_small_arc(seed=seed, n_views=n_views, width=width, height=height, n_segments=n_seg,
                              num_labels=L)
    return wl, synth.make_sequence(wl, n_frames, seed=seed + 1)


def _evals(wl):
    return sum(c.width * c.height for c in wl.cams) * wl.num_labels * (wl.n_views - 1)


def _serve(wl, frames, dtype, chunk_evals, host, rule, slots=2):
    """Serves every frame of one rig, one after another; returns the cost
    and label of each frame and its stats."""
    tdt = torch.float16 if dtype == ivde.F16 else torch.float32
    srv = ivde.Server(1 << 30, max_slots=slots, chunk_evals=chunk_evals)
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    rid = srv.register(dv, lr, ivde.options(ivde.BILINEAR, dtype))
    out = []
    for i, fr in enumerate(frames):
        cost = torch.full((dv.rows, wl.num_labels), -3.0, dtype=tdt, device="cuda")
        lab = torch.full((dv.rows,), -1, dtype=torch.int32, device="cuda")
        mask = None if fr["mask"] is None else np.concatenate(fr["mask"]).astype(np.uint8)
        if host:
            hf = ivde.HostFrame(wl.n_views, fr["Y"], fr["U"], fr["V"], wl.bit_depth, wl.chroma_shift,
                                mask=None if rule else mask)
            mode = (ivde.SUBMIT_RULE_IFRAME if i == 0 else ivde.SUBMIT_RULE) if rule else ivde.SUBMIT_MASK
            t = srv.submit_host(rid, hf, mode, cost_out=cost, label_out=lab)
        else:
            img = ivde.DeviceViews(wl.cams, fr["Y"], fr["U"], fr["V"], wl.seg, wl.S, wl.bit_depth, wl.chroma_shift)
            if rule:
                t = srv.submit_rule(rid, img.c_images, iframe=(i == 0), cost_out=cost, label_out=lab)
            else:
                dm = None if mask is None else torch.from_numpy(mask).cuda()
                t = srv.submit(rid, img.c_images, dm, cost, lab)
        st = srv.wait(t)
        assert st["status"] == 0
        assert st["submit_us"] <= st["start_us"] <= st["done_us"]
        out.append((cost, lab, st))
    srv.close()
    return out


@pytest.mark.parametrize("rule", [False, True])
@pytest.mark.parametrize("dtype", [ivde.F32, ivde.F16])
def test_host_frames_and_cut_sweeps_equal_device_frames(rule, dtype):
    """The same frames through the device-memory path in one launch per
    sweep, and through the host-memory path with every full sweep cut into
    about nine launches (and into launches of a single task): bitwise equal
    costs, labels and row counts."""
    _case(f"host frames, cut sweeps, rule={rule}, dtype={dtype}")
    wl, frames = _sequence(71, 4, 160, 96, 140, 48, 4)
    ev = _evals(wl)
    ref = _serve(wl, frames, dtype, -1, host=False, rule=rule)
    for chunk in (ev // 9, 1):
        got = _serve(wl, frames, dtype, chunk, host=True, rule=rule)
        for i, ((c0, l0, s0), (c1, l1, s1)) in enumerate(zip(ref, got)):
            assert torch.equal(c0, c1), f"frame {i}, chunk {chunk}: costs differ"
            assert torch.equal(l0, l1), f"frame {i}, chunk {chunk}: labels differ"
            assert torch.equal(l1, ivde.argmin(c1))
            for k in ("rows_recomputed", "rows_from_iframe", "rows_total"):
                assert s0[k] == s1[k], (i, k, s0[k], s1[k])
    # the first frame swept every row, later frames only changed ones
    assert ref[0][2]["rows_recomputed"] == ref[0][2]["rows_total"]
    assert all(s["rows_recomputed"] < s["rows_total"] for _, _, s in ref[1:])


def test_cut_sweeps_in_a_mix_of_rigs():
    """Three rigs, every frame submitted at once into four slots, full
    sweeps cut into about six launches, one rig handing over host frames and
    its rule deciding the rows: each rig's frames equal its frames served
    alone in one launch per sweep from device memory."""
    _case("cut sweeps in a mix")
    seqs = [_sequence(80, 3, 120, 72, 90, 64, 5), _sequence(81, 4, 160, 96, 150, 96, 5),
            _sequence(82, 5, 128, 80, 100, 48, 5)]
    setups = [(ivde.F16, True, False), (ivde.F16, False, True), (ivde.F32, False, False)]   # dtype, host, rule
    alone = [_serve(wl, fr, dt, -1, host=False, rule=rule) for (wl, fr), (dt, _, rule) in zip(seqs, setups)]
    chunk = min(_evals(wl) for wl, _ in seqs) // 6
    srv = ivde.Server(2 << 30, max_slots=4, chunk_evals=chunk)
    rigs = []
    for (wl, fr), (dt, host, rule) in zip(seqs, setups):
        dv = ivde.DeviceViews.from_workload(wl)
        lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
        rigs.append(dict(wl=wl, fr=fr, dt=dt, host=host, rule=rule, dv=dv,
                         rid=srv.register(dv, lr, ivde.options(ivde.BILINEAR, dt))))
    tickets, outs, keep = [], [], []
    for i in range(5):
        for k, r in enumerate(rigs):
            wl, fr = r["wl"], r["fr"][i]
            tdt = torch.float16 if r["dt"] == ivde.F16 else torch.float32
            cost = torch.empty((r["dv"].rows, wl.num_labels), dtype=tdt, device="cuda")
            lab = torch.empty(r["dv"].rows, dtype=torch.int32, device="cuda")
            mask = None if fr["mask"] is None else np.concatenate(fr["mask"]).astype(np.uint8)
            if r["host"]:
                hf = ivde.HostFrame(wl.n_views, fr["Y"], fr["U"], fr["V"], wl.bit_depth, wl.chroma_shift, mask=mask)
                keep.append(hf)
                t = srv.submit_host(r["rid"], hf, ivde.SUBMIT_MASK, cost_out=cost, label_out=lab)
            else:
                img = ivde.DeviceViews(wl.cams, fr["Y"], fr["U"], fr["V"], wl.seg, wl.S, wl.bit_depth,
                                       wl.chroma_shift)
                keep.append(img)
                if r["rule"]:
                    t = srv.submit_rule(r["rid"], img.c_images, iframe=(i == 0), cost_out=cost, label_out=lab)
                else:
                    dm = None if mask is None else torch.from_numpy(mask).cuda()
                    keep.append(dm)
                    t = srv.submit(r["rid"], img.c_images, dm, cost, lab)
            tickets.append((k, i, t))
            outs.append((k, i, cost, lab))
    stats = {(k, i): srv.wait(t) for k, i, t in tickets}
    srv.close()
    assert all(s["status"] == 0 for s in stats.values())
    for k, i, cost, lab in outs:
        c0, l0, s0 = alone[k][i]
        assert torch.equal(cost, c0), f"rig {k} frame {i}: costs differ in the mix"
        assert torch.equal(lab, l0), f"rig {k} frame {i}: labels differ in the mix"
        assert stats[(k, i)]["rows_recomputed"] == s0["rows_recomputed"]
    # frames of one rig completed in submission order
    for k in range(3):
        done = [stats[(k, i)]["done_us"] for i in range(5)]
        assert done == sorted(done)
