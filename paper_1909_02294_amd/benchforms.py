"""Benchmarks of the batched and served forms (bench.py --mode batched|served).

Batched: 16 frames of the 8-view 1920x1080 arc-rig generator with segment
counts U{5000..40000} and label counts from {128, 256}; one persistent-kernel
launch in a hipGraph, launch shape from the autotuner, against 16 sequential
plain launches on the same inputs.

Served: a Poisson stream of 60 frames/s in total from three rigs (4 views
1280x720 at 64 labels, 8 views 1920x1080 at 256 labels, 10 views 2048x1088 at
256 labels, FP16 costs, 80 GB arena); each P frame moves 2-6 planes and its
changed-segment mask drives the recompute; with --gop G every G-th frame of a
rig is an I frame (every row; the paper's schedule has 9 P frames between I
frames, Sec. V-A); the same arrivals are replayed with every frame recomputed
in full.
"""
from __future__ import annotations

import sys
import time

import numpy as np

from paper_1909_02294_amd import ivde, synth


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _evals(wl):
    return int(sum(c.width * c.height for c in wl.cams) * wl.num_labels * (wl.n_views - 1))


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs, np.float64), q))


def _batch_case(wls, args):
    """Sequential plain calls against one batched launch on the frames
    `wls`: times, per-frame sweep rates, shapes and bitwise equality."""
    import torch

    stream = torch.cuda.Stream()        # the graph is captured on a non-null stream
    dvs = [ivde.DeviceViews.from_workload(wl) for wl in wls]
    lrs = [ivde.label_range(wl.z_near, wl.z_far, wl.num_labels) for wl in wls]
    # the launch shape: tuned once per shape class (cached), the batch takes
    # the shape of the class that carries the most evaluations
    base = ivde.options(ivde.BILINEAR, ivde.F32)
    classes = {}
    for i, (dv, lr, wl) in enumerate(zip(dvs, lrs, wls)):
        classes.setdefault(ivde.shape_class(dv, lr, base), []).append(i)
    shapes, table = {}, {}
    for key, members in classes.items():
        o, t = ivde.autotune_cached(dvs[members[0]], lrs[members[0]], base, args.tune_cache, reps=1)
        shapes[key] = (o.labels_per_lane, o.waves_per_group, o.pixels_per_step)
        table[key] = t
    weight = {k: sum(_evals(wls[i]) for i in m) for k, m in classes.items()}
    main_class = max(weight, key=weight.get)
    tuned = ivde.options(ivde.BILINEAR, ivde.F32, labels_per_lane=shapes[main_class][0],
                         waves_per_group=shapes[main_class][1], pixels_per_step=shapes[main_class][2])
    _log(f"shape classes {shapes}; batch shape {shapes[main_class]} from {main_class}")
    opt = ivde.options(ivde.BILINEAR, ivde.F32, labels_per_lane=tuned.labels_per_lane,
                       waves_per_group=tuned.waves_per_group)
    costs = [torch.empty((dv.rows, wl.num_labels), dtype=torch.float32, device="cuda") for dv, wl in zip(dvs, wls)]
    labs = [torch.empty(dv.rows, dtype=torch.int32, device="cuda") for dv in dvs]
    # plain: one workspace of the largest size, 16 launches back to back
    wsz = max(ivde.sizes(dv, lr, opt)[1] for dv, lr in zip(dvs, lrs))
    ws = ivde.alloc_bytes(wsz)

    def plain_pass():
        for dv, lr, c, l in zip(dvs, lrs, costs, labs):
            ivde.cost_volume(dv, lr, opt, workspace=ws, out=c, stream=stream)
            ivde.argmin(c, stream=stream, out=l)

    evals = sum(_evals(wl) for wl in wls)
    K, W = args.steps, args.warmup

    def timed(fn):
        for _ in range(W):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        t = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / K, [a.elapsed_time(b) for a, b in ev]

    plain_s, plain_lat = timed(plain_pass)
    ref = [c.clone() for c in costs]
    _log(f"plain: {plain_s * 1e3:.1f} ms per 16 frames")
    # each frame's own sweep, event-timed (median of 3 plain calls)
    per_frame = []
    for i, (dv, lr, c, wl) in enumerate(zip(dvs, lrs, costs, wls)):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for e in evs:
            o = ivde.options(ivde.BILINEAR, ivde.F32, labels_per_lane=tuned.labels_per_lane,
                             waves_per_group=tuned.waves_per_group, sweep_events=e)
            ivde.cost_volume(dv, lr, o, workspace=ws, out=c, stream=stream)
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
        per_frame.append({"frame": i, "segments": int(sum(wl.S)), "labels": wl.num_labels,
                          "pixels_per_segment": float(sum(cc.width * cc.height for cc in wl.cams) / sum(wl.S)),
                          "class": ivde.shape_class(dv, lr, base), "sweep_ms": ms,
                          "evals_per_s": _evals(wl) / (ms / 1e3)})
    groups = {}
    for f in per_frame:
        key = f"L{f['labels']}"
        g = groups.setdefault(key, {"frames": 0, "evals": 0, "ms": 0.0})
        g["frames"] += 1
        g["evals"] += _evals(wls[f["frame"]])
        g["ms"] += f["sweep_ms"]
    for g in groups.values():
        g["evals_per_s"] = g["evals"] / (g["ms"] / 1e3)
    sweep_ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    bopt = ivde.options(ivde.BILINEAR, ivde.F32, labels_per_lane=tuned.labels_per_lane,
                        waves_per_group=tuned.waves_per_group, sweep_events=sweep_ev)
    batch = ivde.Batch([(dv, lr, c, l) for dv, lr, c, l in zip(dvs, lrs, costs, labs)], bopt)
    for c in costs:
        c.fill_(-1.0)
    torch.cuda.synchronize()
    batch_s, batch_lat = timed(lambda: batch.run(stream, use_graph=True))
    # the persistent sweep alone, from one eager run with its events
    batch.run(stream, use_graph=False)
    torch.cuda.synchronize()
    sweep_ms = sweep_ev[0].elapsed_time(sweep_ev[1])
    identical = all(torch.equal(c, r) for c, r in zip(costs, ref))
    _log(f"batched: {batch_s * 1e3:.1f} ms per 16 frames, identical to plain: {identical}")
    achieved = evals * 24 / (sweep_ms / 1e3) / 1e9
    batch.close()
    return {
        "evals": evals, "batch_s": batch_s, "K": K, "W": W,
        "config": {"segments": [int(sum(wl.S)) for wl in wls], "labels": [wl.num_labels for wl in wls],
                   "evals_per_step": evals,
                   "launch_shape": {"labels_per_lane": tuned.labels_per_lane,
                                    "waves_per_group": tuned.waves_per_group, "from_class": main_class},
                   "shape_classes": {k: {"frames": len(classes[k]), "shape": shapes[k],
                                         "autotune_us": ({"x".join(map(str, a)): v for a, v in table[k].items()}
                                                         if table[k] else "cached")} for k in classes}},
        "per_frame_sweep": per_frame,
        "sweep_rate_by_labels": groups,
        "plain_16_sequential": {"value": evals / plain_s, "ms_per_step": plain_s * 1e3,
                                "latency_ms": {"p50": _pct(plain_lat, 50), "p99": _pct(plain_lat, 99)}},
        "speedup_vs_plain": plain_s / batch_s,
        "bitwise_equal_to_plain": identical,
        "latency_ms": {"p50": _pct(batch_lat, 50), "p99": _pct(batch_lat, 99)},
        "persistent_sweep_ms": sweep_ms,
        "hbm_metric": {"bytes_per_eval": 24, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                       "frac": achieved / 8000.0},
    }


def bench_batched(args):
    t0 = time.perf_counter()
    wls = synth.make_batch_frames(16)
    _log(f"generated 16 frames in {time.perf_counter() - t0:.1f} s")
    big = _batch_case(wls, args)
    # frames too small to fill the GPU one at a time: 16 frames of 4 views
    # 320x240 with 300-1200 segments per view and 64 or 96 levels
    small = synth.make_batch_frames(16, seed=synth.SEED_BATCH + 77, width=320, height=240, n_views=4,
                                    seg_range=(300, 1200), label_choices=(64, 96))
    _log("small frames")
    sm = _batch_case(small, args)
    evals, batch_s = big.pop("evals"), big.pop("batch_s")
    K, W = big.pop("K"), big.pop("W")
    cfg = big.pop("config")
    cfg["workload"] = ("16 frames x 8 views 1920x1080 YUV420 10-bit arc rig, segments U{5000..40000}, "
                       "labels {128, 256}, bilinear, FP32 costs; one persistent launch in a hipGraph")
    return {
        "metric": "pixel·label·view cost evals/s + %HBM roofline; p50/p99 frame latency",
        "value": evals / batch_s, "unit": "evals/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": batch_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic", "config": cfg, **big,
        "small_frames": {"workload": "16 frames x 4 views 320x240 YUV420 10-bit arc rig, segments U{300..1200}, "
                                     "labels {64, 96}, bilinear, FP32 costs",
                         "evals_per_step": sm["evals"], "batched_ms": sm["batch_s"] * 1e3,
                         "plain_16_sequential_ms": sm["plain_16_sequential"]["ms_per_step"],
                         "speedup_vs_plain": sm["speedup_vs_plain"],
                         "bitwise_equal_to_plain": sm["bitwise_equal_to_plain"],
                         "persistent_sweep_ms": sm["persistent_sweep_ms"]},
    }


# ---------------------------------------------------------------- served
RIGS = [
    dict(name="A", n_views=4, width=1280, height=720, n_segments=8900, num_labels=64),
    dict(name="B", n_views=8, width=1920, height=1080, n_segments=20000, num_labels=256),
    dict(name="C", n_views=10, width=2048, height=1088, n_segments=21500, num_labels=256),
]


def _make_rig(spec, seed, n_frames):
    arc = 30.0 * (spec["n_views"] - 1) / 7.0        # same spacing as the 8-view rig
    f = 1400.0 * spec["width"] / 1920.0
    wl = synth.make_arc_workload(f"rig{spec['name']}", seed, n_views=spec["n_views"], width=spec["width"],
                                 height=spec["height"], f=f, n_segments=spec["n_segments"],
                                 num_labels=spec["num_labels"], arc_deg=arc)
    frames = synth.make_sequence(wl, n_frames, seed + 7, tries=3)
    return wl, frames


def bench_served(args):
    import torch

    n_cycle = args.served_frames
    rigs = []
    t0 = time.perf_counter()
    for i, spec in enumerate(RIGS):
        wl, frames = _make_rig(spec, synth.SEED_SERVING + 17 * i, n_cycle)
        rigs.append((spec, wl, frames))
        _log(f"rig {spec['name']}: {len(frames)} frames, change rates "
             f"{[round(f['rate'], 3) for f in frames[1:]]} ({time.perf_counter() - t0:.0f} s)")
    arena_bytes = 80 << 30
    duration = args.served_seconds
    rate = 60.0
    rng = np.random.default_rng(synth.SEED_SERVING)
    n_req = int(duration * rate)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n_req))
    which = rng.integers(0, len(rigs), n_req)
    host = not args.device_frames

    # ping-pong through each rig's frames: 0 1 2 .. n-1 n-2 .. 1 0 1 ...; a
    # step back changes the same segments as the step forward
    def frame_index(k):
        period = 2 * (n_cycle - 1)
        m = k % period
        return m if m < n_cycle else period - m

    rule = args.rule
    # every frame's planes (and masks) in pinned host memory, as a capture
    # process delivers them; with --device-frames, resident on the device
    frames_in = []
    for spec, wl, frames in rigs:
        if host:
            fin = [ivde.HostFrame(wl.n_views, f["Y"], f["U"], f["V"], wl.bit_depth, wl.chroma_shift,
                                  mask=None if f["mask"] is None else np.concatenate(f["mask"]).astype(np.uint8))
                   for f in frames]
        else:
            fin = [(ivde.DeviceViews(wl.cams, f["Y"], f["U"], f["V"], wl.seg, wl.S, wl.bit_depth, wl.chroma_shift),
                    None if f["mask"] is None
                    else torch.from_numpy(np.concatenate(f["mask"]).astype(np.uint8)).cuda()) for f in frames]
        frames_in.append(fin)

    # host frames without a mask (I frames) and with the mask of the step
    # that reaches them from the next frame
    extra = []
    for spec, wl, frames in rigs:
        nomask, withmask = {}, {}
        if host and not rule:
            for fi, f in enumerate(frames):
                nomask[fi] = ivde.HostFrame(wl.n_views, f["Y"], f["U"], f["V"], wl.bit_depth, wl.chroma_shift)
                if fi + 1 < len(frames):
                    m = np.concatenate(frames[fi + 1]["mask"]).astype(np.uint8)
                    withmask[(fi, fi + 1)] = ivde.HostFrame(wl.n_views, f["Y"], f["U"], f["V"], wl.bit_depth,
                                                            wl.chroma_shift, mask=m)
        extra.append(dict(nomask=nomask, withmask=withmask))

    def submit(srv, st, fi, iframe, mask_from):
        if host:
            hf = frames_in[st["ri"]][fi]
            if rule:
                mode = ivde.SUBMIT_RULE_IFRAME if iframe else ivde.SUBMIT_RULE
            else:
                mode = ivde.SUBMIT_MASK
                if iframe:
                    hf = st["nomask"][fi]
                elif mask_from != fi:
                    hf = st["withmask"][(fi, mask_from)]
            return srv.submit_host(st["rid"], hf, mode, label_out=st["labs"])
        img, _ = frames_in[st["ri"]][fi]
        if rule:
            return srv.submit_rule(st["rid"], img.c_images, iframe=iframe, label_out=st["labs"])
        mask = None if iframe else frames_in[st["ri"]][mask_from][1]
        return srv.submit(st["rid"], img.c_images, mask, None, st["labs"])

    def run(temporal: bool, chunk_evals: int):
        srv = ivde.Server(arena_bytes, max_slots=args.slots, chunk_evals=chunk_evals)
        state = []
        for ri, (spec, wl, frames) in enumerate(rigs):
            dv = ivde.DeviceViews.from_workload(wl)
            lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
            opt = ivde.options(ivde.BILINEAR, ivde.F16)
            rid = srv.register(dv, lr, opt)
            labs = torch.empty(dv.rows, dtype=torch.int32, device="cuda")
            st = dict(ri=ri, rid=rid, labs=labs, count=1, last=0, wl=wl, **extra[ri])
            state.append(st)
        torch.cuda.synchronize()
        # each rig's first frame (an I frame: every row) fills its resident
        # volume before the arrival clock starts
        for st in state:
            srv.wait(submit(srv, st, 0, True, 0))
        tickets = []
        t_start = time.perf_counter()
        for k in range(n_req):
            target = t_start + arrivals[k]
            while True:
                d = target - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 0.002))
            st = state[which[k]]
            fi = frame_index(st["count"])
            iframe = not temporal or (args.gop > 0 and st["count"] % args.gop == 0)
            st["count"] += 1
            # the mask of a step between frames fi and last marks the same
            # segments either way; frames store the forward step's mask
            t = submit(srv, st, fi, iframe, max(fi, st["last"]))
            st["last"] = fi
            tickets.append((which[k], iframe, t))
        stats = [(r, i, srv.wait(t)) for r, i, t in tickets]
        wall = time.perf_counter() - t_start
        srv.close()
        lat = [s["latency_ms"] for _, _, s in stats]
        swept = sum(s["rows_recomputed"] / max(s["rows_total"], 1) * _evals(rigs[r][1]) for r, _, s in stats)
        per_rig = {}
        for ri, (spec, wl, frames) in enumerate(rigs):
            l = [s["latency_ms"] for r, _, s in stats if r == ri]
            per_rig[spec["name"]] = {"frames": len(l), "p50_ms": _pct(l, 50), "p99_ms": _pct(l, 99)}
        # a frame that arrived while its rig's previous frame was still in
        # flight waits for it by construction (it starts from that frame's
        # volume); the others wait only for the device
        behind = []
        last_done = {}
        for r, i, s in stats:
            behind.append(last_done.get(r, -1.0) > s["submit_us"])
            last_done[r] = s["done_us"]
        from_i = float(np.mean([s["rows_from_iframe"] / max(s["rows_total"], 1) for _, _, s in stats]))
        out = {"frames": len(stats), "wall_s": wall, "frames_per_s": len(stats) / wall,
               "from_iframe_fraction": from_i,
               "swept_evals_per_s": swept / wall,
               "latency_ms": {"p50": _pct(lat, 50), "p90": _pct(lat, 90), "p99": _pct(lat, 99), "max": max(lat)},
               "recomputed_fraction": float(np.mean([s["rows_recomputed"] / max(s["rows_total"], 1)
                                                     for _, _, s in stats])),
               "per_rig": per_rig}
        for kind, flag in (("p_frames", False), ("i_frames", True)):
            sel = [(s["latency_ms"], b) for (_, i, s), b in zip(stats, behind) if i == flag]
            if sel and temporal:
                l = [x for x, _ in sel]
                out[kind] = {"frames": len(l), "p50_ms": _pct(l, 50), "p90_ms": _pct(l, 90), "p99_ms": _pct(l, 99)}
                free = [x for x, b in sel if not b]
                tied = [x for x, b in sel if b]
                if free:
                    out[kind]["own_rig_idle"] = {"frames": len(free), "p50_ms": _pct(free, 50),
                                                 "p99_ms": _pct(free, 99)}
                if tied:
                    out[kind]["behind_own_rig"] = {"frames": len(tied), "p50_ms": _pct(tied, 50),
                                                   "p99_ms": _pct(tied, 99)}
        return out

    chunks = [int(float(c)) for c in str(args.chunk_evals).split(",")]
    _log(f"temporal run, cut full sweeps ({chunks[0] or 'default'} evaluations per launch)")
    tmp = run(True, chunks[0])
    by_chunk = {}
    for c in chunks[1:]:
        _log(f"temporal run, {c} evaluations per launch")
        r = run(True, c)
        by_chunk[str(c)] = {k: r[k] for k in ("latency_ms", "p_frames", "i_frames", "frames_per_s") if k in r}
    uncut = None
    if args.gop > 0 and not args.no_uncut:
        _log("temporal run, full sweeps in one launch")
        uncut = run(True, -1)
    _log("full-recompute run")
    full = run(False, chunks[0])
    demand_full = sum(_evals(wl) for _, wl, _ in rigs) / len(rigs) * rate
    return {
        "metric": "pixel·label·view cost evals/s + %HBM roofline; p50/p99 frame latency",
        "value": tmp["frames_per_s"], "unit": "frames/s", "n_gpus": 1, "steps": n_req, "warmup": 0,
        "ms_per_step": tmp["wall_s"] / max(tmp["frames"], 1) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (FP16 storage)", "data": "synthetic",
        "config": {"workload": "Poisson 60 frames/s from rigs A (4x1280x720, 64 labels), B (8x1920x1080, 256), "
                               "C (10x2048x1088, 256); YUV420 10-bit, bilinear, FP16 costs, 80 GB arena",
                   "seconds": duration, "slots": args.slots, "gop": args.gop,
                   "distinct_frames_per_rig": n_cycle,
                   "chunk_evals": chunks[0] or "library default (8e9)",
                   "mask": "temporal rule on the GPU (T_P = 3, T_I = 1)" if rule else "changed-segment mask input",
                   "protocol": "each rig's first (I) frame is computed before the arrival clock; " +
                               ("frames in pinned host memory, uploaded by the server on the request's stream; "
                                "latency = arrival (submit) to completion, upload included" if host else
                                "images resident on the device; latency = submit to completion, no upload"),
                   "change_rates": {s["name"]: [round(f["rate"], 3) for f in fr[1:]] for s, _, fr in rigs}},
        "latency_ms": tmp["latency_ms"],
        "temporal": tmp,
        "temporal_uncut_sweeps": uncut,
        "temporal_other_chunk_sizes": by_chunk,
        "full_recompute": full,
        "load_factor_full": demand_full / max(full["swept_evals_per_s"], 1.0),
    }


# ---------------------------------------------------------------- shapes
def bench_shapes(args):
    """Sweep rate of the plain single-frame call by shape class: the 8-view
    1920x1080 arc scene (10-bit, or --bit-depth) segmented into 5000, 10000,
    20000 and 40000 segments per view (the batching workload's range) at 128
    and 256 levels, each
    with the launch shape the autotuner picks for it (cached per shape
    class).  Explains per-frame rates inside a batch."""
    import torch

    rows = []
    samp = ivde.NEAREST if args.sampling == "nearest" else ivde.BILINEAR
    cache = args.tune_cache
    stream = torch.cuda.current_stream()
    seg_list = [int(x) for x in args.shape_segments.split(",")]
    lab_list = [int(x) for x in args.shape_labels.split(",")]
    for S in seg_list:
        t0 = time.perf_counter()
        wl = synth.make_arc_workload(f"shapes-S{S}", synth.SEED_BATCH + 5, n_segments=S, num_labels=256,
                                     bit_depth=args.bit_depth)
        dv = ivde.DeviceViews.from_workload(wl)
        _log(f"S={S}: generated in {time.perf_counter() - t0:.1f} s, {dv.rows} rows")
        for L in lab_list:
            lr = ivde.label_range(wl.z_near, wl.z_far, L)
            base = ivde.options(samp, ivde.F32, pixels_per_step=args.pixels_per_step)
            if args.no_tune:
                tuned, table = base, None
            else:
                tuned, table = ivde.autotune_cached(dv, lr, base, cache, reps=2)
            res = {}
            variants = [("j1", base)]
            if not args.no_tune:
                variants.append(("tuned", tuned))
            if args.compare_px:
                variants.append(("one", ivde.options(samp, ivde.F32, labels_per_lane=1, pixels_per_step=1)))
                variants.append(("pairs", ivde.options(samp, ivde.F32, labels_per_lane=1, pixels_per_step=2)))
                variants.append(("quads", ivde.options(samp, ivde.F32, labels_per_lane=1, pixels_per_step=4)))
            for name, o in variants:
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(args.steps)]
                opts = [ivde.options(samp, ivde.F32, labels_per_lane=o.labels_per_lane,
                                     waves_per_group=o.waves_per_group, sweep_events=e,
                                     pixels_per_step=o.pixels_per_step) for e in ev]
                C, ws = ivde.cost_volume(dv, lr, opts[0])
                torch.cuda.synchronize()
                for op in opts:
                    ivde.cost_volume(dv, lr, op, workspace=ws, out=C, stream=stream)
                torch.cuda.synchronize()
                ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
                evals = sum(c.width * c.height for c in wl.cams) * L * (wl.n_views - 1)
                res[name] = {"sweep_ms": ms, "evals_per_s": evals / (ms / 1e3),
                             "labels_per_lane": o.labels_per_lane or 1, "waves_per_group": o.waves_per_group,
                             "pixels_per_step": o.pixels_per_step,
                             "pair_wave_steps": dict(zip(("all", "projected", "inside"), ivde.sweep_steps(ws)))}
            row = {"segments_per_view": S, "labels": L, "pixels_per_segment": 1920 * 1080 / S,
                   "class": ivde.shape_class(dv, lr, base), **res,
                   "autotune_us": {"x".join(map(str, k)): v for k, v in table.items()} if table else None}
            if "pairs" in res:
                _log(f"S={S} L={L}: one pixel {res['one']['sweep_ms']:.2f} ms, pixel pairs "
                     f"{res['pairs']['sweep_ms']:.2f} ms, four pixels {res['quads']['sweep_ms']:.2f} ms")
            _log(f"S={S} L={L}: {res['j1']['sweep_ms']:.2f} ms, {res['j1']['evals_per_s']:.3g} evals/s" +
                 ("" if args.no_tune else f" (tuned {res['tuned']['labels_per_lane']}x"
                                          f"{res['tuned']['waves_per_group']}: {res['tuned']['sweep_ms']:.2f} ms)"))
            rows.append(row)
        del dv
    return {"mode": "shapes", "workload": f"8-view 1920x1080 YUV420 {args.bit_depth}-bit arc rig, {args.sampling}, "
                                          "FP32 costs",
            "timing": f"median of {args.steps} event-timed sweeps per shape", "rows": rows}


# ---------------------------------------------------------------- precision
def bench_precision(args):
    """The precision workload: the 8-view arc rig at 4096x2160 (10-bit
    4:2:0), 40000 segments per view, 512 levels, bilinear; projection and
    accumulation in FP32, the cost volume stored in FP16 and, beside it, in
    FP32.  One step is the whole path (pack, index, work list, sweep,
    argmin).  The FP16 volume is compared with the FP32 one entry by entry
    (the error of both against the FP64 oracle is the GPU tests' part)."""
    import torch

    t0 = time.perf_counter()
    wl = synth.make_arc_workload("arc-8x4096x2160", synth.SEED_PRECISION, width=4096, height=2160,
                                 f=1400.0 * 4096 / 1920, n_segments=40000, num_labels=512)
    _log(f"generated {wl.name} in {time.perf_counter() - t0:.1f} s")
    dv = ivde.DeviceViews.from_workload(wl)
    lr = ivde.label_range(wl.z_near, wl.z_far, wl.num_labels)
    evals = _evals(wl)
    stream = torch.cuda.current_stream()
    out, vols, labs = {}, {}, {}
    for name, dt in (("f16", ivde.F16), ("f32", ivde.F32)):
        C, ws = ivde.cost_volume(dv, lr, ivde.options(ivde.BILINEAR, dt, pixels_per_step=args.pixels_per_step))
        lab = torch.empty(dv.rows, dtype=torch.int32, device="cuda")
        for _ in range(args.warmup):
            ivde.cost_volume(dv, lr, ivde.options(ivde.BILINEAR, dt, pixels_per_step=args.pixels_per_step),
                             workspace=ws, out=C, stream=stream)
        torch.cuda.synchronize()
        K = args.steps
        step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        sweep_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        opts = [ivde.options(ivde.BILINEAR, dt, sweep_events=e, pixels_per_step=args.pixels_per_step)
                for e in sweep_ev]
        t = time.perf_counter()
        for (a, b), o in zip(step_ev, opts):
            a.record(stream)
            ivde.cost_volume(dv, lr, o, workspace=ws, out=C, stream=stream)
            ivde.argmin(C, stream=stream, out=lab)
            b.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / K
        sweep_ms = float(np.median([a.elapsed_time(b) for a, b in sweep_ev]))
        lat = [a.elapsed_time(b) for a, b in step_ev]
        out[name] = {"evals_per_s": evals / wall, "ms_per_step": wall * 1e3,
                     "latency_ms": {"p50": _pct(lat, 50), "p99": _pct(lat, 99)},
                     "sweep_ms": sweep_ms, "sweep_evals_per_s": evals / (sweep_ms / 1e3),
                     "volume_bytes": int(C.numel() * C.element_size())}
        _log(f"{name}: {wall * 1e3:.1f} ms per step, sweep {sweep_ms:.1f} ms")
        vols[name], labs[name] = C, lab
        del ws
    d = (vols["f16"].float() - vols["f32"]).abs()
    storage = {"max_abs": float(d.max()), "mean_abs": float(d.double().mean()),
               "argmin_agreement": float((labs["f16"] == labs["f32"]).double().mean()),
               "bound": "FP16 rounding of values in [0, 1]: at most 2^-12 = 2.44e-4"}
    return {
        "metric": "pixel·label·view cost evals/s + %HBM roofline; p50/p99 frame latency",
        "value": out["f16"]["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": out["f16"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (FP16 storage)", "data": "synthetic",
        "config": {"workload": "8-view 4096x2160 YUV420 10-bit arc rig, 40000 segments per view, 512 levels, "
                               "bilinear, FP32 projection and accumulation, FP16 cost storage (FP32 beside it)",
                   "evals_per_step": evals, "segments": int(sum(wl.S)), "seed": wl.seed,
                   "step": "pack + segment index + work list + sweep + argmin"},
        "fp16_storage": out["f16"], "fp32_storage": out["f32"], "fp16_vs_fp32_storage": storage,
    }
