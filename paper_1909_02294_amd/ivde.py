"""Python binding of libivde (the C ABI in include/ivde.h).

Argument marshalling only: torch provides device memory and streams, every
computation runs in the library's gfx950 kernels.  There is no fallback:
if libivde.so is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# IVDE_LIB selects another build of the same library (the host-sanitizer build)
LIB_PATH = os.environ.get("IVDE_LIB") or os.path.join(HERE, "libivde.so")

IVDE_OK, IVDE_EINVAL, IVDE_ENOMEM, IVDE_EBUDGET, IVDE_EHIP, IVDE_EBUSY, IVDE_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
REF_RIG_CENTER, REF_OWN = -1, -2
NEAREST, BILINEAR = 0, 1
F32, F16 = 0, 1
TARGETS_ALL, TARGETS_NEAREST_LR, TARGETS_EXPLICIT = 0, 1, 2
SUBMIT_MASK, SUBMIT_RULE, SUBMIT_RULE_IFRAME = 0, 1, 2
NOALLOC_SCRATCH_BYTES = 64 << 20     # IVDE_NOALLOC_SCRATCH_BYTES


class IvdeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ivde status {status}: {msg}")
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double * 9), ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class Image(ctypes.Structure):
    _fields_ = [("plane", ctypes.c_void_p * 3), ("pitch", ctypes.c_int64 * 3),
                ("bit_depth", ctypes.c_int32), ("chroma_shift", ctypes.c_int32)]


class Segmentation(ctypes.Structure):
    _fields_ = [("seg_map", ctypes.c_void_p), ("pitch", ctypes.c_int64), ("num_segments", ctypes.c_int32)]


class LabelRange(ctypes.Structure):
    _fields_ = [("z_near", ctypes.c_double), ("z_far", ctypes.c_double),
                ("num_labels", ctypes.c_int32), ("depth_ref", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("sampling", ctypes.c_int32), ("cost_dtype", ctypes.c_int32), ("targets", ctypes.c_int32),
                ("target_mask", ctypes.c_void_p), ("labels_per_lane", ctypes.c_int32),
                ("waves_per_group", ctypes.c_int32), ("sweep_events", ctypes.c_void_p * 2),
                ("pixels_per_step", ctypes.c_int32)]


class Frame(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("cams", ctypes.POINTER(Camera)), ("views", ctypes.POINTER(Image)),
                ("segs", ctypes.POINTER(Segmentation)), ("labels", LabelRange), ("cost_out", ctypes.c_void_p),
                ("label_out", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("chunk_evals", ctypes.c_int64)]


class FrameStats(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("rig_id", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rows_recomputed", ctypes.c_int64), ("rows_from_iframe", ctypes.c_int64),
                ("rows_total", ctypes.c_int64),
                ("submit_us", ctypes.c_double), ("start_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class EnergyDesc(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("num_labels", ctypes.c_int32), ("unary", ctypes.c_void_p),
                ("unary_weight", ctypes.c_double), ("window_m", ctypes.c_void_p), ("window_hit", ctypes.c_void_p), ("K", ctypes.c_float),
                ("adj_offsets", ctypes.c_void_p), ("adj_index", ctypes.c_void_p), ("adj_beta", ctypes.c_void_p),
                ("fixed_labels", ctypes.c_void_p), ("quantum", ctypes.c_double)]


PARTITION_BLOCKS, PARTITION_INTERLEAVED = 0, 1


# every symbol include/ivde.h declares, with its ctypes signature
_P = ctypes.c_void_p
_I32, _I64, _SZ = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
SIGNATURES = {
    "ivde_cost_volume_size": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _P]),
    "ivde_sweep_shape": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _P, _P]),
    "ivde_workspace_sweep_steps": (_I32, [_P, _P, _P, _P, _P]),
    "ivde_cost_volume": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _SZ, _P, _P]),
    "ivde_cost_volume_noalloc": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _P]),
    "ivde_argmin": (_I32, [_I64, _I32, _I32, _P, _P, _P]),
    "ivde_workspace_status": (_I32, [_P, _P]),
    "ivde_batch_size": (_I32, [_I32, _P, _P, _P]),
    "ivde_batch_create": (_I32, [_I32, _P, _P, _P, _SZ, _P]),
    "ivde_batch_run": (_I32, [_P, _P, _I32]),
    "ivde_batch_destroy": (None, [_P]),
    "ivde_server_create": (_I32, [_P, _P]),
    "ivde_rig_register": (_I32, [_P, _I32, _P, _P, _P, _P, _P]),
    "ivde_stream_submit": (_I32, [_P, _I32, _P, _P, _P, _P, _P]),
    "ivde_stream_poll": (_I32, [_P, ctypes.c_uint64, _P]),
    "ivde_stream_wait": (_I32, [_P, ctypes.c_uint64, _P]),
    "ivde_rig_resident": (_I32, [_P, _I32, _P, _P]),
    "ivde_rig_reset": (_I32, [_P, _I32]),
    "ivde_server_destroy": (None, [_P]),
    "ivde_autotune": (_I32, [_I32, _P, _P, _P, _P, _P, _P, _SZ, _P, _P, _I32, _P, _P, _I32]),
    "ivde_stream_submit_rule": (_I32, [_P, _I32, _P, _I32, _P, _P, _P]),
    "ivde_server_footprint": (_I32, [_I32, _P, _P, _P, _P, _I32, _I32, _P, _P, _P]),
    "ivde_stream_submit_host": (_I32, [_P, _I32, _P, _I32, _P, _P, _P, _P]),
    "ivde_rig_set_temporal": (_I32, [_P, _I32, ctypes.c_float, ctypes.c_float]),
    "ivde_segment_stats_size": (_I32, [_I32, _P, _P, _I32, _P]),
    "ivde_segment_stats": (_I32, [_I32, _P, _P, _P, _P, _SZ, _P, _P, _P, _P]),
    "ivde_adjacency_size": (_I32, [_I32, _P, _P, _I32, _P]),
    "ivde_adjacency": (_I32, [_I32, _P, _P, _P, ctypes.c_float, ctypes.c_float, _P, _SZ, _P, _P, _P, _I64, _P]),
    "ivde_intra_cost": (_I32, [_I64, _I32, _P, _P, _P, _P, _P, _P, _P]),
    "ivde_depth_map": (_I32, [_I32, _P, _P, _P, _P, _P, _SZ, _P, _P]),
    "ivde_energy_value": (_I32, [_P, _P, _P]),
    "ivde_expansion": (_I32, [_P, _P, _P, _I32, _I32, _P, _P]),
    "ivde_optimize": (_I32, [_P, _I32, _I32, _I32, _P, _P]),
    "ivde_temporal_rule": (_I32, [_I64, _P, _P, _P, ctypes.c_float, ctypes.c_float, _I32, _P, _P]),
    "ivde_window_cost_size": (_I32, [_I32, _P, _P, _P, _I32, _P, _P]),
    "ivde_window_cost": (_I32, [_I32, _P, _P, _P, _P, _I32, _P, _SZ, _P, _P, _P]),
    "ivde_window_energy": (_I32, [_I64, _I32, _P, _P, _P, ctypes.c_float, _P, _P]),
    "ivde_status_string": (ctypes.c_char_p, [_I32]),
    "ivde_last_error": (ctypes.c_char_p, []),
    "ivde_version": (ctypes.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libivde.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run __graft_entry__.build() (or python -m "
                           f"paper_1909_02294_amd.build) first; there is no CPU fallback")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != IVDE_OK:
        lib = load()
        raise IvdeError(status, lib.ivde_last_error().decode() or lib.ivde_status_string(status).decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libivde needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _check(t, name, dtypes, shape=None, cuda=True):
    """Reject a tensor the C entry points would misread: wrong dtype, not
    contiguous, not on the GPU, or a shape other than `shape` (None entries
    match any extent).  The library reads raw pointers, so a mismatch here
    would otherwise read or write past the tensor."""
    if not isinstance(dtypes, (tuple, list)):
        dtypes = (dtypes,)
    if t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {' or '.join(str(d) for d in dtypes)}")
    if cuda and not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None:
        if t.dim() != len(shape) or any(e is not None and int(a) != int(e) for a, e in zip(t.shape, shape)):
            raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_cameras(cams):
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i].K[:] = [float(v) for v in np.asarray(c.K, np.float64).ravel()]
        arr[i].R[:] = [float(v) for v in np.asarray(c.R, np.float64).ravel()]
        arr[i].t[:] = [float(v) for v in np.asarray(c.t, np.float64).ravel()]
        arr[i].width, arr[i].height = int(c.width), int(c.height)
    return arr


class DeviceViews:
    """Device copies (torch tensors) of a rig's images and segment maps,
    and the C descriptors pointing at them."""

    def __init__(self, cams, Y, U, V, seg, S, bit_depth, chroma_shift, device="cuda"):
        torch = _torch()
        self.cams = list(cams)
        self.n = len(self.cams)
        self.bit_depth, self.chroma_shift = int(bit_depth), int(chroma_shift)
        dt = torch.uint8 if bit_depth <= 8 else torch.int16   # uint16 bits carried in int16
        npdt = np.uint8 if bit_depth <= 8 else np.uint16

        def up(a, dtype, ndt):
            a = np.ascontiguousarray(a, ndt)
            if ndt == np.uint16:
                a = a.view(np.int16)
            return torch.from_numpy(a).to(device)

        self.Y = [up(a, dt, npdt) for a in Y]
        self.U = [up(a, dt, npdt) for a in U]
        self.V = [up(a, dt, npdt) for a in V]
        self.seg = [up(a, torch.int32, np.int32) for a in seg]
        self.S = [int(s) for s in S]
        self.c_cams = make_cameras(self.cams)
        self.c_images = self._images()
        self.c_segs = (Segmentation * self.n)()
        for i in range(self.n):
            self.c_segs[i].seg_map = self.seg[i].data_ptr()
            self.c_segs[i].pitch = self.seg[i].shape[1]
            self.c_segs[i].num_segments = self.S[i]

    def _images(self):
        imgs = (Image * self.n)()
        for i in range(self.n):
            for p, t in enumerate((self.Y[i], self.U[i], self.V[i])):
                imgs[i].plane[p] = t.data_ptr()
                imgs[i].pitch[p] = t.shape[1]
            imgs[i].bit_depth, imgs[i].chroma_shift = self.bit_depth, self.chroma_shift
        return imgs

    def replace_images(self, Y, U, V):
        """Copy a new frame's planes into the existing device buffers."""
        torch = _torch()
        for dst, src in ((self.Y, Y), (self.U, U), (self.V, V)):
            for d, a in zip(dst, src):
                a = np.ascontiguousarray(a)
                if a.dtype == np.uint16:
                    a = a.view(np.int16)
                d.copy_(torch.from_numpy(a), non_blocking=False)

    @classmethod
    def from_workload(cls, wl, device="cuda"):
        return cls(wl.cams, wl.Y, wl.U, wl.V, wl.seg, wl.S, wl.bit_depth, wl.chroma_shift, device)

    @property
    def rows(self):
        return sum(self.S)


def label_range(z_near, z_far, num_labels, depth_ref=REF_RIG_CENTER):
    return LabelRange(float(z_near), float(z_far), int(num_labels), int(depth_ref))


def options(sampling=BILINEAR, cost_dtype=F32, targets=TARGETS_ALL, target_mask=None,
            labels_per_lane=0, waves_per_group=0, sweep_events=None, pixels_per_step=0):
    """sweep_events: optional pair of torch.cuda.Event(enable_timing=True),
    recorded by the library around its sweep kernel; pixels_per_step: 1 for
    the one-pixel sweep, 2 or 4 pixels per wave step, 0 the library's
    choice (4 where neighbouring levels land 3 px or more apart, 6 px with
    nearest sampling, else 2)."""
    o = Options(int(sampling), int(cost_dtype), int(targets), None, int(labels_per_lane), int(waves_per_group))
    o.pixels_per_step = int(pixels_per_step)
    if sweep_events is not None:
        torch = _torch()
        for ev in sweep_events:           # make torch create the underlying events
            ev.record(torch.cuda.current_stream())
        o.sweep_events[0] = sweep_events[0].cuda_event
        o.sweep_events[1] = sweep_events[1].cuda_event
        o._events = sweep_events
    if target_mask is not None:
        m = np.ascontiguousarray(target_mask, np.uint8)
        o._mask = m          # keep alive
        o.target_mask = m.ctypes.data
    return o


def sizes(dv: DeviceViews, lr: LabelRange, opt: Options):
    lib = load()
    cb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    check(lib.ivde_cost_volume_size(dv.n, dv.c_cams, dv.c_segs, ctypes.byref(lr), ctypes.byref(opt),
                                    dv.bit_depth, ctypes.byref(cb), ctypes.byref(wb)))
    return cb.value, wb.value


def sweep_shape(dv: DeviceViews, lr: LabelRange, opt: Options):
    """(labels_per_lane, waves_per_group, pixels_per_step) of the sweep
    ivde_cost_volume runs for these arguments."""
    lib = load()
    j, w, p = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib.ivde_sweep_shape(dv.n, dv.c_cams, dv.c_segs, ctypes.byref(lr), ctypes.byref(opt), dv.bit_depth,
                               ctypes.byref(j), ctypes.byref(w), ctypes.byref(p)))
    return j.value, w.value, p.value


def alloc_bytes(nbytes, device="cuda"):
    """A 256-byte aligned device byte buffer from torch's allocator."""
    torch = _torch()
    t = torch.empty(max(int(nbytes), 1) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + max(int(nbytes), 1)]


def cost_volume(dv: DeviceViews, lr: LabelRange, opt: Options, workspace=None, out=None, stream=None):
    """ivde_cost_volume: returns the [rows, L] cost tensor (float32 or float16)."""
    torch = _torch()
    lib = load()
    cb, wb = sizes(dv, lr, opt)
    if workspace is None or workspace.numel() < wb:
        workspace = alloc_bytes(wb)
    L = lr.num_labels
    dtype = torch.float16 if opt.cost_dtype == F16 else torch.float32
    if out is None:
        out = torch.empty((dv.rows, L), dtype=dtype, device="cuda")
    _check(out, "out", dtype, (dv.rows, L))
    check(lib.ivde_cost_volume(dv.n, dv.c_cams, dv.c_images, dv.c_segs, ctypes.byref(lr), ctypes.byref(opt),
                               ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                               ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out, workspace


def cost_volume_noalloc(dv: DeviceViews, lr: LabelRange, opt: Options, out=None, stream=None):
    """ivde_cost_volume_noalloc: the cost volume with the library's fixed
    device scratch array as workspace; the call itself allocates no device
    memory (pass `out` to allocate nothing here either)."""
    torch = _torch()
    L = lr.num_labels
    dtype = torch.float16 if opt.cost_dtype == F16 else torch.float32
    if out is None:
        out = torch.empty((dv.rows, L), dtype=dtype, device="cuda")
    _check(out, "out", dtype, (dv.rows, L))
    check(load().ivde_cost_volume_noalloc(dv.n, dv.c_cams, dv.c_images, dv.c_segs, ctypes.byref(lr),
                                          ctypes.byref(opt), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def argmin(cost, stream=None, out=None):
    torch = _torch()
    lib = load()
    _check(cost, "cost", (torch.float32, torch.float16), (None, None))
    rows, L = cost.shape
    if out is None:
        out = torch.empty(rows, dtype=torch.int32, device=cost.device)
    _check(out, "out", torch.int32, (rows,))
    dt = F16 if cost.dtype == torch.float16 else F32
    check(lib.ivde_argmin(rows, L, dt, ctypes.c_void_p(cost.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                          _stream_ptr(stream)))
    return out


def workspace_status(workspace, stream=None):
    lib = load()
    return lib.ivde_workspace_status(ctypes.c_void_p(workspace.data_ptr()), _stream_ptr(stream))


def sweep_steps(workspace, stream=None):
    """(all, on projected records, inside the validity band): the wave steps
    of the multi-pixel sweep of the last cost_volume call on `workspace`."""
    lib = load()
    a, p, i = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    check(lib.ivde_workspace_sweep_steps(ctypes.c_void_p(workspace.data_ptr()), _stream_ptr(stream), ctypes.byref(a),
                                         ctypes.byref(p), ctypes.byref(i)))
    return a.value, p.value, i.value


def last_error() -> str:
    return load().ivde_last_error().decode()


# ---------------------------------------------------------------- batched form
class Batch:
    """ivde_batch: one persistent sweep over many frames (optionally replayed
    from a hipGraph).  `frames` is a list of (DeviceViews, LabelRange,
    cost tensor, label tensor or None); the tensors must outlive the batch."""

    def __init__(self, frames, opt: Options):
        torch = _torch()
        lib = load()
        self._keep = [frames, opt]
        arr = (Frame * len(frames))()
        cdt = torch.float16 if opt.cost_dtype == F16 else torch.float32
        for i, (dv, lr, cost, lab) in enumerate(frames):
            _check(cost, f"frame {i} cost", cdt, (dv.rows, lr.num_labels))
            if lab is not None:
                _check(lab, f"frame {i} labels", torch.int32, (dv.rows,))
            arr[i].n_views = dv.n
            arr[i].cams = ctypes.cast(dv.c_cams, ctypes.POINTER(Camera))
            arr[i].views = ctypes.cast(dv.c_images, ctypes.POINTER(Image))
            arr[i].segs = ctypes.cast(dv.c_segs, ctypes.POINTER(Segmentation))
            arr[i].labels = lr
            arr[i].cost_out = cost.data_ptr()
            arr[i].label_out = lab.data_ptr() if lab is not None else None
        self._frames = arr
        wb = ctypes.c_size_t(0)
        check(lib.ivde_batch_size(len(frames), arr, ctypes.byref(opt), ctypes.byref(wb)))
        self.workspace = alloc_bytes(wb.value)
        h = ctypes.c_void_p()
        check(lib.ivde_batch_create(len(frames), arr, ctypes.byref(opt), ctypes.c_void_p(self.workspace.data_ptr()),
                                    self.workspace.numel(), ctypes.byref(h)))
        self.handle = h

    def run(self, stream=None, use_graph=True):
        check(load().ivde_batch_run(self.handle, _stream_ptr(stream), int(bool(use_graph))))

    def close(self):
        if self.handle:
            load().ivde_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- serving form
def server_footprint(dv: DeviceViews, lr: LabelRange, opt: Options, host=False):
    """(resident bytes, per-request bytes) a rig needs in a server arena;
    host=True: per-request bytes of a frame handed over in host memory."""
    r, q, qh = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    check(load().ivde_server_footprint(dv.n, dv.c_cams, dv.c_segs, ctypes.byref(lr), ctypes.byref(opt), dv.bit_depth,
                                       dv.chroma_shift, ctypes.byref(r), ctypes.byref(q), ctypes.byref(qh)))
    return r.value, (qh.value if host else q.value)


class HostFrame:
    """One frame's planes in pinned host memory (as a camera rig delivers
    them) and the C descriptors pointing at them, for Server.submit_host."""

    def __init__(self, n, Y, U, V, bit_depth, chroma_shift, mask=None):
        torch = _torch()
        self.n = int(n)
        self.bit_depth, self.chroma_shift = int(bit_depth), int(chroma_shift)

        def pin(a):
            a = np.ascontiguousarray(a)
            if a.dtype == np.uint16:
                a = a.view(np.int16)
            return torch.from_numpy(a).pin_memory()

        self.planes = [[pin(a) for a in (y, u, v)] for y, u, v in zip(Y, U, V)]
        self.mask = None if mask is None else pin(np.ascontiguousarray(mask, np.uint8))
        self.c_images = (Image * self.n)()
        for i in range(self.n):
            for p, t in enumerate(self.planes[i]):
                self.c_images[i].plane[p] = t.data_ptr()
                self.c_images[i].pitch[p] = t.shape[1]
            self.c_images[i].bit_depth, self.c_images[i].chroma_shift = self.bit_depth, self.chroma_shift


class Server:
    """ivde_server over a torch-allocated arena (its size is the budget)."""

    def __init__(self, arena_bytes, max_slots=4, chunk_evals=0):
        """chunk_evals: evaluations per launch of a full-frame sweep (0: the
        library's default, < 0: one launch)."""
        lib = load()
        self.arena = alloc_bytes(arena_bytes)
        cfg = ServerConfig(self.arena.data_ptr(), self.arena.numel(), int(max_slots), 0, int(chunk_evals))
        h = ctypes.c_void_p()
        check(lib.ivde_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self._rigs = {}
        self._inflight = {}

    def register(self, dv: DeviceViews, lr: LabelRange, opt: Options) -> int:
        rid = ctypes.c_int32(-1)
        check(load().ivde_rig_register(self.handle, dv.n, dv.c_cams, dv.c_segs, ctypes.byref(lr),
                                       ctypes.byref(opt), ctypes.byref(rid)))
        self._rigs[rid.value] = (dv.n, sum(dv.S), lr.num_labels, opt.cost_dtype)
        return rid.value

    def _check_outputs(self, rig, cost_out, label_out, mask=None):
        torch = _torch()
        if rig not in self._rigs:
            return          # the library reports the unknown rig
        _, R, L, dt = self._rigs[rig]
        if cost_out is not None:
            _check(cost_out, "cost_out", torch.float16 if dt == F16 else torch.float32, (R, L))
        if label_out is not None:
            _check(label_out, "label_out", torch.int32, (R,))
        if mask is not None:
            _check(mask, "mask", torch.uint8, (R,))

    def submit(self, rig: int, images, mask=None, cost_out=None, label_out=None) -> int:
        """images: a ctypes Image array (DeviceViews.c_images of the frame);
        mask: device uint8 tensor [rows] or None (recompute every row)."""
        self._check_outputs(rig, cost_out, label_out, mask)
        t = ctypes.c_uint64(0)
        check(load().ivde_stream_submit(self.handle, int(rig), images,
                                        ctypes.c_void_p(mask.data_ptr()) if mask is not None else None,
                                        ctypes.c_void_p(cost_out.data_ptr()) if cost_out is not None else None,
                                        ctypes.c_void_p(label_out.data_ptr()) if label_out is not None else None,
                                        ctypes.byref(t)))
        self._inflight[t.value] = (images, mask, cost_out, label_out)   # keep alive
        return t.value

    def submit_host(self, rig: int, frame: HostFrame, mode=SUBMIT_MASK, cost_out=None, label_out=None) -> int:
        """A frame in host memory (HostFrame); the server uploads it.  mode
        SUBMIT_MASK uses frame.mask (None: every row), SUBMIT_RULE and
        SUBMIT_RULE_IFRAME the temporal rule."""
        self._check_outputs(rig, cost_out, label_out)
        mask = frame.mask if mode == SUBMIT_MASK else None
        if mask is not None and rig in self._rigs and mask.numel() != self._rigs[rig][1]:
            raise ValueError(f"mask: expected {self._rigs[rig][1]} rows, got {mask.numel()}")
        t = ctypes.c_uint64(0)
        check(load().ivde_stream_submit_host(
            self.handle, int(rig), frame.c_images, int(mode),
            ctypes.c_void_p(mask.data_ptr()) if mask is not None else None,
            ctypes.c_void_p(cost_out.data_ptr()) if cost_out is not None else None,
            ctypes.c_void_p(label_out.data_ptr()) if label_out is not None else None, ctypes.byref(t)))
        self._inflight[t.value] = (frame, cost_out, label_out)   # keep the host buffers alive
        return t.value

    def submit_rule(self, rig: int, images, iframe=False, cost_out=None, label_out=None) -> int:
        """A frame whose changed rows the server derives by the temporal rule."""
        self._check_outputs(rig, cost_out, label_out)
        t = ctypes.c_uint64(0)
        check(load().ivde_stream_submit_rule(
            self.handle, int(rig), images, int(bool(iframe)),
            ctypes.c_void_p(cost_out.data_ptr()) if cost_out is not None else None,
            ctypes.c_void_p(label_out.data_ptr()) if label_out is not None else None, ctypes.byref(t)))
        self._inflight[t.value] = (images, cost_out, label_out)
        return t.value

    def set_temporal(self, rig: int, t_p=3.0, t_i=1.0):
        check(load().ivde_rig_set_temporal(self.handle, int(rig), float(t_p), float(t_i)))

    @staticmethod
    def _stats(st):
        return dict(ticket=st.ticket, rig=st.rig_id, status=st.status, rows_recomputed=st.rows_recomputed,
                    rows_from_iframe=st.rows_from_iframe, rows_total=st.rows_total, submit_us=st.submit_us,
                    start_us=st.start_us, done_us=st.done_us, latency_ms=(st.done_us - st.submit_us) / 1e3)

    def wait(self, ticket: int):
        st = FrameStats()
        rc = load().ivde_stream_wait(self.handle, ctypes.c_uint64(ticket), ctypes.byref(st))
        self._inflight.pop(ticket, None)
        check(rc)
        return self._stats(st)

    def poll(self, ticket: int):
        st = FrameStats()
        rc = load().ivde_stream_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(st))
        if rc == IVDE_EBUSY:
            return None
        self._inflight.pop(ticket, None)
        check(rc)
        return self._stats(st)

    def resident(self, rig: int):
        """The rig's resident cost volume as a torch tensor view (copy it)."""
        torch = _torch()
        p, rows = ctypes.c_void_p(), ctypes.c_int64()
        check(load().ivde_rig_resident(self.handle, int(rig), ctypes.byref(p), ctypes.byref(rows)))
        n, R, L, dt = self._rigs[rig]
        dtype = torch.float16 if dt == F16 else torch.float32
        esz = 2 if dt == F16 else 4
        base = self.arena.data_ptr()
        off = p.value - base
        flat = self.arena[off: off + R * L * esz]
        return flat.view(dtype).view(R, L)

    def reset(self, rig: int):
        check(load().ivde_rig_reset(self.handle, int(rig)))

    def close(self):
        if self.handle:
            load().ivde_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- tuning
# (labels per lane, waves per group, pixels per step), in the library's order
AUTOTUNE_SHAPES = [(1, 1, 1), (1, 2, 1), (1, 4, 1), (2, 1, 1), (2, 2, 1), (2, 4, 1), (4, 1, 1), (4, 2, 1), (4, 4, 1),
                   (8, 1, 1), (8, 2, 1), (8, 4, 1), (1, 1, 2), (1, 2, 2), (1, 4, 2), (1, 1, 4), (1, 2, 4), (1, 4, 4)]


def autotune(dv: DeviceViews, lr: LabelRange, opt: Options, reps=2, stream=None):
    """ivde_autotune: returns (best Options, {(J, wpg, px): microseconds or None})."""
    torch = _torch()
    lib = load()
    probe = Options(opt.sampling, opt.cost_dtype, opt.targets, opt.target_mask, 1, 1)
    cb, wb = sizes(dv, lr, probe)             # one label per lane needs the longest task list
    ws = alloc_bytes(wb)
    dtype = torch.float16 if opt.cost_dtype == F16 else torch.float32
    out = torch.empty((dv.rows, lr.num_labels), dtype=dtype, device="cuda")
    best = Options()
    times = (ctypes.c_float * len(AUTOTUNE_SHAPES))()
    check(lib.ivde_autotune(dv.n, dv.c_cams, dv.c_images, dv.c_segs, ctypes.byref(lr), ctypes.byref(opt),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(out.data_ptr()),
                            _stream_ptr(stream), int(reps), ctypes.byref(best), times, len(AUTOTUNE_SHAPES)))
    table = {s: (float(t) if t >= 0 else None) for s, t in zip(AUTOTUNE_SHAPES, times)}
    return best, table


def shape_class(dv: DeviceViews, lr: LabelRange, opt: Options) -> str:
    """The class of problems that share a tuned launch shape: what the
    sweep's speed depends on.  Sampling, storage type, texel encoding (FP16
    channels up to 11 bits, 16-bit code values above), levels rounded up to a 64-level
    block, pixels per segment to the nearest power of two (per-task overhead
    against per-pixel work), and targets per view."""
    npx = sum(c.width * c.height for c in dv.cams)
    px = npx / max(1, sum(dv.S))
    if opt.targets == TARGETS_NEAREST_LR:
        tg = 2 if dv.n > 2 else 1
    elif opt.targets == TARGETS_EXPLICIT:
        tg = "x"
    else:
        tg = dv.n - 1
    return (f"{'bil' if opt.sampling == BILINEAR else 'nn'}-{'f16' if opt.cost_dtype == F16 else 'f32'}"
            f"-tex{'f16' if dv.bit_depth <= 11 else 'u16'}-L{(lr.num_labels + 63) // 64 * 64}"
            f"-px{2 ** int(round(math.log2(max(px, 1.0))))}-t{tg}")


_TUNE_MEMO = {}


def autotune_cached(dv: DeviceViews, lr: LabelRange, opt: Options, cache_path=None, reps=2, stream=None):
    """The launch shape for this problem's shape class: from the cache (a
    JSON file at cache_path, or this process's memory if None) when the
    class has been tuned, else tuned now on this problem by ivde_autotune
    and stored.  Returns (Options, the timing table or None if cached)."""
    key = shape_class(dv, lr, opt)
    cache = _TUNE_MEMO
    if cache_path is not None:
        try:
            with open(cache_path) as fh:
                cache = json.load(fh)
        except FileNotFoundError:
            cache = {}
    hit = cache.get(key)
    if hit is not None:
        return options(opt.sampling, opt.cost_dtype, opt.targets, getattr(opt, "_mask", None),
                       labels_per_lane=hit["labels_per_lane"], waves_per_group=hit["waves_per_group"],
                       pixels_per_step=hit.get("pixels_per_step", 1)), None
    best, table = autotune(dv, lr, opt, reps=reps, stream=stream)
    cache[key] = {"labels_per_lane": best.labels_per_lane, "waves_per_group": best.waves_per_group,
                  "pixels_per_step": best.pixels_per_step,
                  "us": {"x".join(map(str, k)): v for k, v in table.items()}}
    if cache_path is not None:
        tmp = f"{cache_path}.tmp{os.getpid()}"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, table


# ---------------------------------------------------------------- the paper's window term
def window_cost(dv: DeviceViews, lr: LabelRange, radius=1, stream=None):
    """ivde_window_cost: (m [rows, 2, L] float32, hit [rows, 2, L] int32)."""
    torch = _torch()
    lib = load()
    ob, wb = ctypes.c_size_t(), ctypes.c_size_t()
    check(lib.ivde_window_cost_size(dv.n, dv.c_cams, dv.c_segs, ctypes.byref(lr), dv.bit_depth, ctypes.byref(ob),
                                    ctypes.byref(wb)))
    ws = alloc_bytes(wb.value)
    L = lr.num_labels
    m = torch.empty((dv.rows, 2, L), dtype=torch.float32, device="cuda")
    hit = torch.empty((dv.rows, 2, L), dtype=torch.int32, device="cuda")
    check(lib.ivde_window_cost(dv.n, dv.c_cams, dv.c_images, dv.c_segs, ctypes.byref(lr), int(radius),
                               ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(m.data_ptr()),
                               ctypes.c_void_p(hit.data_ptr()), _stream_ptr(stream)))
    return m, hit, ws


def window_energy(m, hit, labelling, K=30.0, stream=None):
    """ivde_window_energy: [rows, L] float32."""
    torch = _torch()
    _check(m, "m", torch.float32, (None, 2, None))
    rows, _, L = m.shape
    _check(hit, "hit", torch.int32, (rows, 2, L))
    _check(labelling, "labelling", torch.int32, (rows,))
    out = torch.empty((rows, L), dtype=torch.float32, device=m.device)
    check(load().ivde_window_energy(rows, L, ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(hit.data_ptr()),
                                    ctypes.c_void_p(labelling.data_ptr()), float(K), ctypes.c_void_p(out.data_ptr()),
                                    _stream_ptr(stream)))
    return out


# ---------------------------------------------------------------- segment statistics, temporal rule
def segment_stats(dv: DeviceViews, stream=None):
    """ivde_segment_stats: (count [rows] int32, centre [rows, 2] int32, mean [rows, 4] float32)."""
    torch = _torch()
    lib = load()
    wb = ctypes.c_size_t()
    check(lib.ivde_segment_stats_size(dv.n, dv.c_cams, dv.c_segs, dv.bit_depth, ctypes.byref(wb)))
    ws = alloc_bytes(wb.value)
    R = dv.rows
    cnt = torch.empty(R, dtype=torch.int32, device="cuda")
    cen = torch.empty((R, 2), dtype=torch.int32, device="cuda")
    mean = torch.empty((R, 4), dtype=torch.float32, device="cuda")
    check(lib.ivde_segment_stats(dv.n, dv.c_cams, dv.c_images, dv.c_segs, ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), ctypes.c_void_p(cnt.data_ptr()), ctypes.c_void_p(cen.data_ptr()),
                                 ctypes.c_void_p(mean.data_ptr()), _stream_ptr(stream)))
    return cnt, cen, mean, ws


def temporal_rule(mean, mean_prev, mean_iframe=None, t_p=3.0, t_i=1.0, bit_depth=8, stream=None):
    """ivde_temporal_rule: uint8 [rows] with 0 recompute, 1 previous frame, 2 I frame."""
    torch = _torch()
    _check(mean, "mean", torch.float32, (None, 4))
    rows = mean.shape[0]
    _check(mean_prev, "mean_prev", torch.float32, (rows, 4))
    if mean_iframe is not None:
        _check(mean_iframe, "mean_iframe", torch.float32, (rows, 4))
    out = torch.empty(rows, dtype=torch.uint8, device=mean.device)
    check(load().ivde_temporal_rule(rows, ctypes.c_void_p(mean.data_ptr()), ctypes.c_void_p(mean_prev.data_ptr()),
                                    ctypes.c_void_p(mean_iframe.data_ptr()) if mean_iframe is not None else None,
                                    float(t_p), float(t_i), int(bit_depth), ctypes.c_void_p(out.data_ptr()),
                                    _stream_ptr(stream)))
    return out


def adjacency(dv: DeviceViews, beta0: float, eps: float = 1.0, capacity=None, stream=None):
    """ivde_adjacency: (offsets [rows + 1] int64, index [edges] int32,
    beta [edges] float32).  With capacity None the entry count is learned
    first (a call with capacity 0), then the lists are filled."""
    torch = _torch()
    lib = load()
    wb = ctypes.c_size_t()
    check(lib.ivde_adjacency_size(dv.n, dv.c_cams, dv.c_segs, dv.bit_depth, ctypes.byref(wb)))
    ws = alloc_bytes(wb.value)
    offsets = torch.empty(dv.rows + 1, dtype=torch.int64, device="cuda")

    def run(cap, index, beta):
        check(lib.ivde_adjacency(dv.n, dv.c_cams, dv.c_images, dv.c_segs, float(beta0), float(eps),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(offsets.data_ptr()),
                                 ctypes.c_void_p(index.data_ptr()) if index is not None else None,
                                 ctypes.c_void_p(beta.data_ptr()) if beta is not None else None, int(cap),
                                 _stream_ptr(stream)))

    if capacity is None:
        run(0, None, None)
        (stream if stream is not None else torch.cuda.current_stream()).synchronize()
        capacity = int(offsets[-1].item())
    index = torch.empty(max(int(capacity), 1), dtype=torch.int32, device="cuda")
    beta = torch.empty(max(int(capacity), 1), dtype=torch.float32, device="cuda")
    run(capacity, index, beta)
    return offsets, index[:capacity], beta[:capacity], ws


def intra_cost(offsets, index, beta, labelling, num_labels: int, fixed=None, stream=None):
    """ivde_intra_cost: float32 [rows, num_labels]."""
    torch = _torch()
    _check(offsets, "offsets", torch.int64, (None,))
    rows = offsets.shape[0] - 1
    _check(index, "index", torch.int32, (None,))
    _check(beta, "beta", torch.float32, (index.shape[0],))
    _check(labelling, "labelling", torch.int32, (rows,))
    if fixed is not None:
        _check(fixed, "fixed", torch.uint8, (rows,))
    out = torch.empty((rows, int(num_labels)), dtype=torch.float32, device=offsets.device)
    check(load().ivde_intra_cost(rows, int(num_labels), ctypes.c_void_p(offsets.data_ptr()),
                                 ctypes.c_void_p(index.data_ptr()), ctypes.c_void_p(beta.data_ptr()),
                                 ctypes.c_void_p(labelling.data_ptr()),
                                 ctypes.c_void_p(fixed.data_ptr()) if fixed is not None else None,
                                 ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


class Energy:
    """Host-side Eq. (1) (ivde_energy): numpy arrays or CPU tensors, kept
    alive by this object while the library reads them."""

    def __init__(self, rows, num_labels, unary=None, m=None, hit=None, K=30.0, offsets=None, index=None,
                 beta=None, fixed=None, quantum=1024.0, unary_weight=1.0):
        def host(a, dt):
            if a is None:
                return None
            if hasattr(a, "detach"):
                a = a.detach().cpu().numpy()
            return np.ascontiguousarray(a, dt)

        self._keep = [host(unary, np.float32), host(m, np.float32), host(hit, np.int32), host(offsets, np.int64),
                      host(index, np.int32), host(beta, np.float32), host(fixed, np.int32)]
        u, mm, h, o, i, b, f = self._keep
        ptr = lambda a: a.ctypes.data if a is not None else None  # noqa: E731
        self.desc = EnergyDesc(int(rows), int(num_labels), ptr(u), float(unary_weight), ptr(mm), ptr(h), float(K),
                               ptr(o), ptr(i), ptr(b), ptr(f), float(quantum))
        self.rows, self.num_labels = int(rows), int(num_labels)

    def value(self, labels) -> int:
        d = np.ascontiguousarray(labels, np.int32)
        e = ctypes.c_int64()
        check(load().ivde_energy_value(ctypes.byref(self.desc), d.ctypes.data, ctypes.byref(e)))
        return e.value

    def expansion(self, labels, label_list, max_cycles=8):
        """(labels, energy, cycles) after alpha-expansion from `labels`."""
        d = np.array(labels, np.int32)
        ls = np.ascontiguousarray(label_list, np.int32)
        e, c = ctypes.c_int64(), ctypes.c_int32()
        check(load().ivde_expansion(ctypes.byref(self.desc), d.ctypes.data, ls.ctypes.data, len(ls), int(max_cycles),
                                    ctypes.byref(e), ctypes.byref(c)))
        return d, e.value, c.value

    def optimize(self, n_threads=1, partition=PARTITION_BLOCKS, max_cycles=8):
        """(labels, energy) of the label-partitioned estimation."""
        d = np.empty(self.rows, np.int32)
        e = ctypes.c_int64()
        check(load().ivde_optimize(ctypes.byref(self.desc), int(n_threads), int(partition), int(max_cycles),
                                   d.ctypes.data, ctypes.byref(e)))
        return d, e.value


def depth_map(dv: DeviceViews, lr: LabelRange, labels, stream=None):
    """ivde_depth_map: float32 [sum of W * H] depth maps, view after view."""
    torch = _torch()
    n_px = sum(int(c.width) * int(c.height) for c in dv.c_cams)
    out = torch.empty(n_px, dtype=torch.float32, device="cuda")
    lab = labels if hasattr(labels, "data_ptr") else torch.from_numpy(np.ascontiguousarray(labels, np.int32)).cuda()
    _check(lab, "labels", torch.int32, (dv.rows,))
    table = torch.empty(int(lr.num_labels), dtype=torch.float32, device="cuda")
    check(load().ivde_depth_map(dv.n, dv.c_cams, dv.c_segs, ctypes.byref(lr), ctypes.c_void_p(lab.data_ptr()),
                                ctypes.c_void_p(table.data_ptr()), table.numel() * 4, ctypes.c_void_p(out.data_ptr()),
                                _stream_ptr(stream)))
    out._ivde_keep = table          # the table is read until the stream completes
    return out
